// search_lds.hip - LDS tier of the exact-cover search (components of more
// than 64 nodes), one 64-lane wavefront per component.
//
// Same matrix and rules as the register tier (Sec. 2.3, Algorithm 1), with
// state that scales past one lane per node:
//   rm[v]    open colors of node v (one byte; 0 once v's column is covered);
//   B[t]     bitset of uncovered nodes whose column has exactly t rows,
//            t = 0..k (W = ceil(n/64) words each);
//   S[t]     summary of B[t]: bit w set whenever word w of B[t] may be
//            nonzero (set on every insert, cleared lazily at selection).
// Column choice: for t = 0..k, the lowest set summary bit leads to the
// lowest nonzero word of B[t] and its lowest bit is the lowest index with t
// rows - the min-count, lowest-index column, without scanning all columns.
// Cover of row (v, c) walks v's neighbour list, one neighbour per lane:
// lanes whose neighbour still has color c open clear it and move the
// neighbour from B[t] to B[t-1] (LDS atomics, several lanes may share a
// word); the ballot of those lanes is the undo record (Eq. 2 uncover ORs
// them back, moving each neighbour up one bucket).
//
// Placement: rm, B, S always in LDS.  Small components also keep their
// neighbour lists and search stack in LDS; "big" components keep them in
// global memory (stack in a per-worker scratch area).
#include <hip/hip_runtime.h>

#include "device_types.h"
#include "mpld.h"

namespace mpld {

static constexpr uint64_t kFnvOffsetL = 0xcbf29ce484222325ull;
static constexpr uint64_t kFnvPrimeL = 0x100000001b3ull;
static constexpr uint32_t kNoneL = 0xffffffffu;
static constexpr int32_t kStatusBroken = 3;   // reported to the host as an internal error

__device__ __forceinline__ uint64_t fnv_u32_l(uint64_t h, uint32_t v) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    h ^= (v >> (8 * b)) & 0xffu;
    h *= kFnvPrimeL;
  }
  return h;
}

__device__ __forceinline__ uint64_t trace_node_l(uint64_t h, uint32_t depth, uint32_t row_in,
                                                 uint32_t col, uint32_t size) {
  h = fnv_u32_l(h, depth);
  h = fnv_u32_l(h, row_in);
  h = fnv_u32_l(h, col);
  return fnv_u32_l(h, size);
}

__device__ __forceinline__ uint32_t uni(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t x, uint32_t lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)lane);
  return ((uint64_t)hi << 32) | lo;
}

// Byte layout of the LDS area of one component.
struct LdsLayout {
  uint32_t W, SW, frame_words, rm_off, b_off, s_off, adj_off, stk_off, total;
};

__host__ __device__ inline LdsLayout lds_layout(int32_t n, int32_t k, int64_t adj_words,
                                                int32_t max_deg, bool big) {
  LdsLayout L;
  L.W = (uint32_t)((n + 63) / 64);
  L.SW = (L.W + 63) / 64;
  L.frame_words = 1u + (uint32_t)((max_deg + 63) / 64);   // u64: header + removed masks
  uint32_t off = 0;
  L.rm_off = off;
  off += ((uint32_t)n + 7u) & ~7u;
  L.b_off = off;
  off += 8u * (uint32_t)(k + 1) * L.W;
  L.s_off = off;
  off += 8u * (uint32_t)(k + 1) * L.SW;
  L.adj_off = off;
  if (!big) off += 4u * (uint32_t)adj_words;
  off = (off + 7u) & ~7u;
  L.stk_off = off;
  if (!big) off += 8u * L.frame_words * (uint32_t)n;
  L.total = off;
  return L;
}

template <bool TRACE, bool BIG>
__device__ void solve_lds(const DevDesc& d, const uint32_t* __restrict__ gadj, char* lds,
                          uint64_t* gstack, int8_t* __restrict__ colors,
                          DevRecord* __restrict__ rec) {
  const uint32_t lane = __lane_id();
  const int32_t n = d.n, k = d.k;
  // adjacency block: [0..n] row offsets, [n+1 ..] neighbour ids; the host
  // stores the largest degree right after the ids.
  const uint32_t adj_words = uni(gadj[n]) + (uint32_t)n + 1u;
  const uint32_t mdeg = uni(gadj[adj_words]);
  const LdsLayout L = lds_layout(n, k, adj_words, (int32_t)mdeg, BIG);
  uint8_t* rm = reinterpret_cast<uint8_t*>(lds + L.rm_off);
  uint64_t* B = reinterpret_cast<uint64_t*>(lds + L.b_off);
  uint64_t* S = reinterpret_cast<uint64_t*>(lds + L.s_off);
  const uint32_t* adj;
  uint64_t* stk;
  if (BIG) {
    adj = gadj;
    stk = gstack;
  } else {
    uint32_t* la = reinterpret_cast<uint32_t*>(lds + L.adj_off);
    for (uint32_t i = lane; i < adj_words; i += 64) la[i] = gadj[i];
    adj = la;
    stk = reinterpret_cast<uint64_t*>(lds + L.stk_off);
  }
  const uint32_t* ids = adj + n + 1;
  const uint32_t W = L.W, SW = L.SW, FW = L.frame_words;
  // initial state: every node uncovered with all k colors open
  const uint8_t full = (uint8_t)((1u << k) - 1u);
  for (uint32_t v = lane; v < (uint32_t)n; v += 64) rm[v] = full;
  for (uint32_t i = lane; i < (uint32_t)(k + 1) * W; i += 64) {
    const uint32_t t = i / W, w = i % W;
    uint64_t val = 0;
    if (t == (uint32_t)k) {
      const uint32_t lo = w * 64u;
      const uint32_t cnt = (uint32_t)n - lo >= 64u ? 64u : (uint32_t)n - lo;
      val = cnt == 64u ? ~0ull : ((1ull << cnt) - 1ull);
    }
    B[i] = val;
  }
  for (uint32_t i = lane; i < (uint32_t)(k + 1) * SW; i += 64) {
    const uint32_t t = i / SW, j = i % SW;
    uint64_t val = 0;
    if (t == (uint32_t)k) {
      const uint32_t lo = j * 64u;
      const uint32_t cnt = W - lo >= 64u ? 64u : W - lo;
      val = cnt == 64u ? ~0ull : ((1ull << cnt) - 1ull);
    }
    S[i] = val;
  }
  __syncthreads();

  uint32_t depth = 0, open = (uint32_t)n, row_in = kNoneL;
  uint64_t nodes = 0, h = kFnvOffsetL;
  int32_t status;
  const uint64_t budget = (uint64_t)d.budget;

  auto move_up = [&](uint32_t w, uint32_t t) {  // node w: bucket t -> t+1
    const uint32_t word = w >> 6;
    const uint64_t bit = 1ull << (w & 63u);
    atomicAnd(reinterpret_cast<unsigned long long*>(&B[t * W + word]), ~bit);
    atomicOr(reinterpret_cast<unsigned long long*>(&B[(t + 1) * W + word]), bit);
    atomicOr(reinterpret_cast<unsigned long long*>(&S[(t + 1) * SW + (word >> 6)]),
             1ull << (word & 63u));
  };
  auto move_down = [&](uint32_t w, uint32_t t) {  // node w: bucket t -> t-1
    const uint32_t word = w >> 6;
    const uint64_t bit = 1ull << (w & 63u);
    atomicAnd(reinterpret_cast<unsigned long long*>(&B[t * W + word]), ~bit);
    atomicOr(reinterpret_cast<unsigned long long*>(&B[(t - 1) * W + word]), bit);
    atomicOr(reinterpret_cast<unsigned long long*>(&S[(t - 1) * SW + (word >> 6)]),
             1ull << (word & 63u));
  };

  for (;;) {
    // ---- one search node
    if (nodes == budget) { status = MPLD_BUDGET_EXHAUSTED; break; }
    ++nodes;
    if (open == 0) {
      if (TRACE) h = trace_node_l(h, depth, row_in, kNoneL, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    // column choice: smallest t with a nonzero bucket, lowest index in it
    uint32_t v = 0, size = 0;
    bool any = false;
    for (uint32_t t = 0; t <= (uint32_t)k; ++t) {
      uint64_t s = lane < SW ? S[t * SW + lane] : 0ull;
      bool found = false;
      for (;;) {
        const uint64_t bal = __ballot(s != 0ull);
        if (bal == 0ull) break;
        const uint32_t j = (uint32_t)__ffsll((unsigned long long)bal) - 1u;
        const uint64_t sj = rdlane64(s, j);
        const uint32_t b = (uint32_t)__ffsll((unsigned long long)sj) - 1u;
        const uint32_t w = j * 64u + b;
        const uint64_t word = uni64(B[t * W + w]);
        if (word) {
          v = w * 64u + (uint32_t)__ffsll((unsigned long long)word) - 1u;
          size = t;
          found = true;
          break;
        }
        // stale summary bit: drop it and look again (lane j owns word j)
        if (lane == j) {
          s &= ~(1ull << b);
          S[t * SW + j] = s;
        }
      }
      if (found) { any = true; break; }
    }
    if (!any) { status = kStatusBroken; break; }   // open > 0 but no bucket: a bug
    if (TRACE) h = trace_node_l(h, depth, row_in, v, size);
    uint32_t c, rows;
    if (size != 0) {
      // cover column v
      rows = uni(rm[v]);
      if (lane == (v & 63u)) {   // one owner lane; see the note at the record store
        rm[v] = 0;
        atomicAnd(reinterpret_cast<unsigned long long*>(&B[size * W + (v >> 6)]),
                  ~(1ull << (v & 63u)));
      }
      --open;
      c = (uint32_t)__ffs(rows) - 1u;
    } else {
      // dead end: undo rows and columns until one has a next row
      for (;;) {
        if (depth == 0) { status = MPLD_INFEASIBLE; goto done; }
        --depth;
        const uint64_t hdr = uni64(stk[(uint64_t)depth * FW]);
        v = (uint32_t)hdr;
        const uint32_t cp = (uint32_t)(hdr >> 32) & 0xffu;
        rows = (uint32_t)(hdr >> 40) & 0xffu;
        const uint32_t beg = uni(adj[v]), deg = uni(adj[v + 1]) - beg;
        for (uint32_t ch = 0; ch * 64u < deg; ++ch) {
          const uint64_t rem = uni64(stk[(uint64_t)depth * FW + 1 + ch]);
          if ((rem >> lane) & 1ull) {
            const uint32_t w = ids[beg + ch * 64u + lane];
            const uint32_t r = rm[w];
            rm[w] = (uint8_t)(r | (1u << cp));
            move_up(w, (uint32_t)__popc(r));
          }
        }
        __syncthreads();   // lanes' LDS updates visible to every lane
        const uint32_t next = rows & ~((2u << cp) - 1u);
        if (next) { c = (uint32_t)__ffs(next) - 1u; break; }
        // uncover column v
        if (lane == (v & 63u)) {
          rm[v] = (uint8_t)rows;
          const uint32_t t = (uint32_t)__popc(rows);
          atomicOr(reinterpret_cast<unsigned long long*>(&B[t * W + (v >> 6)]), 1ull << (v & 63u));
          atomicOr(reinterpret_cast<unsigned long long*>(&S[t * SW + (v >> 12)]),
                   1ull << ((v >> 6) & 63u));
        }
        __syncthreads();
        ++open;
      }
    }
    // ---- include row (v, c): close color c at v's open neighbours
    {
      const uint32_t beg = uni(adj[v]), deg = uni(adj[v + 1]) - beg;
      if (lane == (depth & 63u))
        stk[(uint64_t)depth * FW] = (uint64_t)v | ((uint64_t)c << 32) | ((uint64_t)rows << 40);
      for (uint32_t ch = 0; ch * 64u < deg; ++ch) {
        bool hit = false;
        const uint32_t j = ch * 64u + lane;
        if (j < deg) {
          const uint32_t w = ids[beg + j];
          const uint32_t r = rm[w];
          if ((r >> c) & 1u) {
            hit = true;
            rm[w] = (uint8_t)(r & ~(1u << c));
            move_down(w, (uint32_t)__popc(r));
          }
        }
        const uint64_t rem = __ballot(hit);
        if (lane == ((depth + 1u + ch) & 63u)) stk[(uint64_t)depth * FW + 1 + ch] = rem;
      }
      __syncthreads();
      ++depth;
      row_in = v * (uint32_t)k + c;
    }
  }
done:
  __syncthreads();
  if (status == MPLD_FEASIBLE) {
    for (uint32_t f = lane; f < depth; f += 64) {
      const uint64_t hdr = stk[(uint64_t)f * FW];
      colors[(uint32_t)hdr] = (int8_t)((hdr >> 32) & 0xffu);
    }
  } else {
    for (uint32_t v = lane; v < (uint32_t)n; v += 64) colors[v] = -1;
  }
  // Every lane stores the same (uniform) record: no branch in the loop may
  // share the queue pop's "lane 0" condition, or the compiler can thread the
  // two across the loop back-edge and split the wave at the pop.
  rec->status = status;
  rec->depth = status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
  rec->nodes = nodes;
  rec->hash = h;
  __syncthreads();
}

// Persistent kernel, one wave per workgroup; work distribution as in the
// register tier: static first item, then atomic pops, the last pop resets
// the counter.
template <bool TRACE, bool BIG>
__global__ __launch_bounds__(64) void lds_batched_kernel(
    const DevDesc* __restrict__ descs, const uint32_t* __restrict__ adj32, int32_t qlen,
    int32_t* __restrict__ counter, uint64_t* gstack, uint64_t stack_words_per_wave,
    DevRecord* __restrict__ recs, int8_t* __restrict__ colors) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* my_stack = BIG ? gstack + (uint64_t)blockIdx.x * stack_words_per_wave : nullptr;
  const int32_t gw = (int32_t)gridDim.x;
  int32_t item = (int32_t)uni(blockIdx.x);
  while (item < qlen) {
    const DevDesc d = descs[item];
    solve_lds<TRACE, BIG>(d, adj32 + d.nbr_off, lds, my_stack, colors + d.out_off, recs + d.comp);
    if (gw >= qlen) break;
    int32_t r = 0;
    if (__lane_id() == 0) r = atomicAdd(counter, 1);
    r = (int32_t)uni((uint32_t)r);
    item = gw + r;
    if (r == qlen - 1) atomicExch(counter, 0);
  }
}

template <bool TRACE, bool BIG>
__global__ __launch_bounds__(64) void lds_single_kernel(const DevDesc* __restrict__ descs,
                                                        const uint32_t* __restrict__ adj32,
                                                        int32_t item, uint64_t* gstack,
                                                        DevRecord* __restrict__ recs,
                                                        int8_t* __restrict__ colors) {
  extern __shared__ __align__(16) char lds[];
  const DevDesc d = descs[item];
  solve_lds<TRACE, BIG>(d, adj32 + d.nbr_off, lds, gstack, colors + d.out_off, recs + d.comp);
}

// ---- host side --------------------------------------------------------------

int64_t lds_bytes_for(int32_t n, int32_t k, int64_t adj_words, int32_t max_deg, bool big) {
  // adj_words: row offsets + neighbour ids (n + 1 + 2m)
  return (int64_t)lds_layout(n, k, adj_words, max_deg, big).total;
}

int64_t lds_stack_words(int32_t n, int32_t max_deg) {
  return (int64_t)n * (1 + (max_deg + 63) / 64);
}

template <bool TRACE, bool BIG>
static void lds_attr(int bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_batched_kernel<TRACE, BIG>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_single_kernel<TRACE, BIG>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

void lds_configure(int bytes) {
  lds_attr<true, true>(bytes);
  lds_attr<true, false>(bytes);
  lds_attr<false, true>(bytes);
  lds_attr<false, false>(bytes);
  (void)hipGetLastError();
}

template <bool TRACE, bool BIG>
static hipError_t lds_batched_t(int grid, int lds_bytes, const DevDesc* descs,
                                const uint32_t* adj32, int32_t qlen, int32_t* counter,
                                uint64_t* gstack, uint64_t stack_words, DevRecord* recs,
                                int8_t* colors, hipStream_t s) {
  hipLaunchKernelGGL((lds_batched_kernel<TRACE, BIG>), dim3(grid), dim3(64), (size_t)lds_bytes, s,
                     descs, adj32, qlen, counter, gstack, stack_words, recs, colors);
  return hipGetLastError();
}

hipError_t launch_lds_batched(bool trace, bool big, int grid, int lds_bytes, const DevDesc* descs,
                              const uint32_t* adj32, int32_t qlen, int32_t* counter,
                              uint64_t* gstack, uint64_t stack_words, DevRecord* recs,
                              int8_t* colors, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  if (trace)
    return big ? lds_batched_t<true, true>(grid, lds_bytes, descs, adj32, qlen, counter, gstack,
                                           stack_words, recs, colors, s)
               : lds_batched_t<true, false>(grid, lds_bytes, descs, adj32, qlen, counter, gstack,
                                            stack_words, recs, colors, s);
  return big ? lds_batched_t<false, true>(grid, lds_bytes, descs, adj32, qlen, counter, gstack,
                                          stack_words, recs, colors, s)
             : lds_batched_t<false, false>(grid, lds_bytes, descs, adj32, qlen, counter, gstack,
                                           stack_words, recs, colors, s);
}

template <bool TRACE, bool BIG>
static hipError_t lds_single_t(int lds_bytes, const DevDesc* descs, const uint32_t* adj32,
                               int32_t item, uint64_t* gstack, DevRecord* recs, int8_t* colors,
                               hipStream_t s) {
  hipLaunchKernelGGL((lds_single_kernel<TRACE, BIG>), dim3(1), dim3(64), (size_t)lds_bytes, s,
                     descs, adj32, item, gstack, recs, colors);
  return hipGetLastError();
}

hipError_t launch_lds_single(bool trace, bool big, int lds_bytes, const DevDesc* descs,
                             const uint32_t* adj32, int32_t item, uint64_t* gstack,
                             DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (trace)
    return big ? lds_single_t<true, true>(lds_bytes, descs, adj32, item, gstack, recs, colors, s)
               : lds_single_t<true, false>(lds_bytes, descs, adj32, item, gstack, recs, colors, s);
  return big ? lds_single_t<false, true>(lds_bytes, descs, adj32, item, gstack, recs, colors, s)
             : lds_single_t<false, false>(lds_bytes, descs, adj32, item, gstack, recs, colors, s);
}

}  // namespace mpld
