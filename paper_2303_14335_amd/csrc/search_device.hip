// search_device.hip - device-wide tier of the exact-cover search: one giant
// component spread over every CU in a cooperative launch.
//
// Same matrix and rules as the other tiers (Sec. 2.3, Algorithm 1).  Block b
// owns a contiguous slice of the columns (nodes) and keeps, in LDS, each of
// its nodes' open colors (bits 0..k-1) and a covered flag (bit 15).  Per
// search node:
//   1. every block finds, over its slice, the uncovered column with the
//      fewest rows (key = count << 32 | index) and folds it into one global
//      64-bit key with atomicMin: the device-wide column-count reduction;
//   2. one grid barrier; every block reads the winning key.
//   3. every block replays the same decision on its own slice: cover the
//      column, take / undo rows (Eq. 2) for the neighbours it owns, keeping
//      its own undo stack (frame header + removed bits of its neighbours).
// Decisions depend only on the global key and on state every block tracks
// identically (depth, counters), so the reduction is the only cross-block
// exchange.  Three key slots rotate so that a slot is reset two nodes before
// its next use, with a barrier in between.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "device_types.h"
#include "mpld.h"
#include "trace.h"

namespace cg = cooperative_groups;

namespace mpld {

static constexpr uint32_t kNoneD = 0xffffffffu;
static constexpr uint16_t kCovered = 0x8000u;
static constexpr int kDevThreads = 256;

__device__ __forceinline__ uint64_t min64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Minimum over the block (every thread gets it).
__device__ __forceinline__ uint64_t block_min(uint64_t x, uint64_t* red) {
  for (int off = 32; off > 0; off >>= 1) x = min64(x, (uint64_t)__shfl_xor((unsigned long long)x, off));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = x;
  __syncthreads();
  uint64_t m = red[0];
  for (int w = 1; w < kDevThreads / 64; ++w) m = min64(m, red[w]);
  __syncthreads();
  return m;
}

// adj: the component's block in adj32 ([0..n] offsets, ids, max degree).
// keys: 3 u64 slots, ~0 at launch (and again at exit).  A key is
// count << 40 | index << 8 | open colors, so its minimum is the column of
// fewest rows, lowest index on ties, and carries that column's rows to
// every block.  stacks: per block, n * FW u64 words (FW = 1 + ceil(maxdeg /
// 64)): word 0 of frame d is v | c << 32 | rows << 40, then the bits of the
// block's neighbour positions that lost color c.
template <bool TRACE>
__global__ __launch_bounds__(kDevThreads) void device_tier_kernel(
    const DevDesc* __restrict__ descp, const uint32_t* __restrict__ adj32,
    unsigned long long* keys, uint64_t* stacks, DevRecord* __restrict__ recs,
    int8_t* __restrict__ colors_base) {
  extern __shared__ __align__(16) char lds[];
  cg::grid_group grid = cg::this_grid();
  const DevDesc d = *descp;
  const int32_t n = d.n, k = d.k;
  const uint32_t* adj = adj32 + d.nbr_off;
  const uint32_t* ids = adj + n + 1;
  const uint32_t adj_words = adj[n] + (uint32_t)n + 1u;
  const uint32_t maxdeg = adj[adj_words];
  const uint32_t FW = 1u + (maxdeg + 63u) / 64u;
  const uint32_t G = gridDim.x, b = blockIdx.x, tid = threadIdx.x;
  const uint32_t per = ((uint32_t)n + G - 1) / G;
  const uint32_t lo = min((uint32_t)n, b * per), hi = min((uint32_t)n, lo + per);
  uint16_t* rm = reinterpret_cast<uint16_t*>(lds);                 // slice [lo, hi)
  uint64_t* red = reinterpret_cast<uint64_t*>(lds + ((per * 2 + 15) & ~15u));
  uint64_t* stk = stacks + (uint64_t)b * (uint64_t)n * FW;
  const uint16_t full = (uint16_t)((1u << k) - 1u);
  for (uint32_t v = lo + tid; v < hi; v += kDevThreads) rm[v - lo] = full;
  __syncthreads();

  uint64_t nodes = 0, h = 0;
  uint32_t depth = 0, open = (uint32_t)n, row_in = kNoneD;
  int32_t status = -1;
  const uint64_t budget = (uint64_t)d.budget;
  uint32_t slot = 0;

  // row (v, c) on this block's neighbours of v: close color c where open and
  // record which neighbour positions lost it (frame `dep`)
  auto take_row = [&](uint32_t v, uint32_t c, uint32_t dep) {
    const uint32_t beg = adj[v], deg = adj[v + 1] - beg;
    for (uint32_t ch = 0; ch * 64u < deg; ++ch) {
      bool hit = false;
      if (tid < 64) {
        const uint32_t j = ch * 64u + tid;
        if (j < deg) {
          const uint32_t w = ids[beg + j];
          if (w >= lo && w < hi) {
            const uint16_t r = rm[w - lo];
            if (!(r & kCovered) && ((r >> c) & 1u)) {
              rm[w - lo] = (uint16_t)(r & ~(1u << c));
              hit = true;
            }
          }
        }
      }
      const uint64_t mask = __ballot(hit);
      if (tid == 0) stk[(uint64_t)dep * FW + 1 + ch] = mask;
    }
    __syncthreads();
  };
  auto undo_row = [&](uint32_t v, uint32_t c, uint32_t dep) {
    const uint32_t beg = adj[v], deg = adj[v + 1] - beg;
    for (uint32_t ch = 0; ch * 64u < deg; ++ch) {
      const uint64_t mask = stk[(uint64_t)dep * FW + 1 + ch];
      if (tid < 64 && ((mask >> tid) & 1ull)) {
        const uint32_t w = ids[beg + ch * 64u + tid];
        rm[w - lo] = (uint16_t)(rm[w - lo] | (1u << c));
      }
    }
    __syncthreads();
  };

  for (;;) {
    if (nodes == budget) { status = MPLD_BUDGET_EXHAUSTED; break; }
    ++nodes;
    if (open == 0) {
      if (TRACE) h = trace_node(h, depth, row_in, kNoneD, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    // 1. the slice's best column, folded into the device-wide key
    uint64_t key = ~0ull;
    for (uint32_t v = lo + tid; v < hi; v += kDevThreads) {
      const uint16_t r = rm[v - lo];
      if (!(r & kCovered))
        key = min64(key, ((uint64_t)__popc(r) << 40) | ((uint64_t)v << 8) | (r & 0xffu));
    }
    key = block_min(key, red);
    if (tid == 0 && key != ~0ull) atomicMin(&keys[slot], (unsigned long long)key);
    // 2. one barrier across the device; every block reads the winner
    grid.sync();
    const uint64_t win = __hip_atomic_load(&keys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (b == 0 && tid == 0)   // the slot used two nodes on
      __hip_atomic_store(&keys[slot == 0 ? 2 : slot - 1], ~0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    slot = slot == 2 ? 0 : slot + 1;
    uint32_t v = (uint32_t)(win >> 8);
    const uint32_t size = (uint32_t)(win >> 40);
    uint32_t rows = (uint32_t)win & 0xffu;
    if (TRACE) h = trace_node(h, depth, row_in, v, size);
    // 3. the same decision, replayed on this block's slice
    uint32_t c;
    if (size != 0) {
      if (v >= lo && v < hi && tid == 0) rm[v - lo] = (uint16_t)(rm[v - lo] | kCovered);
      --open;
      c = (uint32_t)__ffs(rows) - 1u;
    } else {
      uint32_t next = 0;
      while (depth != 0) {
        --depth;
        const uint64_t hdr = stk[(uint64_t)depth * FW];
        v = (uint32_t)hdr;
        const uint32_t cp = (uint32_t)(hdr >> 32) & 0xffu;
        rows = (uint32_t)(hdr >> 40) & 0xffu;
        undo_row(v, cp, depth);
        next = rows & (0xfffffffeu << cp);
        if (next) break;
        if (v >= lo && v < hi && tid == 0) rm[v - lo] = (uint16_t)(rm[v - lo] & ~kCovered);
        __syncthreads();   // the next undo may touch the same entry
        ++open;
      }
      if (!next) { status = MPLD_INFEASIBLE; break; }
      c = (uint32_t)__ffs(next) - 1u;
    }
    if (tid == 0) stk[(uint64_t)depth * FW] = (uint64_t)v | ((uint64_t)c << 32) | ((uint64_t)rows << 40);
    take_row(v, c, depth);
    ++depth;
    row_in = v * (uint32_t)k + c;
  }
  // block 0 writes the outputs from its frame headers
  if (b == 0) {
    int8_t* colors = colors_base + d.out_off;
    if (status == MPLD_FEASIBLE) {
      for (uint32_t f = tid; f < depth; f += kDevThreads) {
        const uint64_t hdr = stk[(uint64_t)f * FW];
        colors[(uint32_t)hdr] = (int8_t)((hdr >> 32) & 0xffu);
      }
    } else {
      for (uint32_t x = tid; x < (uint32_t)n; x += kDevThreads) colors[x] = -1;
    }
    if (tid == 0) {
      DevRecord* rec = recs + d.comp;
      rec->status = status;
      rec->depth = status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
      rec->nodes = nodes;
      rec->hash = h;
    }
  }
  // leave every key slot at ~0 for the next launch
  grid.sync();
  if (b == 0 && tid < 3) __hip_atomic_store(&keys[tid], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- host side ------------------------------------------------------------


// Stack words of one block (frames of n nodes) and LDS bytes of one block for
// a giant of n nodes on `grid` blocks.
int64_t device_tier_stack_words(int32_t n, int32_t max_deg) {
  return (int64_t)n * (1 + (max_deg + 63) / 64);
}

int device_tier_lds_bytes(int32_t n, int grid) {
  const uint32_t per = ((uint32_t)n + (uint32_t)grid - 1) / (uint32_t)grid;
  return (int)(((per * 2 + 15) & ~15u) + 8 * (kDevThreads / 64));
}

hipError_t launch_device_tier(bool trace, int grid, int lds_bytes, const DevDesc* desc,
                              const uint32_t* adj32, unsigned long long* keys, uint64_t* stacks,
                              DevRecord* recs, int8_t* colors, hipStream_t s) {
  void* args[] = {(void*)&desc, (void*)&adj32, (void*)&keys, (void*)&stacks, (void*)&recs,
                  (void*)&colors};
  const void* fn = trace ? reinterpret_cast<const void*>(&device_tier_kernel<true>)
                         : reinterpret_cast<const void*>(&device_tier_kernel<false>);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kDevThreads), args, (unsigned)lds_bytes, s);
}

}  // namespace mpld
