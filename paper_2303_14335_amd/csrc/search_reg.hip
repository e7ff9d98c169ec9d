// search_reg.hip - register tier of the exact-cover search (components of at
// most 64 nodes), one 64-lane wavefront per component.
//
// Exact-cover matrix (Sec. 2.3): one row (v, c) per node and color, a
// primary column per node, a secondary column per (conflict edge, color).
// Row (v, c) stays in the matrix while v is uncovered and no conflict
// neighbour of v has taken row (u, c); so the rows of primary column v are
// the colors still open to v, and the dancing-links state reduces to
//   rm[v]  - a k-bit mask of v's open colors, one lane per node (VGPR);
//   P      - the 64-bit set of uncovered primary columns (SGPR pair).
// Column choice (Algorithm 1): per lane count = popcount(rm); a wave ballot
// of count == t, masked with P, for t = 0, 1, ... gives the columns of the
// smallest count, and its lowest set bit is the lowest local index.
// Cover of row (v, c) (Eq. 2 "cover"): lanes u with v in N(u) and color c
// open clear bit c; the ballot of those lanes is the undo record.  Uncover
// (Eq. 2 "uncover") ORs the recorded lanes back.  The recursion of
// Algorithm 1 becomes an explicit stack held in three VGPRs, lane d holding
// frame d: (v | c << 8, removed-mask low, removed-mask high).
#include <hip/hip_runtime.h>

#include "device_types.h"
#include "mpld.h"

namespace mpld {

static constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
static constexpr uint64_t kFnvPrime = 0x100000001b3ull;
static constexpr uint32_t kNone = 0xffffffffu;

__device__ __forceinline__ uint64_t fnv_u32(uint64_t h, uint32_t v) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    h ^= (v >> (8 * b)) & 0xffu;
    h *= kFnvPrime;
  }
  return h;
}

__device__ __forceinline__ uint64_t trace_node(uint64_t h, uint32_t depth, uint32_t row_in,
                                               uint32_t col, uint32_t size) {
  h = fnv_u32(h, depth);
  h = fnv_u32(h, row_in);
  h = fnv_u32(h, col);
  return fnv_u32(h, size);
}

__device__ __forceinline__ uint32_t rdlane(uint32_t x, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)lane);
}
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// Search state of one component.  Per lane (VGPRs):
//   rm    open colors of the lane's node (k-bit row mask)
//   lost  bit d set iff this lane's node lost a color when the row at depth
//         d was taken (the undo record)
//   st    lane d holds frame d: v | c << 8
// Wave-uniform (SGPRs): P (uncovered columns), depth, nodes, hash, entering
// row, status (-1 while the search runs or is paused).
struct RegState {
  uint32_t rm, st;
  uint64_t lost;
  uint64_t P, nodes, h;
  uint32_t depth, row_in;
  int32_t status;
};

__device__ __forceinline__ void reg_init(RegState& s, int32_t n, int32_t k) {
  const uint32_t lane = __lane_id();
  s.rm = lane < (uint32_t)n ? ((1u << k) - 1u) : 0u;
  s.st = 0;
  s.lost = 0;
  s.P = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
  s.nodes = 0;
  s.h = kFnvOffset;
  s.depth = 0;
  s.row_in = kNone;
  s.status = -1;
}

// Runs the search until it ends or `nodes` reaches stop_at (<= budget); a
// stop short of the budget leaves status -1 and the state resumable at a
// node boundary.  With floor > 0 the search is confined to the subtree of
// the node at depth `floor` (backtracking never pops below it; exhausting
// the subtree reports MPLD_INFEASIBLE).  NB = bits of a row count
// (k < 2^NB).  Every lane of the wave must call it.
template <bool TRACE, int NB>
__device__ __forceinline__ void reg_run(RegState& s, const uint64_t nb, const int32_t k,
                                        const uint64_t budget, const uint64_t stop_at,
                                        const uint32_t floor = 0) {
  const uint32_t lane = __lane_id();
  uint32_t rm = s.rm, st = s.st, depth = s.depth, row_in = s.row_in;
  uint64_t lost = s.lost, P = s.P, nodes = s.nodes, h = s.h;
  int32_t status = -1;
  for (;;) {
    // ---- one search node
    if (nodes == stop_at) {
      if (nodes == budget) status = MPLD_BUDGET_EXHAUSTED;
      break;
    }
    ++nodes;
    if (P == 0) {
      if (TRACE) h = trace_node(h, depth, row_in, kNone, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    // column choice without branches: narrow the open columns to those of
    // the smallest row count one count bit at a time (most significant
    // first); the lowest survivor is the lowest index of that count
    const uint32_t cnt = __popc(rm);
    uint64_t cand = P;
#pragma unroll
    for (int j = NB - 1; j >= 0; --j) {
      const uint64_t one = __ballot((cnt >> j) & 1u);
      const uint64_t zero = cand & ~one;
      cand = zero ? zero : cand;
    }
    uint32_t v = (uint32_t)__ffsll((unsigned long long)cand) - 1u;
    const uint32_t size = rdlane(cnt, v);
    if (TRACE) h = trace_node(h, depth, row_in, v, size);
    uint32_t c;
    if (size != 0) {
      // cover column v, take its first open row
      P &= ~(1ull << v);
      c = (uint32_t)__ffs(rdlane(rm, v)) - 1u;
    } else {
      // dead end: undo rows and uncover columns until one has a next row
      uint32_t next = 0;
      while (depth != floor) {
        --depth;
        const uint32_t vc = rdlane(st, depth);
        v = vc & 0xffu;
        const uint32_t cp = vc >> 8;
        rm |= (uint32_t)((lost >> depth) & 1ull) << cp;
        lost &= ~(1ull << depth);
        next = rdlane(rm, v) & (0xfffffffeu << cp);
        if (next) break;
        P |= 1ull << v;
      }
      if (!next) { status = MPLD_INFEASIBLE; break; }
      c = (uint32_t)__ffs(next) - 1u;
    }
    // ---- include row (v, c): close color c at v's neighbours that have it
    const uint32_t hit = (uint32_t)(nb >> v) & (rm >> c) & 1u;
    rm &= ~(hit << c);
    lost |= (uint64_t)hit << depth;
    st = lane == depth ? (v | (c << 8)) : st;
    ++depth;
    row_in = v * (uint32_t)k + c;
  }
  s.rm = rm; s.st = st; s.depth = depth; s.row_in = row_in;
  s.lost = lost; s.P = P; s.nodes = nodes; s.h = h;
  s.status = status;
}

// Writes the colors (the chosen row of every column on a solution, -1
// otherwise) and the record of a finished search.
__device__ __forceinline__ void reg_finish(const RegState& s, int32_t n, int8_t* __restrict__ colors,
                                           DevRecord* __restrict__ rec) {
  const uint32_t lane = __lane_id();
  if (s.status == MPLD_FEASIBLE) {
    if (lane < s.depth && (s.st & 0xffu) < (uint32_t)n) colors[s.st & 0xffu] = (int8_t)(s.st >> 8);
  } else if (lane < (uint32_t)n) {
    colors[lane] = -1;
  }
  // Every lane stores the same (uniform) record: no branch here may share
  // the queue pop's "lane 0" condition, or the compiler can thread the two
  // across the loop back-edge and split the wave at the pop.
  rec->status = s.status;
  rec->depth = s.status == MPLD_INFEASIBLE ? 0 : (int32_t)s.depth;
  rec->nodes = s.nodes;
  rec->hash = s.h;
}

// cap < budget stops the search after `cap` nodes (status -1 in the record:
// the component is left to the heavy-component engine).
template <bool TRACE, int NB>
__device__ __forceinline__ void solve_reg(const int32_t n, const int32_t k, const uint64_t budget,
                                          const uint64_t* __restrict__ nbmask,
                                          int8_t* __restrict__ colors,
                                          DevRecord* __restrict__ rec,
                                          const uint64_t cap = ~0ull) {
  const uint32_t lane = __lane_id();
  const uint64_t nb = lane < (uint32_t)n ? nbmask[lane] : 0ull;
  RegState s;
  reg_init(s, n, k);
  reg_run<TRACE, NB>(s, nb, k, budget, cap < budget ? cap : budget);
  reg_finish(s, n, colors, rec);
}

// Resumable state in device memory (kRegStateBytes per component): the
// uniform part first, then the three lane arrays.
struct RegStateHead {
  uint64_t P, nodes, h;
  uint32_t depth, row_in;
};
static_assert(sizeof(RegStateHead) == 32, "state head is 32 bytes");

__device__ __forceinline__ void reg_save(const RegState& s, uint8_t* base) {
  const uint32_t lane = __lane_id();
  RegStateHead* hd = reinterpret_cast<RegStateHead*>(base);
  hd->P = s.P;   // same value from every lane
  hd->nodes = s.nodes;
  hd->h = s.h;
  hd->depth = s.depth;
  hd->row_in = s.row_in;
  reinterpret_cast<uint32_t*>(base + 64)[lane] = s.rm;
  reinterpret_cast<uint32_t*>(base + 64 + 256)[lane] = s.st;
  reinterpret_cast<uint64_t*>(base + 64 + 512)[lane] = s.lost;
}

__device__ __forceinline__ void reg_load(RegState& s, const uint8_t* base) {
  const uint32_t lane = __lane_id();
  const RegStateHead* hd = reinterpret_cast<const RegStateHead*>(base);
  s.P = ((uint64_t)uniform((uint32_t)(hd->P >> 32)) << 32) | uniform((uint32_t)hd->P);
  s.nodes = ((uint64_t)uniform((uint32_t)(hd->nodes >> 32)) << 32) | uniform((uint32_t)hd->nodes);
  s.h = ((uint64_t)uniform((uint32_t)(hd->h >> 32)) << 32) | uniform((uint32_t)hd->h);
  s.depth = uniform(hd->depth);
  s.row_in = uniform(hd->row_in);
  s.rm = reinterpret_cast<const uint32_t*>(base + 64)[lane];
  s.st = reinterpret_cast<const uint32_t*>(base + 64 + 256)[lane];
  s.lost = reinterpret_cast<const uint64_t*>(base + 64 + 512)[lane];
  s.status = -1;
}

// Persistent batched kernel.  Wave w first takes item w of its tier's
// descriptor list (no atomic); while the grid has fewer waves than items,
// waves then pop item gw + atomicAdd(counter, 1).  Every wave fails exactly
// one pop, so the pop that returns qlen - 1 is the last one: it resets the
// counter to 0 and the launch (or the graph holding it) can be replayed with
// no memset.
template <bool TRACE, int NB>
__global__ __launch_bounds__(256) void reg_batched_kernel(
    const DevDesc* __restrict__ descs, const uint64_t* __restrict__ masks, int32_t qlen,
    int32_t* __restrict__ counter, DevRecord* __restrict__ recs, int8_t* __restrict__ colors,
    uint64_t cap) {
  const uint32_t wpb = blockDim.x >> 6;   // waves per workgroup
  const int32_t gw = (int32_t)(gridDim.x * wpb);
  int32_t item = (int32_t)uniform(blockIdx.x * wpb + (threadIdx.x >> 6));
  while (item < qlen) {
    const DevDesc d = descs[item];
    solve_reg<TRACE, NB>(d.n, d.k, (uint64_t)d.budget, masks + d.nbr_off, colors + d.out_off,
                         recs + d.comp, cap);
    if (gw >= qlen) break;   // every item was handed out statically
    int32_t r = 0;
    if (__lane_id() == 0) r = atomicAdd(counter, 1);
    r = (int32_t)uniform((uint32_t)r);
    item = gw + r;
    if (r == qlen - 1) atomicExch(counter, 0);   // the last pop of this launch
  }
}

// One component per launch (the plain solver): a single wave.
template <bool TRACE, int NB>
__global__ __launch_bounds__(64) void reg_single_kernel(const DevDesc* __restrict__ descs,
                                                        const uint64_t* __restrict__ masks,
                                                        int32_t item, DevRecord* __restrict__ recs,
                                                        int8_t* __restrict__ colors) {
  const DevDesc d = descs[item];
  solve_reg<TRACE, NB>(d.n, d.k, (uint64_t)d.budget, masks + d.nbr_off, colors + d.out_off,
                       recs + d.comp);
}

// Serving tick: every listed component advances by at most `slice` search
// nodes from its saved state (entries with bit 31 set start fresh).  A
// finished search writes its colors and record; a paused one saves its
// state.  tick_out[i] receives the record of list entry i (status -1 while
// the search is still running).  Work distribution as in the batched kernel.
template <bool TRACE, int NB>
__global__ __launch_bounds__(256) void reg_tick_kernel(
    const int32_t* __restrict__ list, int32_t len, int32_t* __restrict__ counter,
    const DevDesc* __restrict__ slot_desc, uint8_t* slot_state, DevRecord* __restrict__ slot_rec,
    const uint64_t* __restrict__ arena64, int8_t* __restrict__ arena8, uint64_t slice,
    DevRecord* __restrict__ tick_out) {
  const int32_t gw = (int32_t)gridDim.x * 4;
  int32_t item = (int32_t)uniform(blockIdx.x * 4u + (threadIdx.x >> 6));
  while (item < len) {
    const uint32_t entry = uniform((uint32_t)list[item]);
    const int32_t slot = (int32_t)(entry & 0x7fffffffu);
    const DevDesc d = slot_desc[slot];
    const uint32_t lane = __lane_id();
    const uint64_t nb = lane < (uint32_t)d.n ? arena64[d.nbr_off + lane] : 0ull;
    uint8_t* base = slot_state + (uint64_t)slot * kRegStateBytes;
    RegState s;
    if (entry >> 31)
      reg_init(s, d.n, d.k);
    else
      reg_load(s, base);
    const uint64_t budget = (uint64_t)d.budget;
    const uint64_t stop = budget - s.nodes > slice ? s.nodes + slice : budget;
    reg_run<TRACE, NB>(s, nb, d.k, budget, stop);
    if (s.status >= 0)
      reg_finish(s, d.n, arena8 + d.out_off, slot_rec + slot);
    else
      reg_save(s, base);
    DevRecord* o = tick_out + item;
    o->status = s.status;
    o->depth = (int32_t)s.depth;
    o->nodes = s.nodes;
    o->hash = s.h;
    if (gw >= len) break;
    int32_t r = 0;
    if (__lane_id() == 0) r = atomicAdd(counter, 1);
    r = (int32_t)uniform((uint32_t)r);
    item = gw + r;
    if (r == len - 1) atomicExch(counter, 0);
  }
}

// ---- heavy-component engine: subtree tasks --------------------------------

// Rebuilds the search state at the end of a path of rows from the root:
// cover each row's column and take the row, in order (the same applies the
// sequential search made on the way down).
__device__ __forceinline__ void reg_replay(RegState& s, const uint64_t nb, const int32_t k,
                                           const uint16_t* __restrict__ rows, uint32_t d) {
  const uint32_t lane = __lane_id();
  for (uint32_t j = 0; j < d; ++j) {
    const uint32_t vc = uniform(rows[j]);
    const uint32_t v = vc & 0xffu, c = vc >> 8;
    s.P &= ~(1ull << v);
    const uint32_t hit = (uint32_t)(nb >> v) & (s.rm >> c) & 1u;
    s.rm &= ~(hit << c);
    s.lost |= (uint64_t)hit << j;
    s.st = lane == j ? vc : s.st;
    s.row_in = v * (uint32_t)k + c;
  }
  s.depth = d;
}

// Enumerates the top `levels` levels of the subtree rooted at depth d in
// search order: counts their nodes, and emits a kind-0 item for every node
// at depth d + levels (not counted here: its own task counts it), a kind-2
// item when a solution is met (writing its colors) or a kind-1 item at the
// end.  Returns the number of items.
template <int NB>
__device__ __forceinline__ int32_t reg_enumerate(RegState& s, const uint64_t nb, const int32_t k,
                                                 const int32_t n, const uint32_t d,
                                                 const uint32_t levels, SplitItem* __restrict__ out,
                                                 int8_t* __restrict__ sol) {
  const uint32_t lane = __lane_id();
  const uint32_t limit = d + levels;
  uint32_t rm = s.rm, st = s.st, depth = s.depth;
  uint64_t lost = s.lost, P = s.P;
  uint32_t seg = 0;
  int32_t items = 0;
  auto emit = [&](uint32_t kind) {
    const uint32_t r0 = kind == 0 ? rdlane(st, d) : 0u;
    const uint32_t r1 = kind == 0 && levels > 1 ? rdlane(st, d + 1) : 0u;
    const uint32_t r2 = kind == 0 && levels > 2 ? rdlane(st, d + 2) : 0u;
    const uint32_t r3 = kind == 0 && levels > 3 ? rdlane(st, d + 3) : 0u;
    if (lane == ((uint32_t)items & 63u)) {   // one owner lane per item
      SplitItem it;
      it.seg = seg;
      it.kind = kind;
      it.rows[0] = (uint16_t)r0;
      it.rows[1] = (uint16_t)r1;
      it.rows[2] = (uint16_t)r2;
      it.rows[3] = (uint16_t)r3;
      out[items] = it;
    }
    ++items;
    seg = 0;
  };
  for (;;) {
    bool back;
    uint32_t v = 0, c = 0;
    if (depth == limit) {
      emit(0);        // a subtask root: leave it to its own task
      back = true;
    } else {
      ++seg;
      if (P == 0) {   // a solution among the top levels
        if (lane < depth && (st & 0xffu) < (uint32_t)n) sol[st & 0xffu] = (int8_t)(st >> 8);
        emit(2);
        break;
      }
      const uint32_t cnt = __popc(rm);
      uint64_t cand = P;
#pragma unroll
      for (int j = NB - 1; j >= 0; --j) {
        const uint64_t one = __ballot((cnt >> j) & 1u);
        const uint64_t zero = cand & ~one;
        cand = zero ? zero : cand;
      }
      v = (uint32_t)__ffsll((unsigned long long)cand) - 1u;
      if (rdlane(cnt, v) != 0) {
        P &= ~(1ull << v);
        c = (uint32_t)__ffs(rdlane(rm, v)) - 1u;
        back = false;
      } else {
        back = true;
      }
    }
    if (back) {
      uint32_t next = 0;
      while (depth != d) {
        --depth;
        const uint32_t vc = rdlane(st, depth);
        v = vc & 0xffu;
        const uint32_t cp = vc >> 8;
        rm |= (uint32_t)((lost >> depth) & 1ull) << cp;
        lost &= ~(1ull << depth);
        next = rdlane(rm, v) & (0xfffffffeu << cp);
        if (next) break;
        P |= 1ull << v;
      }
      if (!next) {
        emit(1);
        break;
      }
      c = (uint32_t)__ffs(next) - 1u;
    }
    const uint32_t hit = (uint32_t)(nb >> v) & (rm >> c) & 1u;
    rm &= ~(hit << c);
    lost |= (uint64_t)hit << depth;
    st = lane == depth ? (v | (c << 8)) : st;
    ++depth;
  }
  return items;
}

// One wave per task: explore the task's subtree up to `cap` nodes; if the
// cap is hit, split the task `levels` levels down instead.
template <int NB>
__global__ __launch_bounds__(256) void reg_split_kernel(
    const SplitTask* __restrict__ tasks, int32_t ntasks, int32_t* __restrict__ counter,
    const DevDesc* __restrict__ descs, const uint64_t* __restrict__ masks, uint64_t cap,
    uint32_t levels, int32_t max_items, SplitResult* __restrict__ results,
    SplitItem* __restrict__ items, int8_t* __restrict__ sols) {
  const uint32_t wpb = blockDim.x >> 6;
  const int32_t gw = (int32_t)(gridDim.x * wpb);
  int32_t t = (int32_t)uniform(blockIdx.x * wpb + (threadIdx.x >> 6));
  const uint32_t lane = __lane_id();
  while (t < ntasks) {
    const SplitTask* task = tasks + t;
    const int32_t it = (int32_t)uniform((uint32_t)task->item);
    const uint32_t d = uniform((uint32_t)task->depth);
    const DevDesc dd = descs[it];
    const uint64_t nb = lane < (uint32_t)dd.n ? masks[dd.nbr_off + lane] : 0ull;
    int8_t* sol = sols + (uint64_t)t * 64;
    RegState s;
    reg_init(s, dd.n, dd.k);
    reg_replay(s, nb, dd.k, task->rows, d);
    reg_run<false, NB>(s, nb, dd.k, ~0ull, cap, d);
    int32_t nitems = 0;
    if (s.status == MPLD_FEASIBLE) {
      if (lane < s.depth && (s.st & 0xffu) < (uint32_t)dd.n) sol[s.st & 0xffu] = (int8_t)(s.st >> 8);
    } else if (s.status < 0) {
      RegState r;
      reg_init(r, dd.n, dd.k);
      reg_replay(r, nb, dd.k, task->rows, d);
      nitems = reg_enumerate<NB>(r, nb, dd.k, dd.n, d, levels,
                                 items + (uint64_t)t * (uint64_t)max_items, sol);
    }
    SplitResult res;
    res.status = s.status;
    res.nitems = nitems;
    res.nodes = s.nodes;
    results[t] = res;   // same value from every lane
    if (gw >= ntasks) break;
    int32_t r = 0;
    if (__lane_id() == 0) r = atomicAdd(counter, 1);
    r = (int32_t)uniform((uint32_t)r);
    t = gw + r;
    if (r == ntasks - 1) atomicExch(counter, 0);
  }
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int32_t count, int32_t value) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < count) p[i] = value;
}

// ---- host-side launchers -------------------------------------------------

hipError_t launch_fill_i32(int32_t* p, int32_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

// Row counts of k colors need count_bits(k) bits.
static int count_bits(int k) { return k < 4 ? 2 : (k < 8 ? 3 : 4); }

template <bool TRACE, int NB>
static void reg_batched_t(int grid, int wpb, const DevDesc* descs, const uint64_t* masks,
                          int32_t qlen, int32_t* counter, DevRecord* recs, int8_t* colors,
                          uint64_t cap, hipStream_t s) {
  hipLaunchKernelGGL((reg_batched_kernel<TRACE, NB>), dim3(grid), dim3(64 * wpb), 0, s, descs,
                     masks, qlen, counter, recs, colors, cap);
}

template <bool TRACE, int NB>
static void reg_single_t(const DevDesc* descs, const uint64_t* masks, int32_t item,
                         DevRecord* recs, int8_t* colors, hipStream_t s) {
  hipLaunchKernelGGL((reg_single_kernel<TRACE, NB>), dim3(1), dim3(64), 0, s, descs, masks, item,
                     recs, colors);
}

hipError_t launch_reg_batched(bool trace, int k, int grid, int wpb, const DevDesc* descs,
                              const uint64_t* masks, int32_t qlen, int32_t* counter,
                              DevRecord* recs, int8_t* colors, uint64_t cap, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
  switch (count_bits(k) + (trace ? 8 : 0)) {
    case 2: reg_batched_t<false, 2>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
    case 3: reg_batched_t<false, 3>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
    case 4: reg_batched_t<false, 4>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
    case 10: reg_batched_t<true, 2>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
    case 11: reg_batched_t<true, 3>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
    default: reg_batched_t<true, 4>(grid, wpb, descs, masks, qlen, counter, recs, colors, cap, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_reg_single(bool trace, int k, const DevDesc* descs, const uint64_t* masks,
                             int32_t item, DevRecord* recs, int8_t* colors, hipStream_t s) {
  switch (count_bits(k) + (trace ? 8 : 0)) {
    case 2: reg_single_t<false, 2>(descs, masks, item, recs, colors, s); break;
    case 3: reg_single_t<false, 3>(descs, masks, item, recs, colors, s); break;
    case 4: reg_single_t<false, 4>(descs, masks, item, recs, colors, s); break;
    case 10: reg_single_t<true, 2>(descs, masks, item, recs, colors, s); break;
    case 11: reg_single_t<true, 3>(descs, masks, item, recs, colors, s); break;
    default: reg_single_t<true, 4>(descs, masks, item, recs, colors, s); break;
  }
  return hipGetLastError();
}

template <bool TRACE, int NB>
static void reg_tick_t(int grid, const int32_t* list, int32_t len, int32_t* counter,
                       const DevDesc* slot_desc, uint8_t* slot_state, DevRecord* slot_rec,
                       const uint64_t* arena64, int8_t* arena8, uint64_t slice,
                       DevRecord* tick_out, hipStream_t s) {
  hipLaunchKernelGGL((reg_tick_kernel<TRACE, NB>), dim3(grid), dim3(256), 0, s, list, len, counter,
                     slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out);
}

hipError_t launch_reg_tick(bool trace, int k, int grid, const int32_t* list, int32_t len,
                           int32_t* counter, const DevDesc* slot_desc, uint8_t* slot_state,
                           DevRecord* slot_rec, const uint64_t* arena64, int8_t* arena8,
                           uint64_t slice, DevRecord* tick_out, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  switch (count_bits(k) + (trace ? 8 : 0)) {
    case 2: reg_tick_t<false, 2>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
    case 3: reg_tick_t<false, 3>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
    case 4: reg_tick_t<false, 4>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
    case 10: reg_tick_t<true, 2>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
    case 11: reg_tick_t<true, 3>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
    default: reg_tick_t<true, 4>(grid, list, len, counter, slot_desc, slot_state, slot_rec, arena64, arena8, slice, tick_out, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_reg_split(int k, int grid, const SplitTask* tasks, int32_t ntasks,
                            int32_t* counter, const DevDesc* descs, const uint64_t* masks,
                            uint64_t cap, uint32_t levels, int32_t max_items,
                            SplitResult* results, SplitItem* items, int8_t* sols, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (levels < 1 || levels > (uint32_t)kSplitMaxLevels) return hipErrorInvalidValue;
  switch (count_bits(k)) {
    case 2:
      hipLaunchKernelGGL((reg_split_kernel<2>), dim3(grid), dim3(256), 0, s, tasks, ntasks, counter,
                         descs, masks, cap, levels, max_items, results, items, sols);
      break;
    case 3:
      hipLaunchKernelGGL((reg_split_kernel<3>), dim3(grid), dim3(256), 0, s, tasks, ntasks, counter,
                         descs, masks, cap, levels, max_items, results, items, sols);
      break;
    default:
      hipLaunchKernelGGL((reg_split_kernel<4>), dim3(grid), dim3(256), 0, s, tasks, ntasks, counter,
                         descs, masks, cap, levels, max_items, results, items, sols);
      break;
  }
  return hipGetLastError();
}

int reg_batched_blocks_per_cu(bool trace) {
  int blocks = 0;
  hipError_t e = trace ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<true, 4>, 256, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<false, 4>, 256, 0);
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

}  // namespace mpld
