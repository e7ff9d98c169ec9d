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

// Searches one component; every lane of the wave must call it.
template <bool TRACE>
__device__ __forceinline__ void solve_reg(const int32_t n, const int32_t k, const uint64_t budget,
                                          const uint64_t* __restrict__ nbmask,
                                          int8_t* __restrict__ colors,
                                          DevRecord* __restrict__ rec) {
  const uint32_t lane = __lane_id();
  const uint64_t nb = lane < (uint32_t)n ? nbmask[lane] : 0ull;
  uint32_t rm = lane < (uint32_t)n ? ((1u << k) - 1u) : 0u;
  uint64_t P = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
  uint32_t st_vc = 0, st_lo = 0, st_hi = 0;
  uint32_t depth = 0;
  uint64_t nodes = 0;
  uint64_t h = kFnvOffset;
  uint32_t row_in = kNone;
  int32_t status;
  for (;;) {
    // ---- one search node
    if (nodes == budget) { status = MPLD_BUDGET_EXHAUSTED; break; }
    ++nodes;
    if (P == 0) {
      if (TRACE) h = trace_node(h, depth, row_in, kNone, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    const uint32_t cnt = __popc(rm);
    uint64_t sel = 0;
    uint32_t size = 0;
    for (uint32_t t = 0; t <= (uint32_t)k; ++t) {
      sel = __ballot(cnt == t) & P;
      if (sel) { size = t; break; }
    }
    if (sel == 0) { status = 3; break; }   // cannot happen while P != 0; reported as a bug
    uint32_t v = (uint32_t)__ffsll((unsigned long long)sel) - 1u;
    uint32_t c;
    if (TRACE) h = trace_node(h, depth, row_in, v, size);
    if (size != 0) {
      // cover column v, take its first open row
      P &= ~(1ull << v);
      c = (uint32_t)__ffs(rdlane(rm, v)) - 1u;
    } else {
      // dead end: uncover rows and columns until a column has a next row
      for (;;) {
        if (depth == 0) { status = MPLD_INFEASIBLE; goto done; }
        --depth;
        const uint32_t vc = rdlane(st_vc, depth);
        const uint64_t rem = ((uint64_t)rdlane(st_hi, depth) << 32) | rdlane(st_lo, depth);
        v = vc & 0xffu;
        const uint32_t cp = vc >> 8;
        rm |= (uint32_t)((rem >> lane) & 1ull) << cp;
        const uint32_t next = rdlane(rm, v) & ~((2u << cp) - 1u);
        if (next) { c = (uint32_t)__ffs(next) - 1u; break; }
        P |= 1ull << v;
      }
    }
    // ---- include row (v, c): close color c at the open neighbours of v
    {
      const bool hit = ((nb >> v) & 1ull) && ((rm >> c) & 1u);
      const uint64_t rem = __ballot(hit);
      rm &= ~((uint32_t)hit << c);
      const bool mine = lane == depth;   // frame `depth` lives in lane `depth`
      st_vc = mine ? (v | (c << 8)) : st_vc;
      st_lo = mine ? (uint32_t)rem : st_lo;
      st_hi = mine ? (uint32_t)(rem >> 32) : st_hi;
      ++depth;
      row_in = v * (uint32_t)k + c;
    }
  }
done:
  if (status == MPLD_FEASIBLE) {
    if (lane < depth && (st_vc & 0xffu) < (uint32_t)n) colors[st_vc & 0xffu] = (int8_t)(st_vc >> 8);
  } else if (lane < (uint32_t)n) {
    colors[lane] = -1;
  }
  // Every lane stores the same (uniform) record: no branch here may share
  // the queue pop's "lane 0" condition, or the compiler can thread the two
  // across the loop back-edge and split the wave at the pop.
  rec->status = status;
  rec->depth = status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
  rec->nodes = nodes;
  rec->hash = h;
}

// Persistent batched kernel: every wave pops component ids from the queue
// until it is empty.  counters[0] = queue head, counters[1] = finished
// waves; both are 0 at launch and the last wave to finish resets them, so
// the same launch (or a graph holding it) can be replayed.
template <bool TRACE>
__global__ __launch_bounds__(256) void reg_batched_kernel(
    const DevDesc* __restrict__ descs, const uint64_t* __restrict__ masks,
    const int32_t* __restrict__ queue, int32_t qlen, int32_t* __restrict__ counters,
    int32_t total_waves, DevRecord* __restrict__ recs, int8_t* __restrict__ colors) {
  for (;;) {
    int32_t item = 0;
    if (__lane_id() == 0) item = atomicAdd(&counters[0], 1);
    item = (int32_t)uniform((uint32_t)item);
    if (item >= qlen) break;
    const int32_t comp = (int32_t)uniform((uint32_t)queue[item]);
    const DevDesc d = descs[comp];
    solve_reg<TRACE>(d.n, d.k, (uint64_t)d.budget, masks + d.nbr_off, colors + d.out_off,
                     recs + comp);
  }
  if (__lane_id() == 0) {
    const int32_t done = atomicAdd(&counters[1], 1);
    if (done == total_waves - 1) {
      atomicExch(&counters[0], 0);
      atomicExch(&counters[1], 0);
    }
  }
}

// One component per launch (the plain solver): a single wave.
template <bool TRACE>
__global__ __launch_bounds__(64) void reg_single_kernel(const DevDesc* __restrict__ descs,
                                                        const uint64_t* __restrict__ masks,
                                                        int32_t comp, DevRecord* __restrict__ recs,
                                                        int8_t* __restrict__ colors) {
  const DevDesc d = descs[comp];
  solve_reg<TRACE>(d.n, d.k, (uint64_t)d.budget, masks + d.nbr_off, colors + d.out_off,
                   recs + comp);
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

hipError_t launch_reg_batched(bool trace, int grid, const DevDesc* descs, const uint64_t* masks,
                              const int32_t* queue, int32_t qlen, int32_t* counters,
                              DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  const int32_t waves = grid * 4;
  if (trace)
    hipLaunchKernelGGL(reg_batched_kernel<true>, dim3(grid), dim3(256), 0, s, descs, masks, queue,
                       qlen, counters, waves, recs, colors);
  else
    hipLaunchKernelGGL(reg_batched_kernel<false>, dim3(grid), dim3(256), 0, s, descs, masks, queue,
                       qlen, counters, waves, recs, colors);
  return hipGetLastError();
}

hipError_t launch_reg_single(bool trace, const DevDesc* descs, const uint64_t* masks, int32_t comp,
                             DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (trace)
    hipLaunchKernelGGL(reg_single_kernel<true>, dim3(1), dim3(64), 0, s, descs, masks, comp, recs,
                       colors);
  else
    hipLaunchKernelGGL(reg_single_kernel<false>, dim3(1), dim3(64), 0, s, descs, masks, comp, recs,
                       colors);
  return hipGetLastError();
}

int reg_batched_blocks_per_cu(bool trace) {
  int blocks = 0;
  hipError_t e = trace ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<true>, 256, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<false>, 256, 0);
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

}  // namespace mpld
