// search_min.hip - Eq. 1 minimisation of register-tier components (at most
// 64 nodes), one 64-lane wavefront per component.
//
// Eq. 1 (Sec. 2.1) asks for a coloring of least conflicts + alpha x
// stitches (alpha = 0.1).  The exact-cover search of Algorithm 1 stops at
// the first exact cover or reports that none exists; Algorithm 1's conflict
// candidates (a column left with no related row) give a coloring with
// conflicts but no claim of least cost.  Here the exact cover is relaxed:
// a row (v, c) whose secondary columns are already covered may still be
// taken, each covered (edge, color) column counting one conflict, and a row
// whose node's stitch partner holds another color counts one stitch.  A
// depth-first branch and bound over the rows, started from the incumbent
// coloring the search (or the conflict marking) left, finds a coloring of
// least cost = 10 conflicts + stitches (Eq. 1 scaled by 10, integers):
//   - penalty of (u, c) for an uncolored node u: 10 x (colored neighbours
//     of color c) + 1 if u's partner is colored with a color other than c;
//   - bound = cost so far + the sum over uncolored u of u's least penalty
//     (each term charges edges to colored nodes only, so the terms are
//     disjoint and only grow);
//   - a node entry passing the budget test counts one node; with every node
//     colored it replaces the incumbent when cheaper; otherwise it returns
//     when the bound reaches the incumbent's cost, else branches on the
//     uncolored node with the fewest conflict-free colors (lowest index on
//     ties) and tries the colors in ascending order, skipping a color whose
//     child bound (bound - least(v) + penalty(v, c)) reaches the incumbent's
//     cost when it is tried.
// Lane u holds u's neighbour mask, its stitch partner, its color (-1 while
// uncolored), the per-color counts of its colored neighbours (one byte per
// color) and the color of its partner.  The recursion is an explicit stack
// in VGPRs, lane d holding frame d: the node and color taken at depth d,
// the bound and the node's least penalty at that depth, and the cost
// before the row was taken.  Undoing a row restores that frame.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_types.h"
#include "mpld.h"
#include "reg_items.h"
#include "wave_ops.h"

namespace mpld {

template <int K>
struct MinLane {
  uint64_t nb;     // conflict neighbours
  uint32_t part;   // stitch partner, 0xff none
  int32_t col;     // color, -1 uncolored
  uint64_t cnt;    // byte c: colored neighbours of color c
  int32_t pcol;    // partner's color, -1 none or uncolored
};

template <int K>
__device__ __forceinline__ uint32_t min_pen(const MinLane<K>& L, uint32_t c) {
  return 10u * (uint32_t)((L.cnt >> (8 * c)) & 0xffu) + ((L.pcol >= 0 && L.pcol != (int32_t)c) ? 1u : 0u);
}

// Colors node v with c (on = true) or takes the color back.
template <int K>
__device__ __forceinline__ void min_set(MinLane<K>& L, uint32_t lane, uint32_t v, uint32_t c, bool on) {
  const uint64_t one = 1ull << (8 * c);
  if ((L.nb >> v) & 1ull) L.cnt = on ? L.cnt + one : L.cnt - one;
  if (L.part == v) L.pcol = on ? (int32_t)c : -1;
  if (lane == v) L.col = on ? (int32_t)c : -1;
}

// Returns the branch-and-bound nodes, negated when the budget stopped it;
// 0 when the incumbent costs nothing.  Writes the best coloring.
template <int K>
__device__ int32_t minimize_reg(const RegItems& items, int32_t item, const uint8_t* __restrict__ partners,
                                int8_t* __restrict__ colors_base, uint32_t budget) {
  const uint32_t lane = __lane_id();
  const DevDesc d = item_desc(items, item);
  const uint32_t n = uniform((uint32_t)d.n);
  const bool in = lane < n;
  MinLane<K> L;
  L.nb = item_mask(items, item, lane);
  L.part = in ? (uint32_t)partners[d.nbr_off + lane] : 0xffu;
  const int32_t inc = in ? (int32_t)colors_base[d.out_off + lane] : 0;
  // incumbent cost: conflict ends of each lane (each edge twice) and the
  // stitch pairs seen from their lower end
  uint64_t same = 0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const uint64_t m = __ballot(in && inc == c);
    if (in && inc == c) same = m;
  }
  const uint32_t pinc = (uint32_t)__shfl(inc, (int)(L.part & 63u));
  const uint32_t ends = in ? (uint32_t)__popcll(L.nb & same) : 0u;
  const uint32_t st = (in && L.part != 0xffu && L.part > lane && pinc != (uint32_t)inc) ? 1u : 0u;
  const uint32_t cost0 = uniform(10u * (wave_sum_u32(ends) / 2u) + wave_sum_u32(st));
  if (cost0 == 0u) return 0;

  L.col = -1;
  L.cnt = 0;
  L.pcol = -1;
  int32_t best_col = inc;
  uint32_t best = cost0, cost = 0, depth = 0, nodes = 0;
  bool stopped = false;
  uint32_t fr = 0, flb = 0, fmp = 0, fcost = 0;   // stack, lane = depth
  uint32_t v = 0, c0 = 0, lb = 0, mpv = 0;
  bool enter = true;
  for (;;) {
    bool down = false;
    if (enter) {
      if (nodes == budget) {
        stopped = true;
        break;
      }
      ++nodes;
      const bool unc = in && L.col < 0;
      if (__ballot(unc) == 0ull) {   // every node colored: cheaper than the incumbent?
        if (cost < best) {
          best = cost;
          best_col = L.col;
        }
      } else {
        uint32_t mp = 0xffffffffu, open = 0;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          mp = min(mp, min_pen<K>(L, (uint32_t)c));
          open += ((L.cnt >> (8 * c)) & 0xffu) == 0u ? 1u : 0u;
        }
        lb = uniform(cost + wave_sum_u32(unc ? mp : 0u));
        if (lb < best) {
          const uint32_t key = wave_min_u32(unc ? (open << 8) | lane : 0xffffffffu);
          v = uniform(key & 0xffu);
          mpv = uniform(rdlane(mp, v));
          c0 = 0;
          down = true;
        }
      }
    } else {
      down = true;
    }
    if (down) {
      // the next color of v whose child bound stays below the incumbent
      const uint64_t cntv = rdlane64((uint32_t)L.cnt, (uint32_t)(L.cnt >> 32), v);
      const int32_t pcv = (int32_t)rdlane((uint32_t)L.pcol, v);
      uint32_t take = K, pen = 0;
      for (uint32_t c = c0; c < (uint32_t)K; ++c) {
        const uint32_t p = 10u * (uint32_t)((cntv >> (8 * c)) & 0xffu) + ((pcv >= 0 && pcv != (int32_t)c) ? 1u : 0u);
        if (lb - mpv + p < best) {
          take = c;
          pen = p;
          break;
        }
      }
      if (take < (uint32_t)K) {
        fr = wrlane(fr, depth, v | (take << 8));
        flb = wrlane(flb, depth, lb);
        fmp = wrlane(fmp, depth, mpv);
        fcost = wrlane(fcost, depth, cost);
        min_set<K>(L, lane, v, take, true);
        cost += pen;
        ++depth;
        enter = true;
        continue;
      }
    }
    // back up one level: undo its row, go on with its next color
    if (depth == 0u) break;
    --depth;
    const uint32_t f = uniform(rdlane(fr, depth));
    v = f & 0xffu;
    const uint32_t c = f >> 8;
    lb = uniform(rdlane(flb, depth));
    mpv = uniform(rdlane(fmp, depth));
    cost = uniform(rdlane(fcost, depth));
    min_set<K>(L, lane, v, c, false);
    c0 = c + 1;
    enter = false;
  }
  if (in) colors_base[d.out_off + lane] = (int8_t)best_col;
  return stopped ? -(int32_t)nodes : (int32_t)nodes;
}

// One wave per workgroup, register-tier items taken grid-stride; every
// item's incumbent colors are in `colors` (the search's solution or the
// conflict marking).  min_out[comp] receives the node count (negated when
// the budget stopped the item), 0 when the incumbent costs nothing.
template <int K>
__global__ __launch_bounds__(64) void min_reg_kernel(const RegItems items, int32_t qlen,
                                                     const uint8_t* __restrict__ partners,
                                                     int8_t* __restrict__ colors,
                                                     int32_t* __restrict__ min_out, uint32_t budget) {
  for (int32_t i = (int32_t)uniform(blockIdx.x); i < qlen; i += (int32_t)gridDim.x) {
    const int32_t comp = (int32_t)uniform((uint32_t)item_desc(items, i).comp);
    const int32_t r = minimize_reg<K>(items, i, partners, colors, budget);
    if (__lane_id() == 0) min_out[comp] = r;
  }
}

template <class F>
static void with_colors(int k, F&& f) {
  switch (k) {
    case 2: f(std::integral_constant<int, 2>()); break;
    case 3: f(std::integral_constant<int, 3>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 5: f(std::integral_constant<int, 5>()); break;
    case 6: f(std::integral_constant<int, 6>()); break;
    case 7: f(std::integral_constant<int, 7>()); break;
    default: f(std::integral_constant<int, 8>()); break;
  }
}

hipError_t launch_min_reg(int k, int grid, RegItems items, int32_t qlen, const uint8_t* partners,
                          int8_t* colors, int32_t* min_out, uint32_t budget, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  if (k < 2 || k > 8 || grid < 1 || budget < 1) return hipErrorInvalidValue;
  with_colors(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    hipLaunchKernelGGL((min_reg_kernel<K>), dim3(grid), dim3(64), 0, s, items, qlen, partners,
                       colors, min_out, budget);
  });
  return hipGetLastError();
}

}  // namespace mpld
