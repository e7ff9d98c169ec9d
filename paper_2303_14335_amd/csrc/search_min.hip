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
#include "min_core.h"
#include "reg_items.h"
#include "wave_ops.h"

namespace mpld {

// Returns the branch-and-bound nodes of register-tier item `item`, negated
// when the budget stopped it; 0 when the incumbent costs nothing.
template <int K>
__device__ int32_t minimize_reg(const RegItems& items, int32_t item, const uint8_t* __restrict__ partners,
                                int8_t* __restrict__ colors_base, uint32_t budget) {
  return minimize_core<K>(item_desc(items, item), item_mask(items, item, __lane_id()), partners,
                          colors_base, budget);
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
