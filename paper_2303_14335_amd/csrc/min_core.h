// min_core.h - the Eq. 1 branch and bound of one register-tier component
// on one wavefront (the method is described in search_min.hip), shared by
// the batched minimisation kernel and the serving tick.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_types.h"
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

// Minimises the component of descriptor d (lane u holding u's neighbour
// mask in nb; partners[d.nbr_off + u] its stitch partner, 0xff none) from
// the incumbent colors at colors_base + d.out_off.  Returns the
// branch-and-bound nodes, negated when the budget stopped it; 0 when the
// incumbent costs nothing.  Writes the best coloring.
template <int K>
__device__ int32_t minimize_core(const DevDesc& d, const uint64_t nb,
                                 const uint8_t* __restrict__ partners,
                                 int8_t* __restrict__ colors_base, uint32_t budget) {
  const uint32_t lane = __lane_id();
  const uint32_t n = uniform((uint32_t)d.n);
  const bool in = lane < n;
  MinLane<K> L;
  L.nb = nb;
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

}  // namespace mpld
