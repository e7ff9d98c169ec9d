// search_reg.hip - register tier of the exact-cover search (components of at
// most 64 nodes), one 64-lane wavefront per component.
//
// Exact-cover matrix (Sec. 2.3): one row (v, c) per node and color, a
// primary column per node, a secondary column per (conflict edge, color).
// Row (v, c) stays in the matrix while v is uncovered and no conflict
// neighbour of v has taken row (u, c); so the rows of primary column v are
// the colors still open to v.  With at most 64 nodes the whole
// dancing-links state is a handful of 64-bit words, kept wave-uniform in
// scalar registers:
//   O[c] - color plane c: the nodes for which color c is still open;
//   P    - the uncovered primary columns.
// Column choice (Algorithm 1): the row count of column v is the number of
// planes holding v.  A column with no rows shows as an uncovered node
// missing from every plane (a dead end, chosen first).  Otherwise a
// bit-sliced adder over the planes gives the counts of all 64 columns at
// once as count-bit planes; narrowing P from the most significant count bit
// down keeps the columns of smallest count, and the lowest set bit is the
// lowest local index.
// Cover of row (v, c) (Eq. 2 "cover"): v's conflict neighbours lose color
// c, O[c] &= ~N(v), and column v leaves P.
// The recursion of Algorithm 1 is an explicit stack in VGPRs, lane d
// holding frame d: v | c << 8 and a snapshot of P and the planes from
// right before row (v, c) was taken.  Uncover (Eq. 2 "uncover") of all the
// rows above a frame is restoring that frame's snapshot, so a dead end
// jumps straight to the deepest frame whose column has untried rows (a
// uniform bit set of such depths) instead of popping frame by frame.
// The neighbour sets N(v) sit one per lane (lane v) and are read with
// v_readlane when v is chosen.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_types.h"
#include "min_core.h"
#include "mpld.h"
#include "reg_items.h"
#include "trace.h"
#include "wave_ops.h"

namespace mpld {

static constexpr uint32_t kNone = 0xffffffffu;

constexpr int bit_width(int x) { return x == 0 ? 0 : 1 + bit_width(x >> 1); }

// Search state of one component, K color planes (K >= k; planes k..K-1 stay
// empty).  Wave-uniform: the planes O, the uncovered set P, the set A of
// stack depths whose column still has untried rows, counters, depth, hash,
// entering row, status (-1 while the search runs or is paused).  Per lane
// d (the stack): the frame fr = v | c << 8 of depth d and a snapshot of the
// state right before its row was taken (P with v already covered, and the
// K planes), so that a dead end restores the deepest frame with untried
// rows in one step, whatever the number of frames above it.
template <int K>
using Planes = uint64_t __attribute__((ext_vector_type(K)));
template <int K>
using LaneWords = uint32_t __attribute__((ext_vector_type(K)));

template <int K>
struct RegState {
  Planes<K> O;
  uint64_t P, A, nodes, h;
  uint32_t depth, row_in;
  int32_t status;
  uint32_t fr, sp_lo, sp_hi;
  LaneWords<K> so_lo, so_hi;
  // stitch-aware order only: lane u holds u's stitch partner (bits 8..15,
  // 0xff none) and the color last given to that partner (bits 0..7, 0xff
  // none); it is the partner's current color while the partner is covered
  uint32_t pc;
};

template <int K>
__device__ __forceinline__ void reg_init(RegState<K>& s, int32_t n, int32_t k) {
  const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
#pragma unroll
  for (int c = 0; c < K; ++c) s.O[c] = c < k ? all : 0ull;
  s.P = all;
  s.A = 0;
  s.nodes = 0;
  s.h = 0;
  s.depth = 0;
  s.row_in = kNone;
  s.status = -1;
  s.fr = 0;
  s.sp_lo = 0;
  s.sp_hi = 0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    s.so_lo[c] = 0;
    s.so_hi[c] = 0;
  }
}

// c == j ? a : b on uniform 64-bit words (one compare, one 64-bit select).
// The 32-bit scalar operands of these inline-asm helpers go through
// readfirstlane: free for a value already in an SGPR, and it keeps a value
// the compiler's divergence analysis lost track of out of a VGPR operand.
__device__ __forceinline__ uint64_t sel_eq(uint32_t c, int j, uint64_t a, uint64_t b) {
  uint64_t r;
  asm("s_cmp_eq_u32 %1, %2\n\ts_cselect_b64 %0, %3, %4" : "=s"(r) : "s"(uniform(c)), "i"(j), "s"(a), "s"(b) : "scc");
  return r;
}

// Open colors of node v (the rows of column v), bit c for color c.
template <int K>
__device__ __forceinline__ uint32_t rows_of(const Planes<K>& O, uint32_t v) {
  uint32_t R = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    uint32_t b;
    asm("s_bitcmp1_b64 %1, %2\n\ts_cselect_b32 %0, %3, 0" : "=s"(b) : "s"(O[j]), "s"(uniform(v)), "i"(1 << j) : "scc");
    R |= b;
  }
  return R;
}

// Keeps the columns of `cand` whose count bit `bits` is clear, unless none
// is: one s_andn2 (which sets SCC to "result nonzero") and one 64-bit select.
__device__ __forceinline__ uint64_t narrow(uint64_t cand, uint64_t bits) {
  uint64_t r;
  asm("s_andn2_b64 %0, %1, %2\n\ts_cselect_b64 %0, %0, %1" : "=&s"(r) : "s"(cand), "s"(bits) : "scc");
  return r;
}

// Uncovered columns of the smallest row count (every column of P has at
// least one row).  ge2 receives the columns with two rows or more.  The row
// counts are added bit-sliced: cnt[b] holds bit b of every column's count.
template <int K>
__device__ __forceinline__ uint64_t min_count_columns(const Planes<K>& O, const uint64_t P,
                                                      uint64_t& ge2) {
  constexpr int NB = bit_width(K);
  uint64_t cnt[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) cnt[b] = 0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    // add plane c; afterwards a count is at most c + 1, so only
    // bit_width(c + 1) bits can change
    uint64_t carry = O[c];
#pragma unroll
    for (int b = 0; b < bit_width(c + 1); ++b) {
      const uint64_t t = cnt[b] & carry;
      cnt[b] ^= carry;
      carry = t;
    }
  }
  ge2 = 0;
#pragma unroll
  for (int b = 1; b < NB; ++b) ge2 |= cnt[b];
  uint64_t cand = P;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) cand = narrow(cand, cnt[b]);
  return cand;
}

// Lowest open color of node v (v has at least one): s_bitcmp1 tests bit v
// of a plane into SCC, s_cselect keeps the lower color.
template <int K>
__device__ __forceinline__ uint32_t first_color(const Planes<K>& O, const uint32_t v) {
  uint32_t c = K - 1;
#pragma unroll
  for (int j = K - 2; j >= 0; --j)
    asm("s_bitcmp1_b64 %1, %2\n\ts_cselect_b32 %0, %3, %0" : "+s"(c) : "s"(O[j]), "s"(uniform(v)), "i"(j) : "scc");
  return c;
}

// Cover of row (v, c) on the planes: v's neighbours lose color c.
template <int K>
__device__ __forceinline__ void cover(Planes<K>& O, const uint32_t c, const uint64_t nbv) {
#pragma unroll
  for (int j = 0; j < K; ++j) O[j] = sel_eq(c, j, O[j] & ~nbv, O[j]);
}

// Bits 0 .. d-1 (d <= 64).
__device__ __forceinline__ uint64_t below(uint32_t d) { return d >= 64u ? ~0ull : (1ull << d) - 1ull; }

// Sets bit d of A to `on` (0 or 1), without a branch: s_bitset0, then the
// bit ORed in.
__device__ __forceinline__ uint64_t with_bit(uint64_t A, uint32_t d, uint64_t on) {
  asm("s_bitset0_b64 %0, %1" : "+s"(A) : "s"(uniform(d)));
  return A | (on << d);
}

// Takes row (v, c) at the current depth (column v already removed from P):
// snapshot of P and the planes and the frame to lane `depth`, then the
// cover; `alt` says whether column v has rows after c.
template <int K, bool STITCH = false>
__device__ __forceinline__ void take_row(RegState<K>& s, const uint64_t nbv, const uint32_t v,
                                         const uint32_t c, const uint64_t alt,
                                         const uint32_t tried = 0) {
  const uint32_t d = s.depth;
  s.sp_lo = wrlane(s.sp_lo, d, (uint32_t)s.P);
  s.sp_hi = wrlane(s.sp_hi, d, (uint32_t)(s.P >> 32));
#pragma unroll
  for (int j = 0; j < K; ++j) {
    s.so_lo[j] = wrlane(s.so_lo[j], d, (uint32_t)s.O[j]);
    s.so_hi[j] = wrlane(s.so_hi[j], d, (uint32_t)(s.O[j] >> 32));
  }
  s.fr = wrlane(s.fr, d, STITCH ? (v | (c << 8) | (tried << 16)) : (v | (c << 8)));
  if (STITCH) s.pc = (s.pc >> 8) == v ? (s.pc & 0xff00u) | c : s.pc;   // v's partners see c
  cover(s.O, c, nbv);
  s.A = with_bit(s.A, d, alt);
  s.depth = d + 1;
}

// Dead end: returns to the deepest frame above `floor` whose column has
// untried rows and restores the state from before its row was taken (its
// snapshot; the frames above it are dropped, which undoes their rows and
// uncovers their columns).  Sets v, c to that column and its next row and
// `alt` to whether more rows follow (1 or 0); returns false when no such
// frame exists (the subtree below `floor` is exhausted).
template <int K, bool STITCH = false>
__device__ __forceinline__ bool retreat(RegState<K>& s, const uint32_t floor, uint32_t& v,
                                        uint32_t& c, uint64_t& alt, uint32_t& tried) {
  const uint64_t open = s.A & below(s.depth) & ~below(floor);
  if (open == 0) {   // exhausted: every frame above the floor is dropped
    s.depth = floor;
    return false;
  }
  const uint32_t d = 63u - (uint32_t)__builtin_clzll(open);
  const uint32_t f = rdlane(s.fr, d);
  s.P = rdlane64(s.sp_lo, s.sp_hi, d);
#pragma unroll
  for (int j = 0; j < K; ++j) s.O[j] = rdlane64(s.so_lo[j], s.so_hi[j], d);
  v = f & 0xffu;
  const uint32_t R = rows_of(s.O, v);   // the rows of v when it was chosen
  // rows not tried yet: above the last one in ascending order; with the
  // stitch-aware order the frame keeps the set tried (bits 16..23)
  const uint32_t next = STITCH ? R & ~(f >> 16) : R & (0xfffffffeu << (f >> 8));
  c = (uint32_t)__builtin_ctz(next);
  alt = (next & (next - 1u)) != 0 ? 1ull : 0ull;
  if (STITCH) tried = (f >> 16) | (1u << c);
  s.depth = d;
  return true;
}

// Runs the search until it ends or `nodes` reaches stop_at (<= budget); a
// stop short of the budget leaves status -1 and the state resumable at a
// node boundary.  With floor > 0 the search is confined to the subtree of
// the node at depth `floor` (backtracking never returns above it;
// exhausting the subtree reports MPLD_INFEASIBLE).  nb_lo/nb_hi: lane v
// holds N(v).  Every lane of the wave must call it.
template <bool TRACE, int K, bool STITCH = false>
__device__ __forceinline__ void reg_run(RegState<K>& s, const uint32_t nb_lo, const uint32_t nb_hi,
                                        const int32_t k, const uint64_t budget,
                                        const uint64_t stop_at, const uint32_t floor = 0) {
  int32_t status;
  for (;;) {
    // ---- one search node
    if (__builtin_expect(s.nodes == stop_at, 0)) {
      // paused short of the budget (resumable here), or out of budget
      status = s.nodes != budget ? -1 : MPLD_BUDGET_EXHAUSTED;
      break;
    }
    ++s.nodes;
    if (__builtin_expect(s.P == 0, 0)) {
      if (TRACE) s.h = trace_node(s.h, s.depth, s.row_in, kNone, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    uint64_t any = s.O[0];
#pragma unroll
    for (int j = 1; j < K; ++j) any |= s.O[j];
    const uint64_t zero = s.P & ~any;
    uint32_t v, c, tried = 0;
    uint64_t alt;
    if (__builtin_expect(zero == 0, 1)) {
      // every uncovered column has rows: cover the one of fewest rows and
      // take its first row
      uint64_t ge2;
      v = low_bit(min_count_columns(s.O, s.P, ge2));
      if (TRACE) s.h = trace_node(s.h, s.depth, s.row_in, v, (uint32_t)__popc(rows_of(s.O, v)));
      c = first_color(s.O, v);
      alt = (ge2 >> v) & 1ull;
      if (STITCH) {
        // stitch-aware order: the color of v's stitch partner first, when
        // the partner is on the path (covered) and that row is still open
        const uint32_t R = rows_of(s.O, v);
        tried = R & ((2u << c) - 1u);
        // v's partner and the color it was last given, from v's lane
        const uint32_t x = uniform(rdlane(s.pc, v));
        const uint32_t p = x >> 8, cp = x & 0x1fu;
        const bool use = p < 64u && !((s.P >> (p & 63u)) & 1ull) && ((R >> cp) & 1u);
        c = uniform(use ? cp : c);
        tried = uniform(use ? 1u << cp : tried);
      }
      asm("s_bitset0_b64 %0, %1" : "+s"(s.P) : "s"(uniform(v)));   // cover column v
    } else {
      // a column without rows (the first by index is the one chosen): dead end
      if (TRACE) s.h = trace_node(s.h, s.depth, s.row_in, low_bit(zero), 0);
      if (!retreat<K, STITCH>(s, floor, v, c, alt, tried)) {
        status = MPLD_INFEASIBLE;
        break;
      }
    }
    // ---- include row (v, c)
    take_row<K, STITCH>(s, rdlane64(nb_lo, nb_hi, v), v, c, alt, tried);
    s.row_in = v * (uint32_t)k + c;
  }
  s.status = status;
}

// Writes the colors (the chosen row of every column on a solution, -1
// otherwise) and the record of a finished search.
template <int K>
__device__ __forceinline__ void reg_finish(const RegState<K>& s, int32_t n,
                                           int8_t* __restrict__ colors,
                                           DevRecord* __restrict__ rec) {
  const uint32_t lane = __lane_id();
  const uint32_t depth = uniform(s.depth);
  if (s.status == MPLD_FEASIBLE) {
    if (lane < depth && (s.fr & 0xffu) < (uint32_t)n)
      colors[s.fr & 0xffu] = (int8_t)((s.fr >> 8) & 0xffu);
  } else if (lane < (uint32_t)n) {
    colors[lane] = -1;
  }
  // Every lane stores the same (uniform) record: no branch here may share
  // the queue pop's "lane 0" condition, or the compiler can thread the two
  // across the loop back-edge and split the wave at the pop.
  rec->status = s.status;
  rec->depth = s.status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
  rec->nodes = s.nodes;
  rec->hash = s.h;
}

// Conflict marking (Algorithm 1: a column left with no related row is a
// conflict candidate (cl, cl'), cl' the column whose cover removed cl's
// final row) for a component whose search ended without a solution: one
// descent of the search that never backtracks.  The column is chosen by the
// search's rule (fewest rows, lowest index) and takes its lowest open color;
// a column with no row left takes the color of the row it lost last, which
// conflicts with the neighbour that took that color.  Lane u holds N(u) and
// the color u lost last; the planes are wave-uniform.  Every node is colored.
template <int K>
__device__ __forceinline__ void mark_core(uint32_t n, const uint64_t nb, int8_t* __restrict__ colors) {
  const uint32_t lane = __lane_id();
  n = uniform(n);
  uint64_t P = n >= 64u ? ~0ull : ((1ull << n) - 1ull);
  uint64_t O[K];
#pragma unroll
  for (int c = 0; c < K; ++c) O[c] = P;
  uint32_t last = 0, color = 0;
  while (P != 0ull) {
    uint32_t cnt = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) cnt += (uint32_t)((O[c] >> lane) & 1ull);
    const uint32_t key = wave_min_u32(((P >> lane) & 1ull) ? (cnt << 8) | lane : ~0u);
    const uint32_t v = key & 0xffu;
    uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)last, (int)v);
    if ((key >> 8) != 0u) {   // lowest open color of v
      c = K - 1;
#pragma unroll
      for (int j = K - 2; j >= 0; --j)
        if ((O[j] >> v) & 1ull) c = (uint32_t)j;
    }
    c = uniform(c);
    P &= ~(1ull << v);
    if (lane == v) color = c;
    const uint64_t nv = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(nb >> 32), (int)v) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)nb, (int)v);
    uint64_t removed = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((uint32_t)j == c) {
        removed = nv & O[j];
        O[j] &= ~nv;
      }
    if ((removed >> lane) & 1ull) last = c;
  }
  if (lane < n) colors[lane] = (int8_t)color;
}

// Solves one register-tier item.  The descriptor (scalar loads) and the
// lane's neighbour mask (a vector load) come from one record, so both
// loads are in flight together.  cap < budget stops the search after `cap`
// nodes (status -1 in the record: the component is left to the
// heavy-component engine).
template <bool TRACE, int K, bool STITCH = false>
__device__ __forceinline__ void solve_reg(const RegItems& items, int32_t item,
                                          int8_t* __restrict__ colors_base,
                                          DevRecord* __restrict__ recs,
                                          const uint64_t cap = ~0ull, const uint32_t mark = 0u) {
  const uint32_t lane = __lane_id();
  const uint64_t nb = item_mask(items, item, lane);
  const DevDesc d = item_desc(items, item);
  const uint64_t budget = (uint64_t)d.budget;
  RegState<K> s;
  reg_init(s, d.n, d.k);
  if (STITCH) s.pc = (item_partner(items, item, lane) << 8) | 0xffu;
  reg_run<TRACE, K, STITCH>(s, (uint32_t)nb, (uint32_t)(nb >> 32), d.k, budget,
                            cap < budget ? cap : budget, 0);
  reg_finish(s, d.n, colors_base + d.out_off, recs + d.comp);
  // mark: a search that ended without a solution is colored by the conflict
  // marking right away, by the same wave (lane u rewrites color u)
  if (mark && s.status != MPLD_FEASIBLE && s.status >= 0)
    mark_core<K>((uint32_t)d.n, nb, colors_base + d.out_off);
}

// Root split for the heaviest items (no cap): one
// workgroup of four waves per item.  At the root every column has all k
// rows, so the root column v0 is node 0 and its rows are the k colors.
// Wave 0 (the owner) counts the root node and searches the subtree of row
// 0; wave c = 1 .. min(k, 4) - 1 (a helper) searches the subtree of row c
// from the same start, in chunks of `chunk` nodes with a check of the
// owner's release between them, and publishes its node count, status,
// trace hash of its own nodes and solution in LDS.  The owner takes the rows
// in order: for a helper's row it waits for the helper and adds its count
// and appends its trace hash (an exhausted subtree: next row; a solution:
// done), exactly as the sequential search would have counted and hashed
// them; a helper that ran into the budget, or whose count would cross it,
// is searched again by the owner.  The owner releases the helpers it no
// longer needs.  Status, node count, trace hash, depth and colors equal the
// sequential search's.
struct RootSplitLds {
  uint32_t flag[4], stop[4];
  uint64_t nodes[4], hash[4];
  int32_t status[4], depth[4];
  int8_t colors[4][64];
};

template <bool TRACE, int K, bool STITCH>
__device__ __forceinline__ void root_split(const RegItems& items, int32_t item, uint32_t wave,
                                           uint32_t chunk, int8_t* __restrict__ colors_base,
                                           DevRecord* __restrict__ recs, const uint32_t mark = 0u) {
  __shared__ RootSplitLds L;
  const uint32_t lane = __lane_id();
  constexpr uint32_t kHelpers = (K < 4 ? K : 4) - 1;
  if (wave == 0u && lane < 4u) {
    L.flag[lane] = 0u;
    L.stop[lane] = 0u;
  }
  __syncthreads();
  const DevDesc d = item_desc(items, item);
  const uint64_t nb = item_mask(items, item, lane);
  const uint32_t nb_lo = (uint32_t)nb, nb_hi = (uint32_t)(nb >> 32);
  const uint64_t budget = (uint64_t)d.budget;
  RegState<K> s;
  reg_init(s, d.n, d.k);
  if (STITCH) s.pc = (item_partner(items, item, lane) << 8) | 0xffu;
  if (wave > kHelpers) return;
  if (s.P == 0ull) {   // empty component: the root is a solution
    if (wave == 0u) {
      reg_run<TRACE, K>(s, nb_lo, nb_hi, d.k, budget, budget);
      reg_finish(s, d.n, colors_base + d.out_off, recs + d.comp);
    }
    return;
  }
  // the root column and its rows without counting: every column has all
  // k rows, so the fewest-rows, lowest-index column is node 0
  constexpr uint32_t v0 = 0u;
  const uint32_t R0 = uniform((1u << (uint32_t)d.k) - 1u);
  s.P &= ~(1ull << v0);
  const uint64_t nbv0 = rdlane64(nb_lo, nb_hi, v0);
  if (wave != 0u) {
    // ---- helper: the subtree of root row c
    const uint32_t c = wave;
    if (!((R0 >> c) & 1u)) return;   // the owner never asks for a missing row
    take_row<K, STITCH>(s, nbv0, v0, c, 0ull, R0 & ((2u << c) - 1u));
    s.row_in = v0 * (uint32_t)d.k + c;
    for (;;) {
      reg_run<TRACE, K, STITCH>(s, nb_lo, nb_hi, d.k, ~0ull, s.nodes + chunk, 1);
      if (s.status >= 0) break;
      if (__hip_atomic_load(&L.stop[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u)
        return;   // no longer needed
      if (s.nodes >= budget) {   // the owner re-searches it under its budget
        s.status = -2;
        break;
      }
    }
    const uint32_t depth = uniform(s.depth);
    if (s.status == MPLD_FEASIBLE && lane < depth) L.colors[c][s.fr & 0xffu] = (int8_t)(s.fr >> 8);
    if (lane == 63u) {
      L.status[c] = s.status;
      L.nodes[c] = s.nodes;
      L.hash[c] = s.h;   // the subtree's own trace hash (from 0)
      L.depth[c] = (int32_t)depth;
    }
    __hip_atomic_store(&L.flag[c], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    return;
  }
  // ---- owner: the root node, then the root rows in order; with the trace
  // hash, a helper's subtree hash is appended to the owner's
  ++s.nodes;
  if (TRACE) s.h = trace_node(s.h, 0u, kNone, v0, (uint32_t)__popc(R0));
  const Planes<K> O0 = s.O;
  const uint64_t P0 = s.P;
  int32_t taken = -1;   // helper whose solution ends the search
  int32_t status = MPLD_INFEASIBLE;
  uint32_t rem = R0;
  while (rem != 0u) {
    const uint32_t c = uniform((uint32_t)__builtin_ctz(rem));
    rem &= rem - 1u;
    if (c >= 1u && c <= kHelpers) {
      while (__hip_atomic_load(&L.flag[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u)
        __builtin_amdgcn_s_sleep(1);
      const int32_t hs = (int32_t)uniform((uint32_t)L.status[c]);
      const uint64_t hn = uniform64(L.nodes[c]);
      if (hs >= 0 && s.nodes + hn <= budget) {
        s.nodes += hn;
        if (TRACE) s.h = trace_concat(s.h, uniform64(L.hash[c]), hn);
        if (hs == MPLD_FEASIBLE) {
          status = MPLD_FEASIBLE;
          taken = (int32_t)c;
          break;
        }
        continue;   // the subtree is exhausted: next row
      }
    }
    s.O = O0;
    s.P = P0;
    s.depth = 0;
    take_row<K, STITCH>(s, nbv0, v0, c, rem != 0u ? 1ull : 0ull, R0 & ((2u << c) - 1u));
    s.row_in = v0 * (uint32_t)d.k + c;
    reg_run<TRACE, K, STITCH>(s, nb_lo, nb_hi, d.k, budget, budget, 1);
    if (s.status != MPLD_INFEASIBLE) {
      status = s.status;
      break;
    }
  }
  if (lane < 4u) __hip_atomic_store(&L.stop[lane], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  int8_t* colors = colors_base + d.out_off;
  DevRecord* rec = recs + d.comp;
  if (taken >= 0) {
    if (lane < (uint32_t)d.n) colors[lane] = L.colors[taken][lane];
    rec->status = MPLD_FEASIBLE;
    rec->depth = (int32_t)uniform((uint32_t)L.depth[taken]);
    rec->nodes = s.nodes;
    rec->hash = s.h;
    return;
  }
  s.status = status;
  reg_finish(s, d.n, colors, rec);
  if (mark && status != MPLD_FEASIBLE) mark_core<K>((uint32_t)d.n, nb, colors);
}

// Resumable state in device memory (kRegStateBytes per component): the
// uniform head (counters at 0, planes at 64), then 64-lane arrays of u32:
// frames, P snapshot (low, high), then per plane its snapshot (low, high).
struct RegStateHead {
  uint64_t P, A, nodes, h;
  uint32_t depth, row_in;
};
static_assert(sizeof(RegStateHead) == 40, "state head is 40 bytes");
static_assert(kRegStateBytes >= 128 + 256 * (3 + 2 * 8 + 1), "state layout");
constexpr uint32_t kStatePcLane = (3 + 2 * 8) * 64;   // u32 index of the partner registers

template <int K, bool STITCH = false>
__device__ __forceinline__ void reg_save(const RegState<K>& s, uint8_t* base) {
  const uint32_t lane = __lane_id();
  RegStateHead* hd = reinterpret_cast<RegStateHead*>(base);
  hd->P = s.P;   // same value from every lane
  hd->A = s.A;
  hd->nodes = s.nodes;
  hd->h = s.h;
  hd->depth = s.depth;
  hd->row_in = s.row_in;
  uint64_t* planes = reinterpret_cast<uint64_t*>(base + 64);
#pragma unroll
  for (int c = 0; c < K; ++c) planes[c] = s.O[c];
  uint32_t* lanes = reinterpret_cast<uint32_t*>(base + 128);
  lanes[lane] = s.fr;
  lanes[64 + lane] = s.sp_lo;
  lanes[128 + lane] = s.sp_hi;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    lanes[(3 + 2 * c) * 64 + lane] = s.so_lo[c];
    lanes[(4 + 2 * c) * 64 + lane] = s.so_hi[c];
  }
  if (STITCH) lanes[kStatePcLane + lane] = s.pc;
}

template <int K, bool STITCH = false>
__device__ __forceinline__ void reg_load(RegState<K>& s, const uint8_t* base) {
  const uint32_t lane = __lane_id();
  const RegStateHead* hd = reinterpret_cast<const RegStateHead*>(base);
  s.P = uniform64(hd->P);
  s.A = uniform64(hd->A);
  s.nodes = uniform64(hd->nodes);
  s.h = uniform64(hd->h);
  s.depth = uniform(hd->depth);
  s.row_in = uniform(hd->row_in);
  const uint64_t* planes = reinterpret_cast<const uint64_t*>(base + 64);
#pragma unroll
  for (int c = 0; c < K; ++c) s.O[c] = uniform64(planes[c]);
  const uint32_t* lanes = reinterpret_cast<const uint32_t*>(base + 128);
  s.fr = lanes[lane];
  s.sp_lo = lanes[64 + lane];
  s.sp_hi = lanes[128 + lane];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    s.so_lo[c] = lanes[(3 + 2 * c) * 64 + lane];
    s.so_hi[c] = lanes[(4 + 2 * c) * 64 + lane];
  }
  if (STITCH) s.pc = lanes[kStatePcLane + lane];
  s.status = -1;
}

// The hardware deals workgroups to the eight XCDs round-robin (block b to
// XCD b % 8), and each XCD has its own L2.  Neighbouring items' descriptors
// and masks share cache lines, so blocks are renumbered to give each XCD one
// contiguous range of items (a bijection on 0 .. gridDim.x - 1).
__device__ __forceinline__ uint32_t xcd_block() {
  constexpr uint32_t kXcds = 8;
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t x = b % kXcds, i = b / kXcds, q = G / kXcds, r = G % kXcds;
  return x * q + (x < r ? x : r) + i;
}

// Persistent batched kernel.  Wave w first takes item w of its tier's
// descriptor list (no atomic); while the grid has fewer waves than items,
// waves then pop item gw + atomicAdd(counter, 1).  Every wave fails exactly
// one pop, so the pop that returns qlen - 1 is the last one: it resets the
// counter to 0 and the launch (or the graph holding it) can be replayed with
// no memset.
template <bool TRACE, int K, bool STITCH>
__global__ __launch_bounds__(256) void reg_batched_kernel(
    const RegItems items, int32_t qlen, int32_t* __restrict__ counter,
    DevRecord* __restrict__ recs, int8_t* __restrict__ colors, uint64_t cap, int32_t heavy,
    uint32_t chunk, uint32_t mark) {
  const uint32_t wpb = blockDim.x >> 6;   // waves per workgroup
  if (heavy > 0) {
    // root split: workgroups 0 .. heavy-1 take items 0 .. heavy-1 (four
    // waves each), the rest one item per wave; the host sized the grid so
    // that every item is handed out here
    const uint32_t b = xcd_block(), wave = uniform(threadIdx.x >> 6);
    if (b < (uint32_t)heavy) {
      root_split<TRACE, K, STITCH>(items, (int32_t)b, wave, uniform(chunk), colors, recs,
                                   uniform(mark));
    } else {
      const int32_t item = heavy + (int32_t)((b - (uint32_t)heavy) * wpb + wave);
      if (item < qlen) solve_reg<TRACE, K, STITCH>(items, item, colors, recs, cap, uniform(mark));
    }
    return;
  }
  const int32_t gw = (int32_t)(gridDim.x * wpb);
  int32_t item = (int32_t)uniform(xcd_block() * wpb + (threadIdx.x >> 6));
  while (item < qlen) {
    solve_reg<TRACE, K, STITCH>(items, item, colors, recs, cap, uniform(mark));
    if (gw >= qlen) break;   // every item was handed out statically
    int32_t r = 0;
    if (__lane_id() == 0) r = atomicAdd(counter, 1);
    r = (int32_t)uniform((uint32_t)r);
    item = gw + r;
    if (r == qlen - 1) atomicExch(counter, 0);   // the last pop of this launch
  }
}

// One component per launch (the plain solver): a single wave.
template <bool TRACE, int K, bool STITCH>
__global__ __launch_bounds__(64) void reg_single_kernel(const RegItems items,
                                                        int32_t item, DevRecord* __restrict__ recs,
                                                        int8_t* __restrict__ colors) {
  solve_reg<TRACE, K, STITCH>(items, item, colors, recs);
}

template <int K>
__device__ __forceinline__ void mark_reg(const RegItems& items, int32_t item,
                                         int8_t* __restrict__ colors_base) {
  const DevDesc d = item_desc(items, item);
  mark_core<K>((uint32_t)d.n, item_mask(items, item, __lane_id()), colors_base + d.out_off);
}

// One wave per workgroup over the register-tier items; components whose
// record is FEASIBLE keep the search's colors.
template <int K>
__global__ __launch_bounds__(64) void mark_reg_kernel(const RegItems items, int32_t qlen,
                                                      const DevRecord* __restrict__ recs,
                                                      int8_t* __restrict__ colors) {
  for (int32_t i = (int32_t)uniform(blockIdx.x); i < qlen; i += (int32_t)gridDim.x) {
    const int32_t comp = (int32_t)uniform((uint32_t)item_desc(items, i).comp);
    if ((int32_t)uniform((uint32_t)recs[comp].status) == MPLD_FEASIBLE) continue;
    mark_reg<K>(items, i, colors);
  }
}

// Serving tick: every listed component advances by at most `slice` search
// nodes from its saved state (entries with bit 31 set start fresh; bit 30:
// a component left without a solution is then colored by the conflict
// marking; bit 29: the finished component's colors are then minimised for
// Eq. 1 with a budget of slot_minb[slot] nodes, the count going to
// slot_min[slot] as for the batched minimisation).  A finished search writes its colors and record; a paused one
// saves its state.  tick_out[i] receives the record of list entry i (status -1 while
// the search is still running).  Work distribution as in the batched kernel.
// STITCH: the stitch-aware row order; part8[w] is the stitch partner (local
// id, 0xff none) of the node whose neighbour mask is arena64[w], and the
// lanes' partner registers are part of the saved state.
template <bool TRACE, int K, bool STITCH>
__global__ __launch_bounds__(256) void reg_tick_kernel(
    const int32_t* __restrict__ list, int32_t len, int32_t* __restrict__ counter,
    const DevDesc* __restrict__ slot_desc, uint8_t* slot_state, DevRecord* __restrict__ slot_rec,
    const uint64_t* __restrict__ arena64, int8_t* __restrict__ arena8,
    const uint8_t* __restrict__ part8, const uint32_t* __restrict__ slot_minb,
    int32_t* __restrict__ slot_min, uint64_t slice, DevRecord* __restrict__ tick_out) {
  const int32_t gw = (int32_t)gridDim.x * 4;
  int32_t item = (int32_t)uniform(xcd_block() * 4u + (threadIdx.x >> 6));
  while (item < len) {
    const uint32_t entry = uniform((uint32_t)list[item]);
    const int32_t slot = (int32_t)(entry & 0x1fffffffu);
    const DevDesc d = slot_desc[slot];
    const uint32_t lane = __lane_id();
    const uint64_t nb = lane < (uint32_t)d.n ? arena64[d.nbr_off + lane] : 0ull;
    uint8_t* base = slot_state + (uint64_t)slot * kRegStateBytes;
    RegState<K> s;
    if (entry >> 31) {
      reg_init(s, d.n, d.k);
      if (STITCH) s.pc = ((lane < (uint32_t)d.n ? (uint32_t)part8[d.nbr_off + lane] : 0xffu) << 8) | 0xffu;
    } else {
      reg_load<K, STITCH>(s, base);
    }
    const uint64_t budget = (uint64_t)d.budget;
    const uint64_t stop = budget - s.nodes > slice ? s.nodes + slice : budget;
    reg_run<TRACE, K, STITCH>(s, (uint32_t)nb, (uint32_t)(nb >> 32), d.k, budget, stop);
    if (s.status >= 0) {
      reg_finish(s, d.n, arena8 + d.out_off, slot_rec + slot);
      // conflict marking of a component left without a solution (the
      // wave's own stores, so they follow reg_finish's)
      if (((entry >> 30) & 1u) && s.status != MPLD_FEASIBLE)
        mark_core<K>((uint32_t)d.n, nb, arena8 + d.out_off);
      if ((entry >> 29) & 1u) {
        // the minimisation reads the colors this wave just stored
        __builtin_amdgcn_s_waitcnt(0);
        const int32_t mr = minimize_core<K>(d, nb, part8, arena8, slot_minb[slot]);
        slot_min[slot] = mr;   // the same value from every lane
      }
    } else {
      reg_save<K, STITCH>(s, base);
    }
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

// Stitch-aware order at a forward step on column v (the sequential
// search's rule): when v's stitch partner is on the path (covered) and the
// row of the partner's color is open, that row goes first, the rest follow
// ascending.  In: c = v's lowest open row.  Out: the row to take and the set
// of rows tried once it is taken.
template <int K>
__device__ __forceinline__ void stitch_pick(const RegState<K>& s, const uint32_t v, uint32_t& c,
                                            uint32_t& tried) {
  const uint32_t R = rows_of(s.O, v);
  tried = R & ((2u << c) - 1u);
  const uint32_t x = uniform(rdlane(s.pc, v));
  const uint32_t p = x >> 8, cp = x & 0x1fu;
  const bool use = p < 64u && !((s.P >> (p & 63u)) & 1ull) && ((R >> cp) & 1u);
  c = uniform(use ? cp : c);
  tried = uniform(use ? 1u << cp : tried);
}

// Rebuilds the search state at the end of a path of rows from the root:
// cover each row's column and take the row, in order (the same steps the
// sequential search made on the way down, so planes, snapshots and the
// untried-rows set match).  With the stitch-aware order the row order at
// each step is rebuilt the same way (partner colors come from the rows
// already replayed), and the frame's tried set is every row up to the
// path's row in that order.
template <int K, bool STITCH = false>
__device__ __forceinline__ void reg_replay(RegState<K>& s, const uint32_t nb_lo,
                                           const uint32_t nb_hi, const int32_t k,
                                           const uint16_t* __restrict__ rows, uint32_t d) {
  for (uint32_t j = 0; j < d; ++j) {
    const uint32_t vc = uniform(rows[j]);
    const uint32_t v = vc & 0xffu, c = vc >> 8;
    const uint32_t R = rows_of(s.O, v);
    uint32_t tried = 0;
    uint64_t alt;
    if (STITCH) {
      uint32_t first = (uint32_t)__builtin_ctz(R), t0 = 0;
      stitch_pick(s, v, first, t0);   // first = the row this node tries first
      tried = c == first ? t0 : ((R & ((2u << c) - 1u)) | (1u << first));
      alt = (R & ~tried) != 0 ? 1ull : 0ull;
    } else {
      alt = (R & (0xfffffffeu << c)) != 0 ? 1ull : 0ull;
    }
    s.P &= ~(1ull << v);
    take_row<K, STITCH>(s, rdlane64(nb_lo, nb_hi, v), v, c, alt, tried);
    s.row_in = v * (uint32_t)k + c;
  }
}

// Enumerates the top `levels` levels of the subtree rooted at depth d in
// search order: counts their nodes, and emits a kind-0 item for every node
// at depth d + levels (not counted here: its own task counts it), a kind-2
// item when a solution is met (writing its colors) or a kind-1 item at the
// end.  Returns the number of items; with out == nullptr it only counts.
template <int K>
__device__ __forceinline__ int32_t reg_enumerate(RegState<K>& s, const uint32_t nb_lo,
                                                 const uint32_t nb_hi, const int32_t n,
                                                 const uint32_t d, const uint32_t levels,
                                                 SplitItem* __restrict__ out,
                                                 int8_t* __restrict__ sol) {
  const uint32_t lane = __lane_id();
  const uint32_t limit = d + levels;
  uint32_t seg = 0;
  int32_t items = 0;
  auto emit = [&](uint32_t kind) {
    const uint32_t r0 = kind == 0 ? rdlane(s.fr, d) : 0u;
    const uint32_t r1 = kind == 0 && levels > 1 ? rdlane(s.fr, d + 1) : 0u;
    const uint32_t r2 = kind == 0 && levels > 2 ? rdlane(s.fr, d + 2) : 0u;
    const uint32_t r3 = kind == 0 && levels > 3 ? rdlane(s.fr, d + 3) : 0u;
    if (out != nullptr && lane == ((uint32_t)items & 63u)) {   // one owner lane per item
      SplitItem it;
      it.seg = seg;
      it.kind = kind;
      it.rows[0] = (uint16_t)(r0 & 0xffffu);
      it.rows[1] = (uint16_t)(r1 & 0xffffu);
      it.rows[2] = (uint16_t)(r2 & 0xffffu);
      it.rows[3] = (uint16_t)(r3 & 0xffffu);
      out[items] = it;
    }
    ++items;
    seg = 0;
  };
  for (;;) {
    uint32_t v = 0, c = 0;
    uint64_t alt = 0;
    bool back;
    if (s.depth == limit) {
      emit(0);        // a subtask root: leave it to its own task
      back = true;
    } else {
      ++seg;
      if (s.P == 0) {   // a solution among the top levels
        if (lane < s.depth && (s.fr & 0xffu) < (uint32_t)n)
          sol[s.fr & 0xffu] = (int8_t)((s.fr >> 8) & 0xffu);
        emit(2);
        break;
      }
      uint64_t any = s.O[0];
#pragma unroll
      for (int j = 1; j < K; ++j) any |= s.O[j];
      back = (s.P & ~any) != 0;
      if (!back) {
        uint64_t ge2;
        v = low_bit(min_count_columns(s.O, s.P, ge2));
        c = first_color(s.O, v);
        alt = (ge2 >> v) & 1ull;
        s.P &= ~(1ull << v);
      }
    }
    uint32_t tried_unused = 0;
    if (back && !retreat(s, d, v, c, alt, tried_unused)) {
      emit(1);
      break;
    }
    take_row(s, rdlane64(nb_lo, nb_hi, v), v, c, alt);
  }
  return items;
}

// One wave per task: explore the task's subtree up to `cap` nodes; if the
// cap is hit, split the task `levels` levels down instead.
template <int K>
__global__ __launch_bounds__(256) void reg_split_kernel(
    const SplitTask* __restrict__ tasks, int32_t ntasks, int32_t* __restrict__ counter,
    const RegItems regitems, uint64_t cap,
    uint32_t levels, uint8_t* __restrict__ out, SplitItem* __restrict__ pool,
    int32_t* __restrict__ pool_count) {
  const uint32_t wpb = blockDim.x >> 6;
  const int32_t gw = (int32_t)(gridDim.x * wpb);
  int32_t t = (int32_t)uniform(xcd_block() * wpb + (threadIdx.x >> 6));
  const uint32_t lane = __lane_id();
  while (t < ntasks) {
    const SplitTask* task = tasks + t;
    const int32_t it = (int32_t)uniform((uint32_t)task->item);
    const uint32_t d = uniform((uint32_t)task->depth);
    const DevDesc dd = item_desc(regitems, it);
    const uint64_t nb = item_mask(regitems, it, lane);
    const uint32_t nb_lo = (uint32_t)nb, nb_hi = (uint32_t)(nb >> 32);
    uint8_t* block = out + (uint64_t)t * kSplitBlockBytes;
    int8_t* sol = reinterpret_cast<int8_t*>(block + kSplitSolOffset);
    RegState<K> s;
    reg_init(s, dd.n, dd.k);
    reg_replay(s, nb_lo, nb_hi, dd.k, task->rows, d);
    reg_run<false, K>(s, nb_lo, nb_hi, dd.k, ~0ull, cap, d);
    int32_t nitems = 0;
    uint32_t item_off = 0;
    if (s.status == MPLD_FEASIBLE) {
      if (lane < s.depth && (s.fr & 0xffu) < (uint32_t)dd.n)
        sol[s.fr & 0xffu] = (int8_t)((s.fr >> 8) & 0xffu);
    } else if (s.status < 0) {
      // count the split's items, reserve their range of the pool, then
      // enumerate again writing them (the top levels are cheap to walk)
      RegState<K> r;
      reg_init(r, dd.n, dd.k);
      reg_replay(r, nb_lo, nb_hi, dd.k, task->rows, d);
      nitems = reg_enumerate(r, nb_lo, nb_hi, dd.n, d, levels, nullptr, sol);
      // lane 63 takes the reservation: a lane-0 branch here could be merged
      // with the queue pop's and split the wave across the loop
      uint32_t o = 0;
      if (lane == 63u) o = (uint32_t)atomicAdd(pool_count, nitems);
      item_off = (uint32_t)__builtin_amdgcn_readlane((int)o, 63);
      reg_init(r, dd.n, dd.k);
      reg_replay(r, nb_lo, nb_hi, dd.k, task->rows, d);
      reg_enumerate(r, nb_lo, nb_hi, dd.n, d, levels, pool + item_off, sol);
    }
    SplitResult res;
    res.status = s.status;
    res.nitems = nitems;
    res.nodes = s.nodes;
    res.item_off = item_off;
    res.pad = 0;
    res.hash = 0;
    *reinterpret_cast<SplitResult*>(block) = res;   // same value from every lane
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

// Calls f(std::integral_constant<int, K>) with K = k color planes.
template <class F>
static void with_planes(int k, F&& f) {
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

hipError_t launch_reg_batched(bool trace, int k, int grid, int wpb, RegItems items,
                              int32_t qlen, int32_t* counter, DevRecord* recs, int8_t* colors,
                              uint64_t cap, int32_t heavy, uint32_t chunk, bool mark, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  if (wpb < 1 || wpb > 4) return hipErrorInvalidValue;
  // the root split needs four waves per workgroup and a grid that hands
  // out every item at once
  if (heavy < 0 || heavy > qlen || chunk < 1) return hipErrorInvalidValue;
  if (mark && cap != ~0ull) return hipErrorInvalidValue;   // capped records are not final
  const uint32_t mk = mark ? 1u : 0u;
  if (heavy > 0 && (wpb != 4 || cap != ~0ull ||
                    (int64_t)grid < heavy + ((int64_t)qlen - heavy + wpb - 1) / wpb))
    return hipErrorInvalidValue;
  const bool stitch = items.part_off != 0;   // the items carry stitch partners
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    // every item split: one workgroup per item and one wave per root row
    // (three for k = 3), so that no idle fourth wave is dispatched
    const int wg_waves = heavy == qlen ? (k < 4 ? k : 4) : wpb;
    const dim3 g(grid), b(64 * wg_waves);
    if (trace && stitch)
      hipLaunchKernelGGL((reg_batched_kernel<true, K, true>), g, b, 0, s, items, qlen, counter, recs,
                         colors, cap, heavy, chunk, mk);
    else if (trace)
      hipLaunchKernelGGL((reg_batched_kernel<true, K, false>), g, b, 0, s, items, qlen, counter,
                         recs, colors, cap, heavy, chunk, mk);
    else if (stitch)
      hipLaunchKernelGGL((reg_batched_kernel<false, K, true>), g, b, 0, s, items, qlen, counter,
                         recs, colors, cap, heavy, chunk, mk);
    else
      hipLaunchKernelGGL((reg_batched_kernel<false, K, false>), g, b, 0, s, items, qlen, counter,
                         recs, colors, cap, heavy, chunk, mk);
  });
  return hipGetLastError();
}

hipError_t launch_mark_reg(int k, int grid, RegItems items, int32_t qlen, const DevRecord* recs,
                           int8_t* colors, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    hipLaunchKernelGGL((mark_reg_kernel<K>), dim3(grid), dim3(64), 0, s, items, qlen, recs, colors);
  });
  return hipGetLastError();
}

hipError_t launch_reg_single(bool trace, int k, RegItems items, int32_t item,
                             DevRecord* recs, int8_t* colors, hipStream_t s) {
  const bool stitch = items.part_off != 0;
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    if (trace && stitch)
      hipLaunchKernelGGL((reg_single_kernel<true, K, true>), dim3(1), dim3(64), 0, s, items, item,
                         recs, colors);
    else if (trace)
      hipLaunchKernelGGL((reg_single_kernel<true, K, false>), dim3(1), dim3(64), 0, s, items, item,
                         recs, colors);
    else if (stitch)
      hipLaunchKernelGGL((reg_single_kernel<false, K, true>), dim3(1), dim3(64), 0, s, items, item,
                         recs, colors);
    else
      hipLaunchKernelGGL((reg_single_kernel<false, K, false>), dim3(1), dim3(64), 0, s, items, item,
                         recs, colors);
  });
  return hipGetLastError();
}

hipError_t launch_reg_tick(bool trace, bool stitch, int k, int grid, const int32_t* list,
                           int32_t len, int32_t* counter, const DevDesc* slot_desc,
                           uint8_t* slot_state, DevRecord* slot_rec, const uint64_t* arena64,
                           int8_t* arena8, const uint8_t* part8, const uint32_t* slot_minb,
                           int32_t* slot_min, uint64_t slice, DevRecord* tick_out, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    auto go = [&](auto t, auto st) {
      hipLaunchKernelGGL((reg_tick_kernel<decltype(t)::value, K, decltype(st)::value>), dim3(grid),
                         dim3(256), 0, s, list, len, counter, slot_desc, slot_state, slot_rec,
                         arena64, arena8, part8, slot_minb, slot_min, slice, tick_out);
    };
    if (trace && stitch) go(std::true_type{}, std::true_type{});
    else if (trace) go(std::true_type{}, std::false_type{});
    else if (stitch) go(std::false_type{}, std::true_type{});
    else go(std::false_type{}, std::false_type{});
  });
  return hipGetLastError();
}

hipError_t launch_reg_split(int k, int grid, const SplitTask* tasks, int32_t ntasks,
                            int32_t* counter, RegItems regitems, uint64_t cap,
                            uint32_t levels, uint8_t* out, SplitItem* pool,
                            int32_t* pool_count, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (levels < 1 || levels > (uint32_t)kSplitMaxLevels) return hipErrorInvalidValue;
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    hipLaunchKernelGGL((reg_split_kernel<K>), dim3(grid), dim3(256), 0, s, tasks, ntasks, counter,
                       regitems, cap, levels, out, pool, pool_count);
  });
  return hipGetLastError();
}

// ---- device-resident heavy engine ------------------------------------------

// Enumerates the top `levels` levels of the subtree at depth d (as
// reg_enumerate).  With items == nullptr it only counts; returns the items
// and sets nchild to the kind-0 items.  Otherwise item j goes to items[j]
// and the i-th subtask becomes task children_base + i: its path is this
// task's path plus the rows down to depth d + levels, which sit in lanes
// 0 .. d + levels - 1 of the frame register.  TRACE: each item also holds
// the trace hash of its seg nodes.
template <bool TRACE, int K, bool STITCH = false>
__device__ __forceinline__ int32_t engine_enumerate(RegState<K>& s, const uint32_t nb_lo,
                                                    const uint32_t nb_hi, const int32_t n,
                                                    const int32_t k,
                                                    const uint32_t d, const uint32_t levels,
                                                    EngineItem* __restrict__ items,
                                                    EngineTask* __restrict__ tasks,
                                                    const int32_t children_base,
                                                    const int32_t item_idx, const int32_t hc,
                                                    int8_t* __restrict__ sol, int32_t& nchild) {
  const uint32_t lane = __lane_id();
  const uint32_t limit = d + levels;
  uint32_t seg = 0;
  uint64_t segh = 0;
  int32_t count = 0;
  nchild = 0;
  auto emit = [&](uint32_t kind) {
    if (items != nullptr) {
      if (kind == 0) {   // the subtask: every lane writes its row, same header
        EngineTask* ch = tasks + children_base + nchild;
        ch->rows[lane] = lane < limit ? (uint16_t)(s.fr & 0xffffu) : (uint16_t)0;
        ch->item = item_idx;
        ch->depth = (int32_t)limit;
        ch->hc = hc;
        ch->skip = 0;
      }
      if (lane == ((uint32_t)count & 63u)) {   // one owner lane per item
        EngineItem it;
        it.seg = seg;
        it.child = kind == 0 ? children_base + nchild
                             : (kind == 1 ? kEngineItemEnd : kEngineItemSolution);
        it.hash = segh;
        items[count] = it;
      }
    }
    if (kind == 0) ++nchild;
    ++count;
    seg = 0;
    segh = 0;
  };
  for (;;) {
    uint32_t v = 0, c = 0, tried = 0;
    uint64_t alt = 0;
    bool back;
    if (s.depth == limit) {
      emit(0);        // a subtask root: leave it to its own task
      back = true;
    } else {
      ++seg;
      if (s.P == 0) {   // a solution among the top levels
        if (TRACE) segh = trace_node(segh, s.depth, s.row_in, kNone, 0);
        if (lane < s.depth && (s.fr & 0xffu) < (uint32_t)n)
          sol[s.fr & 0xffu] = (int8_t)((s.fr >> 8) & 0xffu);
        emit(2);
        break;
      }
      uint64_t any = s.O[0];
#pragma unroll
      for (int j = 1; j < K; ++j) any |= s.O[j];
      const uint64_t zero = s.P & ~any;
      back = zero != 0;
      if (back) {
        if (TRACE) segh = trace_node(segh, s.depth, s.row_in, low_bit(zero), 0);
      } else {
        uint64_t ge2;
        v = low_bit(min_count_columns(s.O, s.P, ge2));
        if (TRACE) segh = trace_node(segh, s.depth, s.row_in, v, (uint32_t)__popc(rows_of(s.O, v)));
        c = first_color(s.O, v);
        alt = (ge2 >> v) & 1ull;
        if (STITCH) stitch_pick(s, v, c, tried);
        s.P &= ~(1ull << v);
      }
    }
    if (back && !retreat<K, STITCH>(s, d, v, c, alt, tried)) {
      emit(1);
      break;
    }
    take_row<K, STITCH>(s, rdlane64(nb_lo, nb_hi, v), v, c, alt, tried);
    s.row_in = v * (uint32_t)k + c;
  }
  return count;
}

// Moves the round window on: the subtasks appended by the last round are
// the next round's tasks.
__global__ void engine_advance_kernel(EngineHead* head, int32_t task_cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    head->begin = head->end;
    head->end = head->alloc < task_cap ? head->alloc : task_cap;
    head->pop = 0;
    head->rounds += 1;
  }
}

// One round: every task of the window explores its subtree up to `cap`
// nodes (result block g at blocks + g * kSplitBlockBytes); a capped task
// reserves item and task space with atomics and appends its split.  A
// component whose explored nodes pass its limit, or a split that does not
// fit, is not split (status kEngineSkipped; its reserved task slots that
// exist are marked skip) and the host re-runs that component sequentially.
template <bool TRACE, int K, bool STITCH>
__global__ __launch_bounds__(256) void engine_round_kernel(
    EngineHead* __restrict__ head, EngineTask* __restrict__ tasks, int32_t task_cap,
    uint8_t* __restrict__ blocks, EngineItem* __restrict__ pool, int32_t pool_cap,
    const RegItems regitems, unsigned long long* __restrict__ hc_nodes,
    const uint64_t* __restrict__ hc_limit, uint64_t cap, uint32_t levels) {
  const uint32_t wpb = blockDim.x >> 6;
  const int32_t gw = (int32_t)(gridDim.x * wpb);
  const uint32_t lane = __lane_id();
  const int32_t begin = (int32_t)uniform((uint32_t)head->begin);
  const int32_t nt = (int32_t)uniform((uint32_t)head->end) - begin;
  // the grid is fixed and usually much larger than the round: plain block
  // order deals the first tasks to all eight XCDs (the XCD-range renumbering
  // of the other kernels would put them all on the first XCD)
  int32_t t = (int32_t)uniform(blockIdx.x * wpb + (threadIdx.x >> 6));
  while (t < nt) {
    const int32_t g = begin + t;
    const EngineTask* task = tasks + g;
    uint8_t* block = blocks + (uint64_t)g * kSplitBlockBytes;
    int8_t* sol = reinterpret_cast<int8_t*>(block + kSplitSolOffset);
    SplitResult res;
    res.status = kEngineSkipped;
    res.nitems = 0;
    res.nodes = 0;
    res.item_off = 0;
    res.pad = 0;
    res.hash = 0;
    if (uniform((uint32_t)task->skip) == 0) {
      const int32_t it = (int32_t)uniform((uint32_t)task->item);
      const uint32_t d = uniform((uint32_t)task->depth);
      const int32_t hc = (int32_t)uniform((uint32_t)task->hc);
      const DevDesc dd = item_desc(regitems, it);
      const uint64_t nb = item_mask(regitems, it, lane);
      const uint32_t nb_lo = (uint32_t)nb, nb_hi = (uint32_t)(nb >> 32);
      const uint32_t part = STITCH ? (item_partner(regitems, it, lane) << 8) | 0xffu : 0u;
      RegState<K> s;
      reg_init(s, dd.n, dd.k);
      if (STITCH) s.pc = part;
      reg_replay<K, STITCH>(s, nb_lo, nb_hi, dd.k, task->rows, d);
      reg_run<TRACE, K, STITCH>(s, nb_lo, nb_hi, dd.k, ~0ull, cap, d);
      res.nodes = s.nodes;
      res.hash = s.h;   // the task's own nodes, from its root
      if (s.status == MPLD_FEASIBLE) {
        if (lane < s.depth && (s.fr & 0xffu) < (uint32_t)dd.n)
          sol[s.fr & 0xffu] = (int8_t)((s.fr >> 8) & 0xffu);
        res.status = MPLD_FEASIBLE;
      } else if (s.status == MPLD_INFEASIBLE) {
        res.status = MPLD_INFEASIBLE;
      } else {
        // capped: count the split, then reserve space for it.  All of the
        // atomics are taken by lane 63 in one branch (a lane-0 branch here
        // could be merged with the queue pop's and split the wave).
        RegState<K> r;
        reg_init(r, dd.n, dd.k);
        if (STITCH) r.pc = part;
        reg_replay<K, STITCH>(r, nb_lo, nb_hi, dd.k, task->rows, d);
        int32_t nchild = 0;
        const int32_t nitems = engine_enumerate<false, K, STITCH>(r, nb_lo, nb_hi, dd.n, dd.k, d,
                                                                  levels, nullptr, nullptr, 0, it,
                                                                  hc, sol, nchild);
        // the component's explored nodes: the guard reads the total as of
        // the previous round (a plain load), and the add does not wait for
        // its result, so the reservations are the only round trips
        uint32_t io = 0xffffffffu, cb = 0xffffffffu;
        if (lane == 63u) {
          const unsigned long long seen = __hip_atomic_load(hc_nodes + hc, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(hc_nodes + hc, (unsigned long long)s.nodes, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          if (seen + s.nodes <= hc_limit[hc]) {
            io = (uint32_t)atomicAdd(&head->pool, nitems);
            cb = (uint32_t)atomicAdd(&head->alloc, nchild);
          }
        }
        io = (uint32_t)__builtin_amdgcn_readlane((int)io, 63);
        cb = (uint32_t)__builtin_amdgcn_readlane((int)cb, 63);
        const bool limited = io == 0xffffffffu;
        const bool fits = !limited && (int64_t)io + nitems <= pool_cap &&
                          (int64_t)cb + nchild <= task_cap;
        if (fits) {
          reg_init(r, dd.n, dd.k);
          if (STITCH) r.pc = part;
          reg_replay<K, STITCH>(r, nb_lo, nb_hi, dd.k, task->rows, d);
          int32_t nc2 = 0;
          engine_enumerate<TRACE, K, STITCH>(r, nb_lo, nb_hi, dd.n, dd.k, d, levels, pool + io,
                                             tasks, (int32_t)cb, it, hc, sol, nc2);
          res.status = -1;
          res.nitems = nitems;
          res.item_off = io;
        } else {
          if (!limited) {
            // reserved slots that exist must not be run as tasks (a loop
            // with a uniform trip count: every branch here stays uniform)
            for (int32_t j0 = 0; j0 < nchild; j0 += 64) {
              const int32_t j = j0 + (int32_t)lane;
              if (j < nchild && (int64_t)cb + j < task_cap) tasks[cb + j].skip = 1;
            }
            if (lane == 63u) atomicExch(&head->overflow, 1);
          }
          res.status = kEngineSkipped;
        }
      }
    }
    *reinterpret_cast<SplitResult*>(block) = res;   // same value from every lane
    if (gw >= nt) break;
    int32_t q = 0;
    if (lane == 0) q = atomicAdd(&head->pop, 1);
    q = (int32_t)uniform((uint32_t)q);
    t = gw + q;
  }
}

hipError_t launch_engine_advance(EngineHead* head, int32_t task_cap, hipStream_t s) {
  hipLaunchKernelGGL(engine_advance_kernel, dim3(1), dim3(64), 0, s, head, task_cap);
  return hipGetLastError();
}

hipError_t launch_engine_round(int k, int grid, EngineHead* head, EngineTask* tasks,
                               int32_t task_cap, uint8_t* blocks, EngineItem* pool,
                               int32_t pool_cap, RegItems regitems,
                               unsigned long long* hc_nodes, const uint64_t* hc_limit,
                               uint64_t cap, uint32_t levels, bool trace, hipStream_t s) {
  if (levels < 1 || levels > (uint32_t)kSplitMaxLevels) return hipErrorInvalidValue;
  const bool stitch = regitems.part_off != 0;   // the items carry stitch partners
  with_planes(k, [&](auto kp) {
    constexpr int K = decltype(kp)::value;
    if (trace && stitch)
      hipLaunchKernelGGL((engine_round_kernel<true, K, true>), dim3(grid), dim3(256), 0, s, head,
                         tasks, task_cap, blocks, pool, pool_cap, regitems, hc_nodes, hc_limit, cap,
                         levels);
    else if (trace)
      hipLaunchKernelGGL((engine_round_kernel<true, K, false>), dim3(grid), dim3(256), 0, s, head,
                         tasks, task_cap, blocks, pool, pool_cap, regitems, hc_nodes, hc_limit, cap,
                         levels);
    else if (stitch)
      hipLaunchKernelGGL((engine_round_kernel<false, K, true>), dim3(grid), dim3(256), 0, s, head,
                         tasks, task_cap, blocks, pool, pool_cap, regitems, hc_nodes, hc_limit, cap,
                         levels);
    else
      hipLaunchKernelGGL((engine_round_kernel<false, K, false>), dim3(grid), dim3(256), 0, s, head,
                         tasks, task_cap, blocks, pool, pool_cap, regitems, hc_nodes, hc_limit, cap,
                         levels);
  });
  return hipGetLastError();
}

// One wave per entry: the record by one lane, the colors one per lane.
__global__ __launch_bounds__(64) void heavy_writeback_kernel(const HeavyWrite* __restrict__ w,
                                                             DevRecord* __restrict__ recs,
                                                             int8_t* __restrict__ colors) {
  const HeavyWrite& e = w[blockIdx.x];
  const uint32_t lane = threadIdx.x;
  if (lane < (uint32_t)e.n) colors[e.out_off + (int32_t)lane] = e.colors[lane];
  if (lane == 0) recs[e.comp] = e.rec;
}

hipError_t launch_heavy_writeback(const HeavyWrite* w, int32_t count, DevRecord* recs,
                                  int8_t* colors, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(heavy_writeback_kernel, dim3(count), dim3(64), 0, s, w, recs, colors);
  return hipGetLastError();
}

int reg_batched_blocks_per_cu(bool trace) {
  int blocks = 0;
  hipError_t e = trace ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<true, 8, false>, 256, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &blocks, reg_batched_kernel<false, 8, false>, 256, 0);
  return e == hipSuccess && blocks > 0 ? blocks : 1;
}

}  // namespace mpld
