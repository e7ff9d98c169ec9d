// search_lds.hip - LDS tier of the exact-cover search (components of more
// than 64 nodes), one 64-lane wavefront per component.
//
// Same matrix and rules as the register tier (Sec. 2.3, Algorithm 1), with
// the state spread over W = ceil(n/64) words per bit-plane:
//   PL[c][w]  (c < k) color plane: bit v set while color c is open at v,
//             i.e. while row (v, c) is active;
//   PL[k][w]  uncovered primary columns P.
// Column choice (count + select): lane l takes words l, l+64, ...; a
// bit-sliced adder over the k planes gives per-word count-bit planes,
// narrowing P from the top count bit leaves the lowest-count columns of the
// word, and the key (count << 24 | index) of its lowest one goes into a
// DPP min-reduction over the wave: the global minimum is the fewest-rows,
// lowest-index column.  All-ones means P is empty (a solution).
// Cover of row (v, c) (Eq. 2): P loses v, and each neighbour u of v loses
// color c through an LDS atomic AND that returns the old word, so a lane
// knows whether it removed an active row; those rows go to an undo log of
// 32-bit entries (plane << 26 | node), after one entry for v's P bit.
// Uncover (Eq. 2) ORs entries back.  Because OR commutes and the removed
// bits of different levels are disjoint, a backtrack over several levels is
// one lane-parallel pass over the log suffix: a per-depth bit set marks
// levels whose column still has untried rows, and the deepest such level
// is found with a word scan instead of popping level by level.
//
// Placement: the planes always live in LDS.  Small components run on one
// wave and also keep their neighbour lists, level headers and undo log in
// LDS (the per-depth bit set in lane registers); "big" components run on a
// workgroup of up to 16 waves that share the column scan, and keep the
// per-depth bit set in LDS and the rest in global memory (header and log in
// a per-worker scratch area).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_types.h"
#include "mpld.h"
#include "trace.h"
#include "wave_ops.h"

namespace mpld {

static constexpr uint32_t kNoneL = 0xffffffffu;
static constexpr uint32_t kNoKey = 0xffffffffu;
static constexpr uint32_t kEntryNodeBits = 26;   // undo entry: plane << 26 | node

__device__ __forceinline__ uint32_t uni(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

constexpr int bits_for(int x) { return x == 0 ? 0 : 1 + bits_for(x >> 1); }

__device__ __forceinline__ uint32_t wave_min(uint32_t m) { return wave_min_u32(m); }

// Key of the lowest-count, lowest-index uncovered column in word w:
// (count << 24) | (64 w + bit), or kNoKey when the word has none.
template <int K>
__device__ __forceinline__ uint32_t word_key(const uint64_t* PL, uint32_t W, uint32_t w) {
  constexpr int NB = bits_for(K);
  uint64_t a[K];
#pragma unroll
  for (int c = 0; c < K; ++c) a[c] = PL[(uint32_t)c * W + w];
  const uint64_t p = PL[(uint32_t)K * W + w];
  uint64_t cnt[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) cnt[b] = 0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    uint64_t carry = a[c];
#pragma unroll
    for (int b = 0; b < bits_for(c + 1); ++b) {
      const uint64_t t = cnt[b] & carry;
      cnt[b] ^= carry;
      carry = t;
    }
  }
  uint64_t cand = p;
  uint32_t t = 0;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    const uint64_t x = cand & ~cnt[b];
    if (x) cand = x;
    else t |= 1u << b;
  }
  const uint32_t key = (t << 24) | (w << 6) | (uint32_t)__builtin_ctzll(cand | (1ull << 63));
  return p ? key : kNoKey;
}

// Byte layout of the LDS area of one component.
struct LdsLayout {
  uint32_t W, E, pl_off, a_off, adj_off, hdr_off, ent_off, ctl_off, col_off, total;
};

// Undo-log capacity: one entry per level (its P bit) plus the removed rows,
// at most one per (neighbour, color) pair and at most one per incidence.
__host__ __device__ inline uint32_t lds_log_entries(int32_t n, int32_t k, int64_t adj_words) {
  const int64_t incid = adj_words - n - 1;   // 2m
  const int64_t nk = (int64_t)n * k;
  return (uint32_t)(n + (incid < nk ? incid : nk));
}

__host__ __device__ inline LdsLayout lds_layout(int32_t n, int32_t k, int64_t adj_words, bool big,
                                               bool stitch = false) {
  LdsLayout L;
  L.W = (uint32_t)((n + 63) / 64);
  L.E = lds_log_entries(n, k, adj_words);
  uint32_t off = big ? 16u : 0u;   // big: the workgroup's queue pop result first
  L.pl_off = off;
  off += 8u * (uint32_t)(k + 1) * L.W;
  L.a_off = off;
  if (big) off += 8u * L.W;   // one bit per depth 0 .. n-1 (small: in registers)
  L.ctl_off = off;
  if (big) off += 128u;       // per-wave minima, loop status, final depth
  L.col_off = off;            // stitch-aware order: each covered node's color
  if (big && stitch) off += (uint32_t)n;
  L.adj_off = off;
  if (!big) off += 4u * (uint32_t)adj_words;
  off = (off + 7u) & ~7u;
  L.hdr_off = off;
  if (!big) off += 8u * (uint32_t)n;
  L.ent_off = off;
  if (!big) off += 4u * L.E;
  L.total = (off + 7u) & ~7u;
  return L;
}

// Level header: v | c << 24 | rows << 28 | log start << 36.
__device__ __forceinline__ uint64_t make_hdr(uint32_t v, uint32_t c, uint32_t rows, uint32_t est) {
  return (uint64_t)v | ((uint64_t)c << 24) | ((uint64_t)rows << 28) | ((uint64_t)est << 36);
}

// ---- one-wave tier --------------------------------------------------------
//
// Components of at most kLds1MaxN nodes: one wave, 32-bit plane words, one
// node word per lane (lane l holds nodes 32l .. 32l+31), everything in LDS:
//   planes   64 node words x S dwords: word w of plane c (c < k) at w*S + c,
//            P at w*S + k, so a lane reads all of its word's planes with
//            S/4 ds_read_b128 (S = k+1 rounded up to 4, 8 or 16);
//   offs     per node: first neighbour (low 16 bits) | degree << 16;
//   ids      16-bit neighbour ids;
//   hdr      per depth: {offs of the level's column, est | untried << 16 |
//            c << 24} (est: the level's first log entry, which holds the
//            column's P bit, so the column itself is read back from the log;
//            untried: the column's rows not tried yet at this level);
//   ent      the undo log;
//   (stitch-aware order) each node's stitch partner and the color of each
//            covered node.
// The per-depth "untried rows" bit set is one 32-bit word per lane (depth d
// in lane d >> 5).  Per node the dependent chain is: the plane words (read
// at the end of the previous node, behind its cover atomics), the count and
// narrowing in each lane, a wave minimum, then the winner's row set and
// offs word (each lane reads the offs word of its own candidate before the
// minimum, so the winner's is already in a register), one read of the
// neighbour ids, and one atomic AND per neighbour (lane 0 clears the
// column's P bit in the same instruction).
__host__ __device__ constexpr uint32_t lds1_stride(int32_t k) {
  return k + 1 <= 4 ? 4u : (k + 1 <= 8 ? 8u : 16u);
}

struct Lds1Layout {
  uint32_t offs_off, ids_off, hdr_off, ent_off, part_off, col_off, total;
};

// stitch: also each node's stitch partner (16 bits, 0xffff none) and the
// color of each covered node (one byte).
__host__ __device__ inline Lds1Layout lds1_layout(int32_t n, int32_t k, int64_t adj_words,
                                                 bool stitch = false) {
  Lds1Layout L;
  const uint32_t m2 = (uint32_t)(adj_words - n - 1);
  L.offs_off = 64u * 4u * lds1_stride(k);
  L.ids_off = L.offs_off + 4u * (uint32_t)(n > 0 ? n : 1);   // one offs word at least
  L.hdr_off = (L.ids_off + 2u * m2 + 7u) & ~7u;
  L.ent_off = L.hdr_off + 8u * (uint32_t)n;
  L.part_off = L.ent_off + 4u * lds_log_entries(n, k, adj_words);
  L.col_off = L.part_off + (stitch ? 2u * (uint32_t)(n > 0 ? n : 1) : 0u);
  L.total = (L.col_off + (stitch ? (uint32_t)n : 0u) + 15u) & ~15u;
  return L;
}

template <int K>
struct Lds1Words {
  static constexpr int S = (int)lds1_stride(K);
  uint32_t a[S];
  __device__ __forceinline__ void load(const uint32_t* PL, uint32_t lane) {
    const uint4* q = reinterpret_cast<const uint4*>(PL + lane * (uint32_t)S);
#pragma unroll
    for (int j = 0; j < S / 4; ++j) {
      const uint4 x = q[j];
      a[4 * j] = x.x;
      a[4 * j + 1] = x.y;
      a[4 * j + 2] = x.z;
      a[4 * j + 3] = x.w;
    }
  }
};

// root_row >= 0: search only the subtree of root row (0, root_row) (a
// subtree task of the heavy-component split): at the root every column has
// all k rows, so the root column is node 0; its row is taken at depth 0
// with no alternative left at that level, the root node itself is not
// counted, and `budget` (> 0) replaces the component's.
// STITCH: the stitch-aware row order (a column whose stitch partner is on
// the path tries the partner's color first when that row is open, then the
// others ascending); the CSR block then ends with the partners.
template <bool TRACE, int K, bool STITCH>
__device__ void solve_lds(const DevDesc& d, const uint32_t* __restrict__ gadj, char* lds,
                          int8_t* __restrict__ colors, DevRecord* __restrict__ rec,
                          int32_t root_row = -1, uint64_t task_budget = 0) {
  constexpr uint32_t S = lds1_stride(K);
  constexpr uint32_t kLS = S == 4u ? 2u : (S == 8u ? 3u : 4u);   // log2(S)
  constexpr int NB = bits_for(K);
  constexpr uint32_t kNodeMask = (1u << kEntryNodeBits) - 1u;
  const uint32_t lane = __lane_id();
  const uint32_t n = (uint32_t)d.n;
  const uint32_t m2 = uni(gadj[n]);
  const Lds1Layout L = lds1_layout((int32_t)n, K, (int64_t)m2 + n + 1, STITCH);
  uint32_t* PL = reinterpret_cast<uint32_t*>(lds);
  uint32_t* offs = reinterpret_cast<uint32_t*>(lds + L.offs_off);
  uint16_t* ids = reinterpret_cast<uint16_t*>(lds + L.ids_off);
  uint2* hdr = reinterpret_cast<uint2*>(lds + L.hdr_off);
  uint32_t* ent = reinterpret_cast<uint32_t*>(lds + L.ent_off);
  uint16_t* spart = reinterpret_cast<uint16_t*>(lds + L.part_off);
  uint8_t* scol = reinterpret_cast<uint8_t*>(lds + L.col_off);
  for (uint32_t v = lane; v < n; v += 64) {
    const uint32_t b = gadj[v], e = gadj[v + 1];
    offs[v] = b | ((e - b) << 16);
    if (STITCH) {
      const uint32_t p = gadj[n + 1 + m2 + 1 + v];
      spart[v] = p < n ? (uint16_t)p : (uint16_t)0xffffu;
    }
  }
  for (uint32_t i = lane; i < m2; i += 64) ids[i] = (uint16_t)gadj[n + 1 + i];
  {
    // every node uncovered with all k colors open; words past n are empty
    const uint32_t base = lane * 32u;
    const uint32_t cnt = base >= n ? 0u : (n - base >= 32u ? 32u : n - base);
    const uint32_t val = cnt == 32u ? ~0u : ((1u << cnt) - 1u);
#pragma unroll
    for (uint32_t c = 0; c < S; ++c) PL[lane * S + c] = c <= (uint32_t)K ? val : 0u;
  }
  __syncthreads();

  uint32_t depth = 0, row_in = kNoneL, esp = 0;
  uint64_t nodes = 0, h = 0;
  int32_t status = -1;
  uint32_t areg = 0;   // untried-rows bit of depth 32 * lane + b
  const uint64_t budget = root_row >= 0 ? task_budget : (uint64_t)d.budget;
  Lds1Words<K> W;

  // Take row (v, c) at `depth`: the level's header and untried-rows bit,
  // then one atomic AND per neighbour of v on plane c (lanes 1 .. deg) and,
  // if `lane_lo` is 0, on v's P bit (lane 0); the removed rows go to the log from
  // `est` (v's P bit first), and the plane words of the next node are read
  // right behind the atomics.
  const uint16_t* ids_m1 = ids - 1;   // lane j reads neighbour j - 1
  const uint32_t is_l0 = lane == 0u ? ~0u : 0u;
  auto take_row = [&](uint32_t v, uint32_t c, uint32_t rows, uint32_t offv, uint32_t est,
                      uint32_t lane_lo, bool more) {
    const uint32_t beg = offv & 0xffffu, deg = offv >> 16;
    const uint32_t first = deg < 63u ? deg : 63u;
    // lane 0: v's P bit (lane_lo 0); lanes 1 .. first: the first neighbours
    // (lane 0 reads the halfword before the list, a valid LDS word it ignores)
    const bool act = lane >= lane_lo && lane <= first;
    uint32_t old = 0u, bitm = 0u, entry = 0u;
    if (act) {
      const uint32_t idv = ids_m1[beg + lane];
      const uint32_t u = (is_l0 & v) | (~is_l0 & idv);
      const uint32_t pl4 = (is_l0 & ((uint32_t)K * 4u)) | (~is_l0 & (c * 4u));
      bitm = 1u << (u & 31u);
      old = atomicAnd(reinterpret_cast<uint32_t*>(lds + (((u >> 5) << (kLS + 2u)) | pl4)), ~bitm);
      entry = (pl4 << 24) | u;
    }
    // the next node's plane words, behind the atomics (read again below
    // when v has more than 63 neighbours); the empty asm keeps the use of
    // the atomic's result after that read is issued
    W.load(PL, lane);
    asm volatile("" : "+v"(old) : : "memory");
    if (lane == 0u) {
      hdr[depth] = make_uint2(offv, est | (rows << 16) | (c << 24));
      if (STITCH) scol[v] = (uint8_t)c;
    }
    {
      const uint32_t dl = depth >> 5, db = 1u << (depth & 31u);
      const uint32_t sel = lane == dl ? db : 0u;
      areg = (sel & (more ? ~0u : 0u)) | (~sel & areg);
    }
    uint32_t slot = est + lane_lo;
    auto log_hits = [&](bool hit, uint32_t e) {
      const uint64_t bal = __builtin_amdgcn_ballot_w64(hit);
      if (hit) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        ent[slot + rank] = e;
      }
      slot += (uint32_t)__popcll(bal);
    };
    log_hits((old & bitm) != 0u, entry);
    if (deg > 63u) {
      for (uint32_t ch = 63u; ch < deg; ch += 64u) {
        bool hit = false;
        uint32_t uu = 0;
        if (ch + lane < deg) {
          uu = ids[beg + ch + lane];
          const uint32_t b = 1u << (uu & 31u);
          hit = (atomicAnd(&PL[(uu >> 5) * S + c], ~b) & b) != 0u;
        }
        log_hits(hit, (c << kEntryNodeBits) | uu);
      }
      W.load(PL, lane);
    }
    esp = slot;
    // One wave executes its LDS operations in order, so the next node's
    // loads see these writes; this only keeps the compiler from caching
    // LDS values across the loop.
    asm volatile("" ::: "memory");
  };

  if (root_row >= 0) {
    // row (0, root_row) at depth 0, with no alternative at that level
    const uint32_t c = (uint32_t)root_row;
    take_row(0u, c, 0u, uni(offs[0]), 0u, 0u, false);
    depth = 1u;
    row_in = c;
  } else {
    W.load(PL, lane);
  }

  while (status < 0) {
    // ---- one search node
    if (nodes == budget) { status = MPLD_BUDGET_EXHAUSTED; break; }
    ++nodes;
    // column choice: bit-sliced counts of this lane's word, narrowed from
    // the top count bit to the lowest-count uncovered columns
    uint32_t cnt[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) cnt[b] = 0u;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      uint32_t carry = W.a[c];
#pragma unroll
      for (int b = 0; b < bits_for(c + 1); ++b) {
        const uint32_t t = cnt[b] & carry;
        cnt[b] ^= carry;
        carry = t;
      }
    }
    const uint32_t p = W.a[K];
    uint32_t cand = p, t = 0u;
#pragma unroll
    for (int b = NB - 1; b >= 0; --b) {
      const uint32_t x = cand & ~cnt[b];
      if (x) cand = x;
      else t |= 1u << b;
    }
    const uint32_t bit = (uint32_t)__builtin_ctz(cand | 0x80000000u);
    const uint32_t vl = (lane << 5) | bit;
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) r |= __builtin_amdgcn_ubfe(W.a[c], bit, 1u) << c;
    const uint32_t vc = vl < n ? vl : 0u;   // lanes past n read node 0's words
    const uint32_t pre = offs[vc];
    const uint32_t prp = STITCH ? (uint32_t)spart[vc] : 0xffffu;
    // issue those reads before the minimum (which they then overlap)
    asm volatile("" ::: "memory");
    const uint32_t key = wave_min(p ? ((t << 24) | vl) : kNoKey);
    if (key == kNoKey) {   // no uncovered column: the levels hold a solution
      if (TRACE) h = trace_node(h, depth, row_in, kNoneL, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    uint32_t v = key & 0xffffffu;
    const uint32_t size = key >> 24;
    if (TRACE) h = trace_node(h, depth, row_in, v, size);
    uint32_t rows, offv, est, lane_lo, c;
    if (size != 0) {
      const uint32_t wl = v >> 5;
      rows = rdlane(r, wl);
      offv = rdlane(pre, wl);
      est = esp;
      lane_lo = 0u;
      c = (uint32_t)__builtin_ctz(rows);
      if (STITCH) {
        // the partner's color first when the partner is covered (its P bit,
        // in its lane's word, is clear) and that row of v is open
        const uint32_t p = rdlane(prp, wl);
        if (p != 0xffffu && !((rdlane(W.a[K], p >> 5) >> (p & 31u)) & 1u)) {
          const uint32_t cp = uni((uint32_t)scol[p]);
          if ((rows >> cp) & 1u) c = cp;
        }
      }
      rows &= ~(1u << c);   // the level's untried rows
    } else {
      // dead end: back to the deepest level whose column has an untried row
      uint32_t f = kNoneL;
      if (depth != 0) {
        const uint32_t d1 = depth - 1u, dw = d1 >> 5;
        const uint32_t below = ~0u >> (31u - (d1 & 31u));
        const uint32_t m = lane < dw ? areg : (lane == dw ? areg & below : 0u);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(m != 0u);
        if (bal) {
          const uint32_t l = 63u - (uint32_t)__builtin_clzll(bal);
          f = l * 32u + 31u - (uint32_t)__builtin_clz(rdlane(m, l));
        }
      }
      if (f == kNoneL) { status = MPLD_INFEASIBLE; break; }
      const uint2 hd = hdr[f];
      offv = uni(hd.x);
      const uint32_t d1w = uni(hd.y);
      est = d1w & 0xffffu;
      // uncover every level above f, and the rows level f removed; the
      // column stays covered (its P bit is entry est)
      for (uint32_t i = est + 1u + lane; i < esp; i += 64) {
        const uint32_t e = ent[i];
        const uint32_t u = e & kNodeMask;
        atomicOr(&PL[(u >> 5) * S + (e >> kEntryNodeBits)], 1u << (u & 31u));
      }
      if (TRACE || STITCH) v = uni(ent[est]) & kNodeMask;
      // the next untried row of the level, in ascending order
      rows = (d1w >> 16) & 0xffu;
      c = (uint32_t)__builtin_ctz(rows);
      rows &= rows - 1u;
      depth = f;
      lane_lo = 1u;
    }
    take_row(v, c, rows, offv, est, lane_lo, rows != 0u);
    row_in = v * (uint32_t)K + c;
    ++depth;
  }
  __syncthreads();
  if (status == MPLD_FEASIBLE) {
    for (uint32_t f = lane; f < depth; f += 64) {
      const uint32_t d1w = hdr[f].y;
      colors[ent[d1w & 0xffffu] & kNodeMask] = (int8_t)((d1w >> 24) & 0xfu);
    }
  } else {
    for (uint32_t v = lane; v < n; v += 64) colors[v] = -1;
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

// ---- one-wave wide tier ---------------------------------------------------
//
// Big components whose planes and neighbour lists fit in LDS: one wave, as
// the one-wave tier, but up to kWideMaxWords 32-bit node words per lane
// (word w in lane w & 63), so no barrier per node, and the column choice
// reads a cache of per-word keys instead of recounting every word: key(w) =
// count << 28 | node << 8 | rows of the lowest-count, lowest-index
// uncovered column of word w (kNoKey when w has none).  A cover changes
// only the words of the column and of its neighbours, so after the cover
// atomics each lane that made one reads its word's planes back and
// rewrites that word's key; after a backtrack (the undo log touches any
// words) every key is recomputed.  Per node a lane reads its keys (at most
// eight, two ds_read_b128), takes their minimum, and the wave minimum is
// the column with its count and rows.  LDS: the planes, the keys, the
// per-depth "untried rows" bit set, offs (first neighbour | degree << 17),
// 16-bit neighbour ids, and for the stitch-aware order the partners and the
// color of each covered node.  Level headers {log start, v | untried << 16
// | c << 24} and the undo log go to the worker's global area: the forward
// path only stores to it (nothing waits for those stores), and a backtrack
// - rare on components this large - reads it back after a fence.
__host__ __device__ inline uint32_t wide_words(int32_t n) {
  const uint32_t w = (uint32_t)((n + 2047) / 2048);   // 64 lanes x 32 nodes
  return w < 1u ? 1u : w;
}

struct WideLayout {
  uint32_t pl_off, key_off, bits_off, offs_off, ids_off, part_off, col_off, total;
};

__host__ __device__ inline WideLayout wide_layout(int32_t n, int32_t k, int64_t adj_words,
                                                  bool stitch) {
  WideLayout L;
  const uint32_t m2 = (uint32_t)(adj_words - n - 1);
  const uint32_t n1 = (uint32_t)(n > 0 ? n : 1);   // one offs word at least
  L.pl_off = 16u;   // the workgroup's queue pop result first
  L.key_off = L.pl_off + 64u * wide_words(n) * 4u * lds1_stride(k);
  L.bits_off = L.key_off + 64u * 4u * (uint32_t)kWideMaxWords;
  L.offs_off = L.bits_off + ((4u * (((uint32_t)n + 31u) / 32u) + 15u) & ~15u);
  L.ids_off = L.offs_off + 4u * n1;
  L.part_off = (L.ids_off + 2u * m2 + 15u) & ~15u;
  L.col_off = L.part_off + (stitch ? 2u * n1 : 0u);
  L.total = (L.col_off + (stitch ? (uint32_t)n : 0u) + 15u) & ~15u;
  return L;
}

// Key of word w (planes in W): count << 28 | node << 8 | rows (count <= k <= 8,
// node < 2^20).
template <int K>
__device__ __forceinline__ uint32_t wide_key(const Lds1Words<K>& W, uint32_t w) {
  constexpr int NB = bits_for(K);
  uint32_t cnt[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) cnt[b] = 0u;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    uint32_t carry = W.a[c];
#pragma unroll
    for (int b = 0; b < bits_for(c + 1); ++b) {
      const uint32_t t = cnt[b] & carry;
      cnt[b] ^= carry;
      carry = t;
    }
  }
  const uint32_t p = W.a[K];
  uint32_t cand = p, t = 0u;
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    const uint32_t x = cand & ~cnt[b];
    if (x) cand = x;
    else t |= 1u << b;
  }
  const uint32_t bit = (uint32_t)__builtin_ctz(cand | 0x80000000u);
  uint32_t r = 0;
#pragma unroll
  for (int c = 0; c < K; ++c) r |= __builtin_amdgcn_ubfe(W.a[c], bit, 1u) << c;
  return p ? (t << 28) | (((w << 5) | bit) << 8) | r : kNoKey;
}

template <bool TRACE, int K, bool STITCH>
__device__ void solve_lds_wide(const DevDesc& d, const uint32_t* __restrict__ gadj, char* lds,
                               uint64_t* gstack, int8_t* __restrict__ colors,
                               DevRecord* __restrict__ rec, int32_t root_row = -1,
                               uint64_t task_budget = 0) {
  constexpr uint32_t S = lds1_stride(K);
  constexpr uint32_t kLS = S == 4u ? 2u : (S == 8u ? 3u : 4u);   // log2(S)
  constexpr uint32_t NW = (uint32_t)kWideMaxWords;
  constexpr uint32_t kNodeMask = (1u << kEntryNodeBits) - 1u;
  const uint32_t lane = __lane_id();
  const uint32_t n = (uint32_t)d.n;
  const uint32_t m2 = uni(gadj[n]);
  const WideLayout L = wide_layout((int32_t)n, K, (int64_t)m2 + n + 1, STITCH);
  const uint32_t nwl = wide_words((int32_t)n);   // node words per lane (uniform)
  uint32_t* PL = reinterpret_cast<uint32_t*>(lds + L.pl_off);
  // key of word w (lane w & 63, its j = w >> 6) at key_pos(w): a lane's keys
  // j < 4 and j >= 4 each fill 16 contiguous bytes, and the lanes' blocks
  // follow each other, so both ds_read_b128 of the keys are conflict-free
  uint32_t* keys = reinterpret_cast<uint32_t*>(lds + L.key_off);
  auto key_pos = [](uint32_t w) { return ((w >> 8) << 8) | ((w & 63u) << 2) | ((w >> 6) & 3u); };
  uint32_t* dbits = reinterpret_cast<uint32_t*>(lds + L.bits_off);
  uint32_t* offs = reinterpret_cast<uint32_t*>(lds + L.offs_off);
  uint16_t* ids = reinterpret_cast<uint16_t*>(lds + L.ids_off);
  uint16_t* spart = reinterpret_cast<uint16_t*>(lds + L.part_off);
  uint8_t* scol = reinterpret_cast<uint8_t*>(lds + L.col_off);
  uint2* hdr = reinterpret_cast<uint2*>(gstack);
  uint32_t* ent = reinterpret_cast<uint32_t*>(gstack + n);
  for (uint32_t v = lane; v < n; v += 64) {
    const uint32_t b = gadj[v], e = gadj[v + 1];
    offs[v] = b | ((e - b) << kWideBegBits);
    if (STITCH) {
      const uint32_t p = gadj[n + 1 + m2 + 1 + v];
      spart[v] = p < n ? (uint16_t)p : (uint16_t)0xffffu;
    }
  }
  for (uint32_t i = lane; i < m2; i += 64) ids[i] = (uint16_t)gadj[n + 1 + i];
  for (uint32_t w = lane; w < 64u * nwl; w += 64) {
    // every node uncovered with all k colors open; words past n are empty
    const uint32_t base = w * 32u;
    const uint32_t cnt = base >= n ? 0u : (n - base >= 32u ? 32u : n - base);
    const uint32_t val = cnt == 32u ? ~0u : ((1u << cnt) - 1u);
#pragma unroll
    for (uint32_t c = 0; c < S; ++c) PL[w * S + c] = c <= (uint32_t)K ? val : 0u;
  }
#pragma unroll
  for (uint32_t j = 0; j < NW; ++j) keys[j * 64u + lane] = kNoKey;
  __syncthreads();

  uint32_t depth = 0, row_in = kNoneL, esp = 0;
  uint64_t nodes = 0, h = 0;
  int32_t status = -1;
  const uint64_t budget = root_row >= 0 ? task_budget : (uint64_t)d.budget;
  Lds1Words<K> W;
  // every key of this lane's words, from the planes
  auto all_keys = [&]() {
#pragma unroll
    for (uint32_t j = 0; j < NW; ++j) {
      if (j < nwl) {
        const uint32_t w = lane + 64u * j;
        W.load(PL, w);
        keys[key_pos(w)] = wide_key<K>(W, w);
      }
    }
  };
  all_keys();

  // This lane's keys for the next node's column choice (words j >= nwl
  // hold kNoKey).
  uint4 ka, kb = make_uint4(kNoKey, kNoKey, kNoKey, kNoKey);
  auto read_keys = [&]() {
    ka = *reinterpret_cast<const uint4*>(keys + lane * 4u);
    if (nwl > 4u) kb = *reinterpret_cast<const uint4*>(keys + 256u + lane * 4u);
  };

  // Take row (v, c) at `depth`: one atomic AND per neighbour of v on plane
  // c (lanes 1 .. deg) and, if `lane_lo` is 0, on v's P bit (lane 0); then
  // the keys of the words those atomics changed (every key when `full` or
  // with more than 63 neighbours) and this lane's keys for the next node,
  // read before the header, the untried-rows bit and the removed rows
  // (global memory) are written, so that their latency overlaps that work.
  const uint16_t* ids_m1 = ids - 1;   // lane j reads neighbour j - 1
  const uint32_t is_l0 = lane == 0u ? ~0u : 0u;
  auto take_row = [&](uint32_t v, uint32_t c, uint32_t rows, uint32_t offv, uint32_t est,
                      uint32_t lane_lo, bool more, bool full) {
    const uint32_t beg = offv & ((1u << kWideBegBits) - 1u), deg = offv >> kWideBegBits;
    const uint32_t first = deg < 63u ? deg : 63u;
    full = full || deg > 63u;
    const bool act = lane >= lane_lo && lane <= first;
    uint32_t old = 0u, bitm = 0u, entry = 0u, u = 0u;
    if (act) {
      const uint32_t idv = ids_m1[beg + lane];
      u = (is_l0 & v) | (~is_l0 & idv);
      const uint32_t pl4 = (is_l0 & ((uint32_t)K * 4u)) | (~is_l0 & (c * 4u));
      bitm = 1u << (u & 31u);
      old = atomicAnd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(PL) +
                                                  (((u >> 5) << (kLS + 2u)) | pl4)),
                      ~bitm);
      entry = (pl4 << 24) | u;
      // the changed word, read right behind the atomic (LDS operations of
      // one wave complete in order)
      if (!full) W.load(PL, u >> 5);
    }
    asm volatile("" : "+v"(old) : : "memory");
    if (!full) {
      // lanes on the same word compute the same key
      if (act) {
        const uint32_t w = u >> 5;
        keys[key_pos(w)] = wide_key<K>(W, w);
      }
      read_keys();
    }
    asm volatile("" ::: "memory");
    if (lane == 0u) {
      hdr[depth] = make_uint2(est, v | (rows << 16) | (c << 24));
      const uint32_t db = 1u << (depth & 31u);
      atomicAnd(&dbits[depth >> 5], ~db);
      if (more) atomicOr(&dbits[depth >> 5], db);
      if (STITCH) scol[v] = (uint8_t)c;
    }
    uint32_t slot = est + lane_lo;
    auto log_hits = [&](bool hit, uint32_t e) {
      const uint64_t bal = __builtin_amdgcn_ballot_w64(hit);
      if (hit) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        ent[slot + rank] = e;
      }
      slot += (uint32_t)__popcll(bal);
    };
    log_hits((old & bitm) != 0u, entry);
    if (deg > 63u) {
      for (uint32_t ch = 63u; ch < deg; ch += 64u) {
        bool hit = false;
        uint32_t uu = 0;
        if (ch + lane < deg) {
          uu = ids[beg + ch + lane];
          const uint32_t b = 1u << (uu & 31u);
          hit = (atomicAnd(&PL[(uu >> 5) * S + c], ~b) & b) != 0u;
        }
        log_hits(hit, (c << kEntryNodeBits) | uu);
      }
    }
    esp = slot;
    asm volatile("" ::: "memory");
    if (full) {
      all_keys();
      read_keys();
    }
    asm volatile("" ::: "memory");
  };

  if (root_row >= 0) {
    // row (0, root_row) at depth 0, with no alternative at that level
    const uint32_t c = (uint32_t)root_row;
    take_row(0u, c, 0u, uni(offs[0]), 0u, 0u, false, false);
    depth = 1u;
    row_in = c;
  } else {
    read_keys();
  }

  for (;;) {   // every exit sets the status
    // ---- one search node
    if (nodes == budget) { status = MPLD_BUDGET_EXHAUSTED; break; }
    ++nodes;
    // column choice: the lowest key of this lane's words, then of the wave
    const uint32_t best = min(min(min(ka.x, ka.y), min(ka.z, ka.w)),
                              min(min(kb.x, kb.y), min(kb.z, kb.w)));
    // (kNoKey's node field is past n: read node 0's words instead)
    const uint32_t vl = (best >> 8) & 0xfffffu, vc = vl < n ? vl : 0u;
    const uint32_t pre = offs[vc];
    asm volatile("" ::: "memory");
    const uint32_t key = wave_min(best);
    if (key == kNoKey) {   // no uncovered column: the levels hold a solution
      if (TRACE) h = trace_node(h, depth, row_in, kNoneL, 0);
      status = MPLD_FEASIBLE;
      break;
    }
    uint32_t v = (key >> 8) & 0xfffffu;
    const uint32_t size = key >> 28;
    if (TRACE) h = trace_node(h, depth, row_in, v, size);
    uint32_t rows, offv, est, lane_lo, c;
    bool full;
    if (size != 0) {
      rows = key & 0xffu;
      offv = rdlane(pre, (v >> 5) & 63u);
      est = esp;
      lane_lo = 0u;
      full = false;
      c = (uint32_t)__builtin_ctz(rows);
      if (STITCH) {
        // the partner's color first when the partner is covered (its P bit
        // is clear) and that row of v is open
        const uint32_t p = uni((uint32_t)spart[v]);
        if (p != 0xffffu && !((uni(PL[(p >> 5) * S + K]) >> (p & 31u)) & 1u)) {
          const uint32_t cp = uni((uint32_t)scol[p]);
          if ((rows >> cp) & 1u) c = cp;
        }
      }
      rows &= ~(1u << c);   // the level's untried rows
    } else {
      // dead end: the headers and the log written so far must be visible
      // to this wave's loads: a workgroup-scope fence waits for the stores
      // (the workgroup's waves share the CU's write-through vector cache)
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      // back to the deepest level below `depth` whose column has an untried row
      uint32_t f = kNoneL;
      if (depth != 0) {
        const uint32_t d1 = depth - 1u, top = d1 >> 5;
        const uint32_t below = ~0u >> (31u - (d1 & 31u));
        for (uint32_t base = 0; base <= top && f == kNoneL; base += 64u) {
          // lane l looks at word top - base - l
          const bool in = base + lane <= top;
          const uint32_t wi = in ? top - base - lane : 0u;
          uint32_t m = in ? dbits[wi] : 0u;
          if (in && wi == top) m &= below;
          const uint64_t bal = __builtin_amdgcn_ballot_w64(m != 0u);
          if (bal) {
            const uint32_t l = (uint32_t)__builtin_ctzll(bal);
            f = (top - base - l) * 32u + 31u - (uint32_t)__builtin_clz(rdlane(m, l));
          }
        }
      }
      if (f == kNoneL) { status = MPLD_INFEASIBLE; break; }
      const uint2 hd = hdr[f];
      est = uni(hd.x);
      const uint32_t y = uni(hd.y);
      v = y & 0xffffu;
      offv = uni(offs[v]);
      // uncover every level above f, and the rows level f removed; the
      // column stays covered (its P bit is entry est); eight entries per
      // lane in flight at a time
      for (uint32_t i0 = est + 1u; i0 < esp; i0 += 64u * 8u) {
        uint32_t e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t i = i0 + 64u * (uint32_t)q + lane;
          e[q] = i < esp ? ent[i] : 0xffffffffu;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (e[q] != 0xffffffffu) {
            const uint32_t uu = e[q] & kNodeMask;
            atomicOr(&PL[(uu >> 5) * S + (e[q] >> kEntryNodeBits)], 1u << (uu & 31u));
          }
        }
      }
      // the next untried row of the level, in ascending order
      rows = (y >> 16) & 0xffu;
      c = (uint32_t)__builtin_ctz(rows);
      rows &= rows - 1u;
      depth = f;
      lane_lo = 1u;
      full = true;
    }
    take_row(v, c, rows, offv, est, lane_lo, rows != 0u, full);
    row_in = v * (uint32_t)K + c;
    ++depth;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __syncthreads();
  if (status == MPLD_FEASIBLE) {
    for (uint32_t f = lane; f < depth; f += 64) {
      const uint32_t y = hdr[f].y;
      colors[y & 0xffffu] = (int8_t)((y >> 24) & 0xfu);
    }
  } else {
    for (uint32_t v = lane; v < n; v += 64) colors[v] = -1;
  }
  rec->status = status;
  rec->depth = status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
  rec->nodes = nodes;
  rec->hash = h;
  __syncthreads();
}

// Big components: one workgroup of nw waves (nw = blockDim.x / 64).  Every
// wave scans its share of the plane words; the per-wave minima meet in LDS
// and each wave folds them, so all waves hold the same column choice.  The
// rest of the node (cover, backtrack, bookkeeping) is a few lanes of work
// and runs on wave 0 alone; a barrier ends the node, and wave 0 publishes
// the loop status (and the final depth) in LDS for the others.  Adjacency,
// level headers and the undo log are in global memory.
// root_row / task_budget: a subtree task, as for solve_lds.  STITCH: the
// stitch-aware row order, as for solve_lds (partners from the CSR block,
// the color of each covered node in LDS).  Level headers hold the rows
// not tried yet.
template <bool TRACE, int K, bool STITCH>
__device__ void solve_lds_wg(const DevDesc& d, const uint32_t* __restrict__ adj, char* lds,
                             uint64_t* gstack, int8_t* __restrict__ colors,
                             DevRecord* __restrict__ rec, int32_t root_row = -1,
                             uint64_t task_budget = 0) {
  const uint32_t tid = threadIdx.x, lane = __lane_id(), nthr = blockDim.x;
  const uint32_t wid = uni(tid >> 6), nw = nthr >> 6;
  const uint32_t n = (uint32_t)d.n;
  const uint32_t adj_words = uni(adj[n]) + n + 1u;
  const LdsLayout L = lds_layout((int32_t)n, K, adj_words, true, STITCH);
  const uint32_t W = L.W;
  uint64_t* PL = reinterpret_cast<uint64_t*>(lds + L.pl_off);
  uint64_t* A = reinterpret_cast<uint64_t*>(lds + L.a_off);
  uint8_t* scol = reinterpret_cast<uint8_t*>(lds + L.col_off);
  const uint32_t* gpart = adj + adj_words + 1u;   // STITCH: partner of each node
  uint32_t* red = reinterpret_cast<uint32_t*>(lds + L.ctl_off);   // per-wave minima
  int32_t* ctl = reinterpret_cast<int32_t*>(lds + L.ctl_off + 64);  // status, depth
  uint64_t* hdr = gstack;
  uint32_t* ent = reinterpret_cast<uint32_t*>(gstack + n);
  const uint32_t* ids = adj + n + 1;
  for (uint32_t w = tid; w < W; w += nthr) {
    const uint32_t cnt = n - w * 64u >= 64u ? 64u : n - w * 64u;
    const uint64_t val = cnt == 64u ? ~0ull : ((1ull << cnt) - 1ull);
#pragma unroll
    for (int c = 0; c <= K; ++c) PL[(uint32_t)c * W + w] = val;
    A[w] = 0ull;
  }
  if (tid == 0) ctl[0] = -1;   // budget >= 1: the root always counts
  __syncthreads();

  // search state, kept by wave 0
  uint32_t depth = 0, row_in = kNoneL, esp = 0;
  uint64_t nodes = 1, h = 0;
  int32_t status = -1;
  const uint64_t budget = root_row >= 0 ? task_budget : (uint64_t)d.budget;
  if (root_row >= 0) {
    // wave 0 takes row (0, root_row) at depth 0 (A's bit for level 0 stays
    // clear); `nodes` = 1 then counts the first node below it
    if (wid == 0u) {
      const uint32_t c = (uint32_t)root_row;
      const uint32_t beg = uni(adj[0]), deg = uni(adj[1]) - beg;
      if (lane == 63u) {
        ent[0] = (uint32_t)K << kEntryNodeBits;
        atomicAnd(reinterpret_cast<unsigned long long*>(&PL[(uint32_t)K * W]), ~1ull);
        hdr[0] = make_hdr(0u, c, 0u, 0u);   // no other row at this level
        if (STITCH) scol[0] = (uint8_t)c;
      }
      esp = 1u;
      unsigned long long* plane = reinterpret_cast<unsigned long long*>(PL + c * W);
      for (uint32_t ch = 0; ch < deg; ch += 64u) {
        bool hit = false;
        uint32_t u = 0;
        if (ch + lane < deg) {
          u = ids[beg + ch + lane];
          const uint64_t bit = 1ull << (u & 63u);
          hit = (atomicAnd(&plane[u >> 6], ~bit) & bit) != 0ull;
        }
        const uint64_t bal = __ballot(hit);
        if (hit) {
          const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          ent[esp + rank] = (c << kEntryNodeBits) | u;
        }
        esp += (uint32_t)__popcll(bal);
      }
      depth = 1u;
      row_in = c;
    }
    __syncthreads();
  }

  while (ctl[0] < 0) {
    uint32_t key = kNoKey;
    for (uint32_t w = tid; w < W; w += nthr) key = min(key, word_key<K>(PL, W, w));
    key = wave_min(key);
    if (nw > 1u) {
      if (lane == 63u) red[wid] = key;
      __syncthreads();
      key = wave_min(lane < nw ? red[lane] : kNoKey);
    }
    if (wid == 0u) {
      if (key == kNoKey) {   // no uncovered column: the levels hold a solution
        if (TRACE) h = trace_node(h, depth, row_in, kNoneL, 0);
        status = MPLD_FEASIBLE;
      } else {
        uint32_t v = key & 0xffffffu;
        const uint32_t size = key >> 24;
        if (TRACE) h = trace_node(h, depth, row_in, v, size);
        uint32_t c = 0, rows = 0, est = 0, beg = 0, deg = 0;
        if (size != 0) {
          const uint32_t b0 = adj[v], b1 = adj[v + 1];
          uint32_t r = 0;
#pragma unroll
          for (int j = 0; j < K; ++j) r |= (uint32_t)((PL[(uint32_t)j * W + (v >> 6)] >> (v & 63u)) & 1ull) << j;
          beg = uni(b0);
          deg = uni(b1) - beg;
          rows = uni(r);
          c = (uint32_t)__builtin_ctz(rows);
          if (STITCH) {
            // the partner's color first when the partner is covered and
            // that row of v is open
            const uint32_t p = uni(gpart[v]);
            if (p < n && !((uni64(PL[(uint32_t)K * W + (p >> 6)]) >> (p & 63u)) & 1ull)) {
              const uint32_t cp = uni((uint32_t)scol[p]);
              if ((rows >> cp) & 1u) c = cp;
            }
          }
          rows &= ~(1u << c);   // the level's untried rows
          est = esp;
          if (lane == 63u) {
            ent[est] = ((uint32_t)K << kEntryNodeBits) | v;
            atomicAnd(reinterpret_cast<unsigned long long*>(&PL[(uint32_t)K * W + (v >> 6)]),
                      ~(1ull << (v & 63u)));
          }
          esp = est + 1u;
        } else {
          // dead end: back to the deepest level whose column has an untried row
          uint32_t f = kNoneL;
          if (depth != 0) {
            const uint32_t d1 = depth - 1u;
            uint32_t aw = d1 >> 6;
            uint64_t bits = uni64(A[aw]) & (~0ull >> (63u - (d1 & 63u)));
            while (bits == 0ull && aw != 0u) bits = uni64(A[--aw]);
            if (bits) f = aw * 64u + 63u - (uint32_t)__builtin_clzll(bits);
          }
          if (f == kNoneL) {
            status = MPLD_INFEASIBLE;
          } else {
            const uint64_t hd = uni64(hdr[f]);
            v = (uint32_t)hd & 0xffffffu;
            rows = (uint32_t)(hd >> 28) & 0xffu;   // untried rows, next in ascending order
            est = (uint32_t)(hd >> 36);
            beg = uni(adj[v]);
            deg = uni(adj[v + 1]) - beg;
            // uncover every level above f, and the rows level f removed
            for (uint32_t i = est + 1u + lane; i < esp; i += 64) {
              const uint32_t e = ent[i];
              const uint32_t u = e & ((1u << kEntryNodeBits) - 1u);
              atomicOr(reinterpret_cast<unsigned long long*>(&PL[(e >> kEntryNodeBits) * W + (u >> 6)]),
                       1ull << (u & 63u));
            }
            c = (uint32_t)__builtin_ctz(rows);
            rows &= rows - 1u;
            depth = f;
            esp = est + 1u;
          }
        }
        if (status < 0) {
          // include row (v, c) at this depth
          if (lane == 63u) {
            hdr[depth] = make_hdr(v, c, rows, est);
            if (STITCH) scol[v] = (uint8_t)c;
            const uint64_t bit = 1ull << (depth & 63u);
            if (rows != 0u) atomicOr(reinterpret_cast<unsigned long long*>(&A[depth >> 6]), bit);
            else atomicAnd(reinterpret_cast<unsigned long long*>(&A[depth >> 6]), ~bit);
          }
          unsigned long long* plane = reinterpret_cast<unsigned long long*>(PL + c * W);
          for (uint32_t ch = 0; ch < deg; ch += 64u) {
            bool hit = false;
            uint32_t u = 0;
            if (ch + lane < deg) {
              u = ids[beg + ch + lane];
              const uint64_t bit = 1ull << (u & 63u);
              hit = (atomicAnd(&plane[u >> 6], ~bit) & bit) != 0ull;
            }
            const uint64_t bal = __ballot(hit);
            if (hit) {
              const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
              ent[esp + rank] = (c << kEntryNodeBits) | u;
            }
            esp += (uint32_t)__popcll(bal);
          }
          ++depth;
          row_in = v * (uint32_t)K + c;
          // the next node, if the budget allows it
          if (nodes == budget) status = MPLD_BUDGET_EXHAUSTED;
          else ++nodes;
        }
      }
      if (lane == 63u) {
        ctl[0] = status;
        ctl[1] = (int32_t)depth;
      }
    }
    __syncthreads();
  }
  const int32_t fin = ctl[0];
  const uint32_t fdepth = (uint32_t)ctl[1];
  if (fin == MPLD_FEASIBLE) {
    for (uint32_t f = tid; f < fdepth; f += nthr) {
      const uint64_t hd = hdr[f];
      colors[(uint32_t)hd & 0xffffffu] = (int8_t)((hd >> 24) & 0xfu);
    }
  } else {
    for (uint32_t v = tid; v < n; v += nthr) colors[v] = -1;
  }
  if (wid == 0u) {   // uniform record from every lane of wave 0
    rec->status = status;
    rec->depth = status == MPLD_INFEASIBLE ? 0 : (int32_t)depth;
    rec->nodes = nodes;
    rec->hash = h;
  }
  __syncthreads();
}

template <bool TRACE, bool BIG, bool STITCH>
__device__ __forceinline__ void solve_lds_k(const DevDesc& d, const uint32_t* gadj, char* lds,
                                            uint64_t* gstack, int8_t* colors, DevRecord* rec,
                                            uint32_t wide, int32_t root_row = -1,
                                            uint64_t task_budget = 0) {
#define MPLD_LDS_CASE(KK)                                                                     \
  case KK:                                                                                    \
    if (BIG && KK <= kWideMaxK && wide) solve_lds_wide<TRACE, (KK <= kWideMaxK ? KK : 2), STITCH>(d, gadj, lds, gstack, colors, rec, root_row, task_budget); \
    else if (BIG) solve_lds_wg<TRACE, KK, STITCH>(d, gadj, lds, gstack, colors, rec, root_row, task_budget); \
    else solve_lds<TRACE, KK, STITCH>(d, gadj, lds, colors, rec, root_row, task_budget);     \
    break;
  switch (d.k) {
    MPLD_LDS_CASE(2)
    MPLD_LDS_CASE(3)
    MPLD_LDS_CASE(4)
    MPLD_LDS_CASE(5)
    MPLD_LDS_CASE(6)
    MPLD_LDS_CASE(7)
    default:
      if (BIG && wide) solve_lds_wide<TRACE, 8, STITCH>(d, gadj, lds, gstack, colors, rec, root_row, task_budget);
      else if (BIG) solve_lds_wg<TRACE, 8, STITCH>(d, gadj, lds, gstack, colors, rec, root_row, task_budget);
      else solve_lds<TRACE, 8, STITCH>(d, gadj, lds, colors, rec, root_row, task_budget);
      break;
  }
#undef MPLD_LDS_CASE
}

// Persistent kernel, one workgroup per component (one wave for small
// components, nw waves for big ones); work distribution as in the register
// tier: static first item, then atomic pops by one thread, the last pop
// resets the counter.
template <bool TRACE, bool BIG, bool STITCH>
__global__ __launch_bounds__(BIG ? 1024 : 64) void lds_batched_kernel(
    const DevDesc* __restrict__ descs, const uint32_t* __restrict__ adj32, int32_t qlen,
    int32_t* __restrict__ counter, uint64_t* gstack, uint64_t stack_words_per_wave,
    DevRecord* __restrict__ recs, int8_t* __restrict__ colors, uint32_t wide) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* my_stack = BIG ? gstack + (uint64_t)blockIdx.x * stack_words_per_wave : nullptr;
  const int32_t gw = (int32_t)gridDim.x;
  int32_t item = (int32_t)uni(blockIdx.x);
  while (item < qlen) {
    const DevDesc d = descs[item];
    solve_lds_k<TRACE, BIG, STITCH>(d, adj32 + d.nbr_off, lds, my_stack, colors + d.out_off, recs + d.comp,
                                    wide);
    if (gw >= qlen) break;
    int32_t r = 0;
    if constexpr (BIG) {   // one pop per workgroup, shared through LDS
      int32_t* popped = reinterpret_cast<int32_t*>(lds);
      if (threadIdx.x == 0) *popped = atomicAdd(counter, 1);
      __syncthreads();
      r = (int32_t)uni((uint32_t)*popped);
      __syncthreads();
    } else {
      if (__lane_id() == 0) r = atomicAdd(counter, 1);
      r = (int32_t)uni((uint32_t)r);
    }
    item = gw + r;
    if (r == qlen - 1 && threadIdx.x == 0) atomicExch(counter, 0);
  }
}

template <bool TRACE, bool BIG, bool STITCH>
__global__ __launch_bounds__(BIG ? 1024 : 64) void lds_single_kernel(
    const DevDesc* __restrict__ descs, const uint32_t* __restrict__ adj32, int32_t item,
    uint64_t* gstack, DevRecord* __restrict__ recs, int8_t* __restrict__ colors, uint32_t wide) {
  extern __shared__ __align__(16) char lds[];
  const DevDesc d = descs[item];
  solve_lds_k<TRACE, BIG, STITCH>(d, adj32 + d.nbr_off, lds, gstack, colors + d.out_off, recs + d.comp,
                                  wide);
}

// Subtree tasks of the heavy-component split: task t searches the subtree
// of root row tasks[t].row of component tasks[t].item with its own budget,
// and writes its record (with TRACE, the trace hash of its own nodes) to
// task_recs[t] and its colors to task_colors + tasks[t].col_off.  Grid-stride over the tasks, one
// workgroup each (one wave small, nw waves big; big ones use the block's
// stack area).
template <bool TRACE, bool BIG, bool STITCH>
__global__ __launch_bounds__(BIG ? 1024 : 64) void lds_task_kernel(
    const DevDesc* __restrict__ descs, const uint32_t* __restrict__ adj32,
    const LdsTask* __restrict__ tasks, int32_t ntasks, uint64_t* gstack,
    uint64_t stack_words_per_block, DevRecord* __restrict__ task_recs,
    int8_t* __restrict__ task_colors, uint32_t wide) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* my_stack = BIG ? gstack + (uint64_t)blockIdx.x * stack_words_per_block : nullptr;
  for (int32_t t = (int32_t)uni(blockIdx.x); t < ntasks; t += (int32_t)gridDim.x) {
    const LdsTask task = tasks[t];
    const DevDesc d = descs[task.item];
    solve_lds_k<TRACE, BIG, STITCH>(d, adj32 + d.nbr_off, lds, my_stack, task_colors + task.col_off,
                                    task_recs + t, wide, task.row, (uint64_t)task.budget);
  }
}

// Conflict marking (Algorithm 1: a column left with no related row is a
// conflict candidate (cl, cl'), cl' the column whose cover removed cl's
// final row) for a component whose search ended without a solution: one
// descent of the search that never backtracks.  Same column rule and plane
// scan as the search; the column takes its lowest open color, or, with no
// row left, the color it lost last (last[u] in LDS, written by the lane
// whose atomic AND removed u's row).  One wave; adjacency from global
// memory; LDS holds the planes and last[].  Every node is colored.
template <int K>
__device__ void mark_csr(const DevDesc& d, const uint32_t* __restrict__ adj, char* lds,
                         int8_t* __restrict__ colors) {
  const uint32_t lane = __lane_id();
  const uint32_t n = (uint32_t)d.n, W = (n + 63u) / 64u;
  uint64_t* PL = reinterpret_cast<uint64_t*>(lds);
  uint8_t* last = reinterpret_cast<uint8_t*>(PL + (uint32_t)(K + 1) * W);
  const uint32_t* ids = adj + n + 1;
  for (uint32_t w = lane; w < W; w += 64) {
    const uint32_t cnt = n - w * 64u >= 64u ? 64u : n - w * 64u;
    const uint64_t val = cnt == 64u ? ~0ull : ((1ull << cnt) - 1ull);
#pragma unroll
    for (int c = 0; c <= K; ++c) PL[(uint32_t)c * W + w] = val;
  }
  __syncthreads();
  for (;;) {
    uint32_t key = kNoKey;
    for (uint32_t w = lane; w < W; w += 64) key = min(key, word_key<K>(PL, W, w));
    key = wave_min(key);
    if (key == kNoKey) break;
    const uint32_t v = key & 0xffffffu;
    uint32_t c;
    if ((key >> 24) != 0u) {
      uint32_t r = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) r |= (uint32_t)((PL[(uint32_t)j * W + (v >> 6)] >> (v & 63u)) & 1ull) << j;
      c = (uint32_t)__builtin_ctz(uni(r));
    } else {
      c = uni(last[v]);
    }
    if (lane == 63u) {
      colors[v] = (int8_t)c;
      atomicAnd(reinterpret_cast<unsigned long long*>(&PL[(uint32_t)K * W + (v >> 6)]),
                ~(1ull << (v & 63u)));
    }
    const uint32_t beg = uni(adj[v]), deg = uni(adj[v + 1]) - beg;
    unsigned long long* plane = reinterpret_cast<unsigned long long*>(PL + c * W);
    for (uint32_t j = lane; j < deg; j += 64u) {
      const uint32_t u = ids[beg + j];
      const uint64_t bit = 1ull << (u & 63u);
      if (atomicAnd(&plane[u >> 6], ~bit) & bit) last[u] = (uint8_t)c;
    }
    __syncthreads();
  }
  __syncthreads();
}

// One wave per workgroup over the components of the LDS, big and
// device-wide tiers; components whose record is FEASIBLE keep the search's
// colors.
__global__ __launch_bounds__(64) void mark_lds_kernel(const DevDesc* __restrict__ descs,
                                                      const uint32_t* __restrict__ adj32,
                                                      int32_t qlen,
                                                      const DevRecord* __restrict__ recs,
                                                      int8_t* __restrict__ colors) {
  extern __shared__ __align__(16) char lds[];
  for (int32_t i = (int32_t)uni(blockIdx.x); i < qlen; i += (int32_t)gridDim.x) {
    const DevDesc d = descs[i];
    if ((int32_t)uni((uint32_t)recs[d.comp].status) == MPLD_FEASIBLE) continue;
    const uint32_t* adj = adj32 + d.nbr_off;
    int8_t* out = colors + d.out_off;
    switch (d.k) {
      case 2: mark_csr<2>(d, adj, lds, out); break;
      case 3: mark_csr<3>(d, adj, lds, out); break;
      case 4: mark_csr<4>(d, adj, lds, out); break;
      case 5: mark_csr<5>(d, adj, lds, out); break;
      case 6: mark_csr<6>(d, adj, lds, out); break;
      case 7: mark_csr<7>(d, adj, lds, out); break;
      default: mark_csr<8>(d, adj, lds, out); break;
    }
  }
}

// ---- host side --------------------------------------------------------------

int64_t lds_bytes_for(int32_t n, int32_t k, int64_t adj_words, int32_t max_deg, bool big,
                      bool stitch) {
  // adj_words: row offsets + neighbour ids (n + 1 + 2m)
  (void)max_deg;
  return big ? (int64_t)lds_layout(n, k, adj_words, true, stitch).total
             : (int64_t)lds1_layout(n, k, adj_words, stitch).total;
}

int64_t lds_wide_bytes(int32_t n, int32_t k, int64_t adj_words, int32_t max_deg, bool stitch) {
  // -1: the one-wave wide layout does not apply (too many nodes, or ids or
  // degrees beyond its offs fields)
  const int64_t m2 = adj_words - n - 1;
  if (k > kWideMaxK || n > kWideMaxN || m2 >= (int64_t)1 << kWideBegBits ||
      (int64_t)max_deg >= (int64_t)1 << (32 - kWideBegBits))
    return -1;
  return (int64_t)wide_layout(n, k, adj_words, stitch).total;
}

int64_t lds_stack_words(int32_t n, int32_t k, int64_t adj_words) {
  // level headers (one u64 per depth) and the undo log (u32 entries)
  return (int64_t)n + ((int64_t)lds_log_entries(n, k, adj_words) + 1) / 2;
}
template <bool TRACE, bool BIG, bool STITCH>
static void lds_attr(int bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_batched_kernel<TRACE, BIG, STITCH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_single_kernel<TRACE, BIG, STITCH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_task_kernel<TRACE, BIG, STITCH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

int64_t mark_lds_bytes(int32_t n, int32_t k) {
  // planes (k + 1 words of 64 nodes each) and one byte per node
  const int64_t W = ((int64_t)n + 63) / 64;
  return (8 * (int64_t)(k + 1) * W + (int64_t)n + 7) & ~(int64_t)7;
}

hipError_t launch_mark_lds(int grid, int lds_bytes, const DevDesc* descs, const uint32_t* adj32,
                           int32_t qlen, const DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  hipLaunchKernelGGL(mark_lds_kernel, dim3(grid), dim3(64), (size_t)lds_bytes, s, descs, adj32,
                     qlen, recs, colors);
  return hipGetLastError();
}

void lds_configure(int bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&mark_lds_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  lds_attr<true, true, false>(bytes);
  lds_attr<true, false, false>(bytes);
  lds_attr<false, true, false>(bytes);
  lds_attr<false, false, false>(bytes);
  lds_attr<true, true, true>(bytes);
  lds_attr<true, false, true>(bytes);
  lds_attr<false, true, true>(bytes);
  lds_attr<false, false, true>(bytes);
  (void)hipGetLastError();
}

int lds_big_waves(int32_t max_n) {
  // one plane word per lane of the workgroup, at most 16 waves
  const int32_t words = (max_n + 63) / 64;
  const int32_t w = (words + 63) / 64;
  return w < 1 ? 1 : (w > 16 ? 16 : w);
}

// Calls f(trace, big, stitch) with each flag as a std::integral_constant,
// so that the launch names the matching kernel instantiation.
template <typename F>
static hipError_t lds_dispatch(bool trace, bool big, bool stitch, F&& f) {
  auto with_stitch = [&](auto t, auto g) {
    if (stitch) f(t, g, std::true_type{});
    else f(t, g, std::false_type{});
  };
  auto with_big = [&](auto t) {
    if (big) with_stitch(t, std::true_type{});
    else with_stitch(t, std::false_type{});
  };
  if (trace) with_big(std::true_type{});
  else with_big(std::false_type{});
  return hipGetLastError();
}

hipError_t launch_lds_batched(bool trace, bool big, bool stitch, int waves, int grid,
                              int lds_bytes, const DevDesc* descs, const uint32_t* adj32,
                              int32_t qlen, int32_t* counter, uint64_t* gstack,
                              uint64_t stack_words, DevRecord* recs, int8_t* colors,
                              hipStream_t s) {
  if (qlen <= 0) return hipSuccess;
  if (waves < 0 || waves > 16 || (!big && waves != 1)) return hipErrorInvalidValue;
  const uint32_t wide = waves == 0 ? 1u : 0u;   // big tier, one wave, wide layout
  return lds_dispatch(trace, big, stitch, [&](auto t, auto g, auto st) {
    hipLaunchKernelGGL((lds_batched_kernel<decltype(t)::value, decltype(g)::value, decltype(st)::value>),
                       dim3(grid), dim3(64 * (wide ? 1 : waves)), (size_t)lds_bytes, s, descs, adj32,
                       qlen, counter, gstack, stack_words, recs, colors, wide);
  });
}

hipError_t launch_lds_tasks(bool trace, bool big, bool stitch, int waves, int grid, int lds_bytes,
                            const DevDesc* descs, const uint32_t* adj32, const LdsTask* tasks,
                            int32_t ntasks, uint64_t* gstack, uint64_t stack_words,
                            DevRecord* task_recs, int8_t* task_colors, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (waves < 0 || waves > 16 || (!big && waves != 1) || grid < 1) return hipErrorInvalidValue;
  const uint32_t wide = waves == 0 ? 1u : 0u;   // big tier, one wave, wide layout
  return lds_dispatch(trace, big, stitch, [&](auto t, auto g, auto st) {
    hipLaunchKernelGGL((lds_task_kernel<decltype(t)::value, decltype(g)::value, decltype(st)::value>),
                       dim3(grid), dim3(64 * (wide ? 1 : waves)), (size_t)lds_bytes, s, descs, adj32,
                       tasks, ntasks, gstack, stack_words, task_recs, task_colors, wide);
  });
}

// One workgroup per resolved component: its colors and record.
__global__ __launch_bounds__(256) void csr_writeback_kernel(const LdsResolved* __restrict__ w,
                                                            int32_t count, const int8_t* __restrict__ src,
                                                            DevRecord* __restrict__ recs,
                                                            int8_t* __restrict__ colors) {
  for (int32_t i = (int32_t)blockIdx.x; i < count; i += (int32_t)gridDim.x) {
    const LdsResolved r = w[i];
    for (int32_t v = (int32_t)threadIdx.x; v < r.n; v += (int32_t)blockDim.x)
      colors[r.out_off + v] = r.src_off >= 0 ? src[r.src_off + v] : (int8_t)-1;
    if (threadIdx.x == 0) recs[r.comp] = r.rec;
  }
}

hipError_t launch_csr_writeback(const LdsResolved* w, int32_t count, const int8_t* src,
                                DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(csr_writeback_kernel, dim3(count < 1024 ? count : 1024), dim3(256), 0, s, w,
                     count, src, recs, colors);
  return hipGetLastError();
}

hipError_t launch_lds_single(bool trace, bool big, bool stitch, int waves, int lds_bytes,
                             const DevDesc* descs, const uint32_t* adj32, int32_t item,
                             uint64_t* gstack, DevRecord* recs, int8_t* colors, hipStream_t s) {
  if (waves < 0 || waves > 16 || (!big && waves != 1)) return hipErrorInvalidValue;
  const uint32_t wide = waves == 0 ? 1u : 0u;   // big tier, one wave, wide layout
  return lds_dispatch(trace, big, stitch, [&](auto t, auto g, auto st) {
    hipLaunchKernelGGL((lds_single_kernel<decltype(t)::value, decltype(g)::value, decltype(st)::value>),
                       dim3(1), dim3(64 * (wide ? 1 : waves)), (size_t)lds_bytes, s, descs, adj32,
                       item, gstack, recs, colors, wide);
  });
}

}  // namespace mpld
