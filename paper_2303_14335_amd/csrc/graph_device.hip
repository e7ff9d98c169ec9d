// graph_device.hip - the layout graph (Sec. 2.1: a conflict edge joins two
// features closer than d_min) built on the device, for requests large
// enough that the host's pair search dominates their front-end latency.
//
// The host validates the rectangles, applies the midpoint stitch split and
// picks the search grid (prepare_layout, shared with the host builder); the
// device then
//   1. counts the nodes per grid cell (atomics), scans the counts into cell
//      starts, and scatters node ids and boxes into cell order;
//   2. gives every node one thread that tests the nodes of its 3x3 cell
//      neighbourhood (three contiguous runs of the cell order) with the
//      closed-box gap test, skipping its own stitch partner, and counts its
//      neighbours; a scan of the counts gives the CSR row offsets;
//   3. repeats the test writing the neighbour ids, and sorts each node's
//      list in place (lists are short: the graph is a unit-disk-like
//      geometric graph).
// The result is the CSR the rest of the front-end consumes: adjacency
// ascending per node, symmetric, no self loops or duplicates by
// construction.  Scans are three-phase (per-block sums, one block over the
// sums, per-block scan plus offset).
//
// The simplification and sub-graph split that follow (Sec. 2.2; Algorithm 1
// splits the graph into sub-graphs) can run here too, on the CSR while it is
// still on the device: the split kernels reproduce the host's FIFO peeling
// order, components ordered by smallest id and BFS local numbering exactly,
// level by level (see the comment above them).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "runtime.h"

namespace mpld {

static constexpr int kScanBlock = 256;               // threads per scan block
static constexpr int kScanItems = 4;                 // elements per thread
static constexpr int kScanTile = kScanBlock * kScanItems;

struct GridParams {
  int64_t minx, miny, cell;
  int32_t gx, gy;
};

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ int32_t cell_index(const int4 b, const GridParams& g) {
  const int64_t cx = ((int64_t)b.x - g.minx) / g.cell, cy = ((int64_t)b.y - g.miny) / g.cell;
  return (int32_t)(cy * g.gx + cx);
}

__global__ __launch_bounds__(256) void cell_count_kernel(const int4* __restrict__ box, int32_t nn,
                                                         GridParams g, int32_t* __restrict__ cell_of,
                                                         int32_t* __restrict__ cnt) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= nn) return;
  const int32_t c = cell_index(box[i], g);
  cell_of[i] = c;
  atomicAdd(&cnt[c], 1);
}

// Scan phase 1: sum of each tile of kScanTile elements.
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(const int32_t* __restrict__ in,
                                                               int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t red[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) s += base + j < n ? in[base + j] : 0;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

// Exclusive scan of one block's kScanTile elements starting at `carry`.
__device__ void block_scan_tile(const int32_t* __restrict__ in, int64_t n, int64_t base_tile,
                                int32_t carry, int32_t* __restrict__ out, int32_t* lds) {
  const int64_t base = base_tile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems], s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele over the block's per-thread sums
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int32_t t = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
    __syncthreads();
    lds[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = carry + lds[threadIdx.x] - s;   // exclusive prefix of this thread
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  __syncthreads();
}

// Scan phase 2: exclusive scan of the tile sums (one block, looping), and
// the grand total at sums_out[ntiles].
__global__ __launch_bounds__(kScanBlock) void scan_tiles_kernel(const int32_t* __restrict__ sums,
                                                                int64_t ntiles,
                                                                int32_t* __restrict__ sums_out) {
  __shared__ int32_t lds[kScanBlock];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t t0 = 0; t0 < ntiles; t0 += kScanTile) {
    const int32_t c = carry;
    block_scan_tile(sums, ntiles, t0, c, sums_out, lds);
    if (threadIdx.x == kScanBlock - 1) {
      const int64_t last = std::min<int64_t>(t0 + kScanTile, ntiles) - 1;
      carry = sums_out[last] + sums[last];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sums_out[ntiles] = carry;
}

// Scan phase 3: each tile scanned from its offset; out[n] = total.
__global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(const int32_t* __restrict__ in,
                                                                int64_t n,
                                                                const int32_t* __restrict__ offs,
                                                                int64_t ntiles,
                                                                int32_t* __restrict__ out) {
  __shared__ int32_t lds[kScanBlock];
  block_scan_tile(in, n, (int64_t)blockIdx.x * kScanTile, offs[blockIdx.x], out, lds);
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[ntiles];
}

__global__ __launch_bounds__(256) void cell_scatter_kernel(const int4* __restrict__ box,
                                                           const int32_t* __restrict__ partner,
                                                           int32_t nn,
                                                           const int32_t* __restrict__ cell_of,
                                                           int32_t* __restrict__ fill,
                                                           int32_t* __restrict__ ids,
                                                           int4* __restrict__ sbox,
                                                           int32_t* __restrict__ smate) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= nn) return;
  const int32_t pos = atomicAdd(&fill[cell_of[i]], 1);
  ids[pos] = i;
  sbox[pos] = box[i];
  smate[pos] = partner[i];
}

// One thread per node (cell order): test the 3x3 cell neighbourhood.  WRITE
// = false counts the neighbours into deg[id]; WRITE = true writes them at
// adj[ptr[id]] and sorts the list.
template <bool WRITE>
__global__ __launch_bounds__(256) void neighbours_kernel(
    const int4* __restrict__ sbox, const int32_t* __restrict__ ids,
    const int32_t* __restrict__ smate, const int32_t* __restrict__ start, int32_t nn,
    GridParams g, int64_t d2, int32_t* __restrict__ deg, const int32_t* __restrict__ ptr,
    int32_t* __restrict__ adj) {
  const int32_t p = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= nn) return;
  const int4 a = sbox[p];
  const int32_t id = ids[p], mate = smate[p];
  const int64_t cx = ((int64_t)a.x - g.minx) / g.cell, cy = ((int64_t)a.y - g.miny) / g.cell;
  const int64_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx + 1 < g.gx ? cx + 1 : g.gx - 1;
  const int64_t y0 = cy > 0 ? cy - 1 : 0, y1 = cy + 1 < g.gy ? cy + 1 : g.gy - 1;
  int32_t k = 0;
  int32_t* out = WRITE ? adj + ptr[id] : nullptr;
  for (int64_t yy = y0; yy <= y1; ++yy) {
    const int32_t q0 = start[yy * g.gx + x0], q1 = start[yy * g.gx + x1 + 1];
    for (int32_t q = q0; q < q1; ++q) {
      if (q == p) continue;
      const int4 b = sbox[q];
      const int64_t dx = max(max((int64_t)0, (int64_t)b.x - a.z), (int64_t)a.x - b.z);
      const int64_t dy = max(max((int64_t)0, (int64_t)b.y - a.w), (int64_t)a.y - b.w);
      if (dx * dx + dy * dy >= d2) continue;
      const int32_t qid = ids[q];
      if (qid == mate) continue;   // the two halves of a split feature
      if (WRITE) out[k] = qid;
      ++k;
    }
  }
  if (!WRITE) {
    deg[id] = k;
  } else {
    for (int32_t i = 1; i < k; ++i) {   // insertion sort of the short list
      const int32_t x = out[i];
      int32_t j = i - 1;
      while (j >= 0 && out[j] > x) {
        out[j + 1] = out[j];
        --j;
      }
      out[j + 1] = x;
    }
  }
}


// ---- simplification and sub-graph split ------------------------------------
//
// The sequential definitions (FIFO peeling of nodes of conflict degree < k,
// queue seeded in ascending id, a popped node lowering its neighbours'
// degrees in ascending id; components of the rest ordered by smallest id;
// local numbering by BFS from that node, neighbours in ascending id) are
// reproduced exactly, in level-synchronous form:
//
// Peeling.  The queue falls into levels: level 0 is the seed; level L+1
// holds the nodes queued while level L is popped (the rounds of synchronous
// peeling).  A node w outside levels 0..L with deg0(w) = d is queued when
// its (d - k + 1)-th neighbour is popped; if that neighbour (its trigger) is
// in level L, it is the one of rank (d - k + 1 - before) among w's level-L
// neighbours by queue position, `before` counting w's neighbours in earlier
// levels.  Level L+1 is ordered by (trigger's queue position, w's place in
// the trigger's ascending list): one exclusive scan of per-trigger counts.
// Level 0 is ordered by id, so level 1's triggers need only the level-0
// flags: the wide levels 0 and 1 run on the whole device; the rest, usually
// small, on one workgroup whose rounds are separated by barriers.
//
// Components: union-find over the whole device, the larger root hooked
// under the smaller (so each root is its component's smallest id), numbered
// by root id with a scan.  BFS: one wave per component of at most 64 nodes
// (ranks by id, neighbour masks over the ranks, the queue kept in a lane
// register); larger components on one workgroup, level by level, a node's
// parent being its numbered neighbour of smallest local position.
constexpr int kSplitThreads = 1024;   // the one-workgroup kernels
constexpr int kSplitGrid = 2048;      // grid-stride kernels: blocks of 256

struct SplitArgs {
  int32_t n, k, simplify;
  const int32_t* ptr;   // n + 1 CSR offsets
  const int32_t* adj;   // ascending neighbour lists
  // outputs (one contiguous region)
  int32_t* counts;      // [0] removed, [1] components
  int32_t* queue;       // n: removal order
  int32_t* comp_of;     // n: component, -1 if removed
  int32_t* order;       // n: core nodes by component, local order
  int32_t* comp_ptr;    // n + 1
  int32_t* local;       // n: local index, -1 if removed
  // scratch: n each, pos0 / off0 / cid n + 1
  int32_t *f0, *pos0, *cnt0, *off0, *qpos, *lvl, *stamp, *trig, *cand, *parent, *root, *rflag,
      *cid, *csize, *fill, *list, *rank, *fa, *fb, *gex, *cnt, *cbase, *tail, *cntA, *cntB, *offL;
  int32_t* ctl;         // [2L], [2L+1]: queue range of level L (1 .. kWideLevels + 1)
};

// Peel levels 1 .. kWideLevels take their next level with device-wide
// launches; the one-workgroup kernel goes on from level kWideLevels + 1.
constexpr int kWideLevels = 4;

#define SPLIT_FOR(v, n)                                                                 \
  for (int32_t v = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); v < (n);          \
       v += (int32_t)(gridDim.x * blockDim.x))

__global__ __launch_bounds__(256) void split_init_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    a.f0[v] = a.simplify && a.ptr[v + 1] - a.ptr[v] < a.k ? 1 : 0;
    a.cnt0[v] = 0;
    a.cntA[v] = 0;
    a.cntB[v] = 0;
    a.csize[v] = 0;
    a.fill[v] = 0;
    a.qpos[v] = -1;
    a.lvl[v] = -1;
    a.stamp[v] = -1;
    a.trig[v] = -1;
    a.local[v] = -1;
    a.comp_of[v] = -1;
  }
}

// Level 0 in id order, and each other node's level-1 trigger: the
// (d - k + 1)-th level-0 neighbour in its ascending list (level-0 queue
// order is id order), counted per trigger.
__global__ __launch_bounds__(256) void split_level0_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    if (a.f0[v]) {
      const int32_t p = a.pos0[v];
      a.queue[p] = v;
      a.qpos[v] = p;
      a.lvl[v] = 0;
    } else if (a.simplify) {
      int32_t need = a.ptr[v + 1] - a.ptr[v] - a.k + 1;
      for (int32_t t = a.ptr[v]; t < a.ptr[v + 1]; ++t) {
        const int32_t x = a.adj[t];
        if (a.f0[x] && --need == 0) {
          a.trig[v] = x;
          atomicAdd(a.cnt0 + a.pos0[x], 1);
          break;
        }
      }
    }
  }
}

// Level 1: the children of level-0 node x go, in x's list order, at
// |level 0| + off0[position of x].
__global__ __launch_bounds__(256) void split_level1_kernel(SplitArgs a) {
  const int32_t base = a.pos0[a.n];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl[2] = base;
    a.ctl[3] = base + a.off0[a.n];
  }
  SPLIT_FOR(w, a.n) {
    const int32_t x = a.trig[w];
    if (x < 0) continue;
    int32_t r = 0;
    for (int32_t t = a.ptr[x]; t < a.ptr[x + 1]; ++t) {
      const int32_t y = a.adj[t];
      if (y >= w) break;
      r += !a.f0[y] && a.trig[y] == x ? 1 : 0;
    }
    const int32_t p = base + a.off0[a.qpos[x]] + r;
    if (p >= a.n) continue;   // cannot happen: positions are a permutation
    a.queue[p] = w;
    a.qpos[w] = p;
    a.lvl[w] = 1;
  }
}

// Wide level L (>= 1): the trigger of every unqueued node next to level L,
// counted per trigger at its position within the level.
__global__ __launch_bounds__(256) void split_trig_kernel(SplitArgs a, int32_t L, int32_t* cnt) {
  const int32_t lo = a.ctl[2 * L], hi = a.ctl[2 * L + 1];
  if (lo >= hi) return;
  SPLIT_FOR(w, a.n) {
    if (a.qpos[w] >= 0) continue;
    const int32_t t0 = a.ptr[w], t1 = a.ptr[w + 1];
    int32_t before = 0, at = 0;
    for (int32_t t = t0; t < t1; ++t) {
      const int32_t l = a.lvl[a.adj[t]];
      before += l >= 0 && l < L ? 1 : 0;
      at += l == L ? 1 : 0;
    }
    if (at == 0) continue;   // not next to level L: its trigger stays -1
    const int32_t need = t1 - t0 - a.k + 1;
    int32_t tr = -1;
    if (before + at >= need) {
      const int32_t rank = need - before - 1;   // among level-L neighbours by queue position
      for (int32_t t = t0; t < t1 && tr < 0; ++t) {
        const int32_t x = a.adj[t];
        if (a.lvl[x] != L) continue;
        const int32_t px = a.qpos[x];
        int32_t r = 0;
        for (int32_t q = t0; q < t1; ++q) {
          const int32_t y = a.adj[q];
          r += a.lvl[y] == L && a.qpos[y] < px ? 1 : 0;
        }
        if (r == rank) tr = x;
      }
    }
    a.trig[w] = tr;
    if (tr >= 0) atomicAdd(cnt + (a.qpos[tr] - lo), 1);
  }
}

// Wide level L: level L+1 in (trigger position, trigger's list order); the
// range of level L+1 goes to ctl, the other count array is cleared for it.
__global__ __launch_bounds__(256) void split_place_kernel(SplitArgs a, int32_t L,
                                                          const int32_t* off, int32_t* cnt_next) {
  const int32_t lo = a.ctl[2 * L], hi = a.ctl[2 * L + 1];
  SPLIT_FOR(v, a.n) cnt_next[v] = 0;
  const int32_t total = lo < hi ? off[a.n] : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl[2 * L + 2] = hi;
    a.ctl[2 * L + 3] = hi + total;
  }
  if (lo >= hi) return;
  SPLIT_FOR(w, a.n) {
    const int32_t x = a.trig[w];
    if (x < 0 || a.qpos[w] >= 0 || a.lvl[x] != L) continue;
    // x's children this level are exactly the y with trig[y] == x
    int32_t r = 0;
    for (int32_t t = a.ptr[x]; t < a.ptr[x + 1]; ++t) {
      const int32_t y = a.adj[t];
      if (y >= w) break;
      r += a.trig[y] == x ? 1 : 0;
    }
    const int32_t p = hi + off[a.qpos[x] - lo] + r;
    if (p >= a.n) continue;   // cannot happen: positions are a permutation
    a.queue[p] = w;
    a.qpos[w] = p;
    a.lvl[w] = L + 1;
  }
}

// Exclusive prefix of x over the workgroup (16 waves); `total` = the sum.
__device__ __forceinline__ int32_t wg_excl_scan(int32_t x, int32_t* wsum, int32_t& total) {
  const int32_t lane = (int32_t)(threadIdx.x & 63u), w = (int32_t)(threadIdx.x >> 6);
  int32_t incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kSplitThreads / 64; ++i) {
    const int32_t v = wsum[i];
    before += i < w ? v : 0;
    tot += v;
  }
  __syncthreads();   // wsum is reused by the next scan
  total = tot;
  return before + incl - x;
}

// The remaining levels on one workgroup, from level kWideLevels + 1.
__global__ __launch_bounds__(kSplitThreads) void split_peel_kernel(SplitArgs a) {
  __shared__ int32_t wsum[kSplitThreads / 64];
  __shared__ int32_t ncand;
  const int32_t tid = (int32_t)threadIdx.x, T = kSplitThreads, n = a.n;
  const int32_t* __restrict__ ptr = a.ptr;
  const int32_t* __restrict__ adj = a.adj;
  int32_t lo = a.ctl[2 * (kWideLevels + 1)], hi = a.ctl[2 * (kWideLevels + 1) + 1];
  for (int32_t L = kWideLevels + 1; lo < hi; ++L) {
    // candidates: the unqueued neighbours of level L, each listed once
    if (tid == 0) ncand = 0;
    __syncthreads();
    for (int32_t i = lo + tid; i < hi; i += T) {
      const int32_t u = a.queue[i];
      for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
        const int32_t w = adj[t];
        if (a.qpos[w] < 0 && atomicMax(a.stamp + w, L) < L) a.cand[atomicAdd(&ncand, 1)] = w;
      }
    }
    __syncthreads();
    const int32_t nc = ncand;
    // trigger of each candidate in level L, or -1
    for (int32_t j = tid; j < nc; j += T) {
      const int32_t w = a.cand[j];
      const int32_t t0 = ptr[w], t1 = ptr[w + 1];
      const int32_t need = t1 - t0 - a.k + 1;
      int32_t before = 0, at = 0;
      for (int32_t t = t0; t < t1; ++t) {
        const int32_t l = a.lvl[adj[t]];
        before += l >= 0 && l < L ? 1 : 0;
        at += l == L ? 1 : 0;
      }
      int32_t tr = -1;
      if (before + at >= need) {
        const int32_t rank = need - before - 1;   // among level-L neighbours by queue position
        for (int32_t t = t0; t < t1 && tr < 0; ++t) {
          const int32_t x = adj[t];
          if (a.lvl[x] != L) continue;
          const int32_t px = a.qpos[x];
          int32_t r = 0;
          for (int32_t q = t0; q < t1; ++q) {
            const int32_t y = adj[q];
            r += a.lvl[y] == L && a.qpos[y] < px ? 1 : 0;
          }
          if (r == rank) tr = x;
        }
      }
      a.trig[w] = tr;
    }
    __syncthreads();
    // level L+1: each level-L node in queue order appends the nodes it
    // triggered, in its ascending list order
    int32_t next = hi;
    for (int32_t base = lo; base < hi; base += T) {
      const int32_t i = base + tid;
      const int32_t u = i < hi ? a.queue[i] : -1;
      int32_t c = 0;
      if (u >= 0)
        for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
          const int32_t w = adj[t];
          c += a.qpos[w] < 0 && a.trig[w] == u ? 1 : 0;
        }
      int32_t total;
      int32_t pos = next + wg_excl_scan(c, wsum, total);
      if (c)
        for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
          const int32_t w = adj[t];
          if (a.qpos[w] < 0 && a.trig[w] == u && pos < n) {
            a.queue[pos] = w;
            a.qpos[w] = pos;
            a.lvl[w] = L + 1;
            ++pos;
          }
        }
      next += total;
    }
    __syncthreads();
    lo = hi;
    hi = next;
  }
  if (tid == 0) a.counts[0] = hi;
}

__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving (parent[x] < x for every non-root, so every
// rewrite points x at one of its ancestors and the loop ends).
__device__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    const int32_t p = ld_agent(parent + x);
    if (p == x) return x;
    const int32_t g = ld_agent(parent + p);
    if (g == p) return p;
    __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = g;
  }
}

// Union-find start; the candidate stamps and triggers of the peeling are
// reset for the BFS of the big components.
__global__ __launch_bounds__(256) void uf_init_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    a.parent[v] = a.lvl[v] < 0 ? v : -1;
    a.stamp[v] = -1;
    a.trig[v] = -1;
  }
}

// Hooks the larger of two roots under the smaller; a failed CAS means that
// root was just hooked elsewhere: find again.
__global__ __launch_bounds__(256) void uf_unite_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    if (a.lvl[v] >= 0) continue;
    for (int32_t t = a.ptr[v]; t < a.ptr[v + 1]; ++t) {
      const int32_t w = a.adj[t];
      if (w < v || a.lvl[w] >= 0) continue;
      for (;;) {
        const int32_t ra = uf_find(a.parent, v), rb = uf_find(a.parent, w);
        if (ra == rb) break;
        const int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
        if (atomicCAS(a.parent + hi, hi, lo) == hi) break;
      }
    }
  }
}

// Every core node's root (read-only walks: the forest is final here) and
// the root flags to be numbered.
__global__ __launch_bounds__(256) void uf_root_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    int32_t r = -1;
    if (a.lvl[v] < 0) {
      r = v;
      for (int32_t p = a.parent[r]; p != r; p = a.parent[r]) r = p;
    }
    a.root[v] = r;
    a.rflag[v] = r == v ? 1 : 0;
  }
}

// Component of every core node (roots numbered in id order), its size, and
// the root of every component.
__global__ __launch_bounds__(256) void comp_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    const int32_t r = a.root[v];
    if (r < 0) continue;
    const int32_t c = a.cid[r];
    a.comp_of[v] = c;
    if (r == v) a.parent[c] = v;   // parent[] is free now: root of component c
    atomicAdd(a.csize + c, 1);
  }
}

// Core nodes listed per component (any order within it).
__global__ __launch_bounds__(256) void comp_list_kernel(SplitArgs a) {
  SPLIT_FOR(v, a.n) {
    const int32_t c = a.comp_of[v];
    if (c < 0) continue;
    a.list[a.comp_ptr[c] + atomicAdd(a.fill + c, 1)] = v;
  }
}

__device__ __forceinline__ uint64_t rdlane64(uint64_t x, uint32_t l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)l);
  return ((uint64_t)hi << 32) | lo;
}

// BFS numbering of the components of at most 64 nodes, one wave each.
// Lane i holds node x_i of the component; its rank by id is its index in
// the neighbour masks (rank 0 is the smallest id: the root).
__global__ __launch_bounds__(256) void bfs_small_kernel(SplitArgs a) {
  const int32_t lane = (int32_t)(threadIdx.x & 63u);
  const int32_t ncomp = a.cid[a.n];
  const int32_t waves = (int32_t)(gridDim.x * (blockDim.x >> 6));
  for (int32_t c = (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); c < ncomp;
       c += waves) {
    const int32_t base = a.comp_ptr[c], sz = a.comp_ptr[c + 1] - base;
    if (sz > 64) continue;
    const bool in = lane < sz;
    const int32_t x = in ? a.list[base + lane] : INT32_MAX;
    int32_t r = 0;
    for (int32_t j = 0; j < sz; ++j) r += __builtin_amdgcn_readlane(x, j) < x ? 1 : 0;
    if (in) a.rank[x] = r;
    __threadfence_block();
    uint64_t m = 0;
    if (in)
      for (int32_t t = a.ptr[x]; t < a.ptr[x + 1]; ++t) {
        const int32_t w = a.adj[t];
        if (a.comp_of[w] == c) m |= 1ull << a.rank[w];
      }
    // lane i's mask is indexed by its rank: mk[rank] via a lane shuffle
    const int32_t src = [&] {
      // the lane whose rank equals this lane's index
      int32_t s = 0;
      for (int32_t j = 0; j < sz; ++j)
        if (__builtin_amdgcn_readlane(r, j) == lane) s = j;
      return s;
    }();
    const uint32_t mlo = (uint32_t)__shfl((int)(uint32_t)m, src, 64);
    const uint32_t mhi = (uint32_t)__shfl((int)(uint32_t)(m >> 32), src, 64);
    const uint64_t mk = ((uint64_t)mhi << 32) | mlo;   // mask of rank `lane`
    // sequential BFS over ranks; q: lane t holds the rank at queue position t
    int32_t q = 0;
    uint64_t seen = 1ull;
    int32_t tail = 1;
    for (int32_t head = 0; head < tail; ++head) {
      const int32_t u = __builtin_amdgcn_readlane(q, head);
      uint64_t nb = rdlane64(mk, (uint32_t)u) & ~seen;
      seen |= nb;
      while (nb) {
        const int32_t b = (int32_t)__builtin_ctzll(nb);
        nb &= nb - 1;
        q = lane == tail ? b : q;
        ++tail;
      }
    }
    // the lane of rank q[t] is numbered t
    int32_t pos = -1;
    for (int32_t t = 0; t < sz; ++t)
      if (__builtin_amdgcn_readlane(q, t) == r) pos = t;
    if (in && pos >= 0) {
      a.local[x] = pos;
      a.order[base + pos] = x;
    }
  }
}

// BFS numbering of the components of more than 64 nodes, on one workgroup,
// all of them at once; the frontier stays ordered by (component, position).
__global__ __launch_bounds__(kSplitThreads) void bfs_big_kernel(SplitArgs a) {
  __shared__ int32_t wsum[kSplitThreads / 64];
  __shared__ int32_t ncand;
  const int32_t tid = (int32_t)threadIdx.x, T = kSplitThreads;
  const int32_t* __restrict__ ptr = a.ptr;
  const int32_t* __restrict__ adj = a.adj;
  const int32_t ncomp = a.cid[a.n];
  int32_t* F = a.fa;
  int32_t* NF = a.fb;
  // the roots of the big components, in component order
  int32_t fn = 0;
  for (int32_t base = 0; base < ncomp; base += T) {
    const int32_t c = base + tid;
    const int32_t big = c < ncomp && a.comp_ptr[c + 1] - a.comp_ptr[c] > 64 ? 1 : 0;
    int32_t total;
    const int32_t ex = wg_excl_scan(big, wsum, total);
    if (big) {
      const int32_t r = a.parent[c];
      F[fn + ex] = r;
      a.local[r] = 0;
      a.order[a.comp_ptr[c]] = r;
      a.tail[c] = 1;
    }
    fn += total;
  }
  __syncthreads();
  for (int32_t d = 0; fn > 0; ++d) {
    if (tid == 0) ncand = 0;
    __syncthreads();
    for (int32_t i = tid; i < fn; i += T) {
      const int32_t u = F[i];
      for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
        const int32_t w = adj[t];
        if (a.lvl[w] < 0 && a.local[w] < 0 && atomicMax(a.stamp + w, d) < d)
          a.cand[atomicAdd(&ncand, 1)] = w;
      }
    }
    __syncthreads();
    const int32_t nc = ncand;
    // parent: the numbered neighbour of smallest local position (all of
    // them are in level d)
    for (int32_t j = tid; j < nc; j += T) {
      const int32_t w = a.cand[j];
      int32_t best = -1, bp = INT32_MAX;
      for (int32_t t = ptr[w]; t < ptr[w + 1]; ++t) {
        const int32_t x = adj[t];
        const int32_t p = a.local[x];
        if (a.lvl[x] < 0 && p >= 0 && p < bp) {
          bp = p;
          best = x;
        }
      }
      a.trig[w] = best;
    }
    __syncthreads();
    int32_t carry = 0;
    for (int32_t base = 0; base < fn; base += T) {
      const int32_t i = base + tid;
      const int32_t u = i < fn ? F[i] : -1;
      int32_t c = 0;
      if (u >= 0)
        for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
          const int32_t w = adj[t];
          c += a.lvl[w] < 0 && a.local[w] < 0 && a.trig[w] == u ? 1 : 0;
        }
      int32_t total;
      const int32_t ex = carry + wg_excl_scan(c, wsum, total);
      if (u >= 0) {
        a.gex[i] = ex;
        a.cnt[i] = c;
        const int32_t cu = a.comp_of[u];
        if (i == 0 || a.comp_of[F[i - 1]] != cu) a.cbase[cu] = ex;
      }
      carry += total;
    }
    __syncthreads();
    for (int32_t i = tid; i < fn; i += T) {
      if (a.cnt[i] == 0) continue;
      const int32_t u = F[i], cu = a.comp_of[u];
      int32_t p = a.tail[cu] + a.gex[i] - a.cbase[cu], g = a.gex[i];
      for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
        const int32_t w = adj[t];
        if (a.lvl[w] < 0 && a.local[w] < 0 && a.trig[w] == u && g < a.n &&
            a.comp_ptr[cu] + p < a.comp_ptr[cu + 1]) {
          a.local[w] = p;
          a.order[a.comp_ptr[cu] + p] = w;
          NF[g] = w;
          ++p;
          ++g;
        }
      }
    }
    __syncthreads();
    for (int32_t i = tid; i < fn; i += T) {
      const int32_t cu = a.comp_of[F[i]];
      if (i == fn - 1 || a.comp_of[F[i + 1]] != cu) a.tail[cu] += a.gex[i] + a.cnt[i] - a.cbase[cu];
    }
    __syncthreads();
    int32_t* tmp = F;
    F = NF;
    NF = tmp;
    fn = carry;
  }
  if (tid == 0) a.counts[1] = ncomp;
}

// ---- host side --------------------------------------------------------------

struct GraphBuilder {
  mpld_context* ctx = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  DevBuf box, partner, cell_of, cnt, start, fill, ids, sbox, smate, deg, ptr, adj, sums, offs;
  DevBuf split_ws;   // split outputs then scratch (int32)
  PinnedBuf hin, hout;
  ~GraphBuilder() {
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

// Buffers grow geometrically: a reallocation (and, for pinned host memory,
// hipHostMalloc) costs milliseconds, so it should happen rarely.
static void grow(DevBuf& b, mpld_context* ctx, size_t bytes) {
  if (b.bytes < bytes) b.alloc(ctx, std::max(bytes + bytes / 4, 2 * b.bytes));
}
static bool grow_pinned(PinnedBuf& b, size_t bytes) {
  return bytes <= b.bytes || b.reserve(std::max(bytes + bytes / 4, 2 * b.bytes));
}

GraphBuilder* graph_builder_create(mpld_context* ctx, bool own_stream) {
  auto* gb = new GraphBuilder();
  gb->ctx = ctx;
  if (own_stream) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete gb;
      fail(MPLD_E_DEVICE, "hipStreamCreateWithFlags failed for the graph builder");
    }
    gb->stream = s;
    gb->own_stream = true;
  } else {
    gb->stream = ctx->stream;
  }
  return gb;
}

void graph_builder_destroy(GraphBuilder* gb) { delete gb; }


static void scan(GraphBuilder& gb, const int32_t* in, int64_t n, int32_t* out) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  grow(gb.sums, gb.ctx, sizeof(int32_t) * (size_t)(ntiles + 1));
  grow(gb.offs, gb.ctx, sizeof(int32_t) * (size_t)(ntiles + 1));
  hipStream_t s = gb.stream;
  hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, in, n,
                     gb.sums.as<int32_t>());
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(1), dim3(kScanBlock), 0, s, gb.sums.as<int32_t>(),
                     ntiles, gb.offs.as<int32_t>());
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, in, n,
                     gb.offs.as<int32_t>(), ntiles, out);
  check_hip(hipGetLastError(), "graph builder: scan");
}

// split_ws layout (int32): counts (2), queue, comp_of, order (n each),
// comp_ptr (n + 1), local (n) -- the part copied back, split_out_words(n)
// words -- then the scratch arrays, n + 1 words each.
static size_t split_out_words(int64_t n) { return 2 + 5 * (size_t)n + 1; }
static constexpr int kSplitScratch = 27;

// Enqueues the split of the CSR at dptr / dadj (device, int32); no host
// synchronisation.
static void enqueue_split(GraphBuilder& gb, int32_t n, const int32_t* dptr, const int32_t* dadj,
                          int32_t k, bool simplify) {
  const size_t nn = (size_t)n;
  const size_t stride = std::max<size_t>(nn + 1, 64);   // ctl needs 2 * (kWideLevels + 2)
  grow(gb.split_ws, gb.ctx, sizeof(int32_t) * (split_out_words(n) + kSplitScratch * stride));
  int32_t* w = gb.split_ws.as<int32_t>();
  SplitArgs a{};
  a.n = n;
  a.k = k;
  a.simplify = simplify ? 1 : 0;
  a.ptr = dptr;
  a.adj = dadj;
  a.counts = w;
  a.queue = w + 2;
  a.comp_of = a.queue + nn;
  a.order = a.comp_of + nn;
  a.comp_ptr = a.order + nn;
  a.local = a.comp_ptr + nn + 1;
  int32_t* q = a.local + nn;
  int32_t** scratch[kSplitScratch] = {&a.f0,   &a.pos0,  &a.cnt0, &a.off0,  &a.qpos,  &a.lvl,
                                      &a.stamp, &a.trig,  &a.cand, &a.parent, &a.root, &a.rflag,
                                      &a.cid,  &a.csize, &a.fill, &a.list,  &a.rank,  &a.fa,
                                      &a.fb,   &a.gex,   &a.cnt,  &a.cbase, &a.tail,
                                      &a.cntA, &a.cntB,  &a.offL, &a.ctl};
  for (int32_t** d : scratch) {
    *d = q;
    q += stride;
  }
  hipStream_t st = gb.stream;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, kSplitGrid);
  auto wide = [&](void (*kern)(SplitArgs)) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, a);
  };
  wide(split_init_kernel);
  scan(gb, a.f0, n, a.pos0);            // level-0 positions; pos0[n] = |level 0|
  wide(split_level0_kernel);
  scan(gb, a.cnt0, n, a.off0);          // level-1 offsets per level-0 position
  wide(split_level1_kernel);
  for (int32_t L = 1; L <= kWideLevels; ++L) {
    int32_t* cur = (L & 1) ? a.cntA : a.cntB;
    int32_t* nxt = (L & 1) ? a.cntB : a.cntA;
    hipLaunchKernelGGL(split_trig_kernel, dim3(grid), dim3(256), 0, st, a, L, cur);
    scan(gb, cur, n, a.offL);
    hipLaunchKernelGGL(split_place_kernel, dim3(grid), dim3(256), 0, st, a, L, a.offL, nxt);
  }
  hipLaunchKernelGGL(split_peel_kernel, dim3(1), dim3(kSplitThreads), 0, st, a);
  wide(uf_init_kernel);
  wide(uf_unite_kernel);
  wide(uf_root_kernel);
  scan(gb, a.rflag, n, a.cid);          // component ids; cid[n] = components
  wide(comp_kernel);
  scan(gb, a.csize, n, a.comp_ptr);
  wide(comp_list_kernel);
  wide(bfs_small_kernel);
  hipLaunchKernelGGL(bfs_big_kernel, dim3(1), dim3(kSplitThreads), 0, st, a);
  check_hip(hipGetLastError(), "device split");
}

// Split from the copied-back words of split_ws.
static void collect_split(const int32_t* h, int32_t n, Split& s) {
  const size_t nn = (size_t)n;
  const int32_t removed = h[0], ncomp = h[1];
  const int32_t* queue = h + 2;
  const int32_t* comp_of = queue + nn;
  const int32_t* order = comp_of + nn;
  const int32_t* comp_ptr = order + nn;
  const int32_t* local = comp_ptr + nn + 1;
  if (removed < 0 || removed > n || ncomp < 0 || ncomp > n)
    fail(MPLD_E_INTERNAL, "device split returned bad counts");
  s = Split();
  s.removal.assign(queue, queue + removed);
  s.comp_of.assign(comp_of, comp_of + nn);
  s.comp_ptr.assign(comp_ptr, comp_ptr + ncomp + 1);
  s.order.assign(order, order + s.comp_ptr.back());
  s.local.assign(local, local + nn);
}

void graph_builder_reserve(GraphBuilder& gb, int32_t nodes) {
  // sizes as a build and split of `nodes` nodes with up to 8 adjacency
  // entries and 4 grid cells per node would ask for
  std::lock_guard<std::mutex> lk(gb.mu);
  mpld_context* ctx = gb.ctx;
  const size_t n = (size_t)std::max(nodes, 1), cells = 4 * n, adj = 8 * n;
  for (DevBuf* b : {&gb.partner, &gb.cell_of, &gb.ids, &gb.smate}) grow(*b, ctx, 4 * n);
  for (DevBuf* b : {&gb.box, &gb.sbox}) grow(*b, ctx, 16 * n);
  for (DevBuf* b : {&gb.cnt, &gb.start, &gb.fill}) grow(*b, ctx, 4 * (cells + 1));
  for (DevBuf* b : {&gb.deg, &gb.ptr}) grow(*b, ctx, 4 * (n + 1));
  grow(gb.adj, ctx, 4 * adj);
  const size_t tiles = (cells + kScanTile - 1) / kScanTile + 1;
  grow(gb.sums, ctx, 4 * tiles);
  grow(gb.offs, ctx, 4 * tiles);
  grow(gb.split_ws, ctx, 4 * (split_out_words((int64_t)n) + kSplitScratch * std::max<size_t>(n + 1, 64)));
  if (!grow_pinned(gb.hin, 20 * n + 4 * (n + 1 + adj)) ||
      !grow_pinned(gb.hout, 4 * (n + 1 + adj + split_out_words((int64_t)n))))
    fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
}

void split_graph_device(GraphBuilder& gb, const Graph& g, int32_t k, bool simplify, Split& s) {
  const int32_t nn = g.n;
  if (nn == 0) {
    s = Split();
    s.comp_ptr.push_back(0);
    return;
  }
  const int64_t m2 = g.ptr[(size_t)nn];
  if (m2 >= INT32_MAX) fail(MPLD_E_INVALID, "graph too large for the device split");
  std::lock_guard<std::mutex> lk(gb.mu);
  mpld_context* ctx = gb.ctx;
  hipStream_t st = gb.stream;
  check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  const size_t nb = (size_t)nn;
  grow(gb.ptr, ctx, sizeof(int32_t) * (nb + 1));
  grow(gb.adj, ctx, sizeof(int32_t) * (size_t)std::max<int64_t>(m2, 1));
  const size_t in_bytes = sizeof(int32_t) * (nb + 1 + (size_t)m2);
  if (!grow_pinned(gb.hin, in_bytes)) fail(MPLD_E_NOMEM, "device split: pinned host memory");
  int32_t* hp = gb.hin.as<int32_t>();
  for (size_t i = 0; i <= nb; ++i) hp[i] = (int32_t)g.ptr[i];
  std::memcpy(hp + nb + 1, g.adj.data(), sizeof(int32_t) * (size_t)m2);
  check_hip(hipMemcpyAsync(gb.ptr.p, hp, sizeof(int32_t) * (nb + 1), hipMemcpyHostToDevice, st),
            "device split: upload offsets");
  if (m2)
    check_hip(hipMemcpyAsync(gb.adj.p, hp + nb + 1, sizeof(int32_t) * (size_t)m2,
                             hipMemcpyHostToDevice, st),
              "device split: upload lists");
  enqueue_split(gb, nn, gb.ptr.as<int32_t>(), gb.adj.as<int32_t>(), k, simplify);
  const size_t out_bytes = sizeof(int32_t) * split_out_words(nn);
  if (!grow_pinned(gb.hout, out_bytes)) fail(MPLD_E_NOMEM, "device split: pinned host memory");
  check_hip(hipMemcpyAsync(gb.hout.p, gb.split_ws.p, out_bytes, hipMemcpyDeviceToHost, st),
            "device split: download");
  check_hip(hipStreamSynchronize(st), "device split");
  collect_split(gb.hout.as<int32_t>(), nn, s);
}

bool build_layout_graph_device(GraphBuilder& gb, const mpld_rect* rects, int32_t n, int32_t dmin,
                               int32_t split_len, Graph& g, std::vector<int32_t>* se, Split* split,
                               int32_t k, bool simplify) {
  LayoutPrep lp;
  prepare_layout(rects, n, dmin, split_len, lp);
  const int32_t nn = (int32_t)lp.nd.size();
  g = Graph();
  g.n = nn;
  g.partner = lp.partner;
  g.ptr.assign((size_t)nn + 1, 0);
  if (se) *se = lp.se;
  if (nn == 0) {
    if (split) {
      *split = Split();
      split->comp_ptr.push_back(0);
    }
    return split != nullptr;
  }
  const int64_t ncell = lp.gx * lp.gy;
  if (ncell >= INT32_MAX || 2 * (int64_t)nn >= INT32_MAX)
    fail(MPLD_E_INVALID, "layout too large for the device graph builder");
  std::lock_guard<std::mutex> lk(gb.mu);
  mpld_context* ctx = gb.ctx;
  hipStream_t s = gb.stream;
  check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  GridParams gp{lp.minx, lp.miny, lp.cell, (int32_t)lp.gx, (int32_t)lp.gy};
  const size_t nb = (size_t)nn;
  grow(gb.box, ctx, sizeof(int4) * nb);
  grow(gb.partner, ctx, sizeof(int32_t) * nb);
  grow(gb.cell_of, ctx, sizeof(int32_t) * nb);
  grow(gb.cnt, ctx, sizeof(int32_t) * (size_t)(ncell + 1));
  grow(gb.start, ctx, sizeof(int32_t) * (size_t)(ncell + 1));
  grow(gb.fill, ctx, sizeof(int32_t) * (size_t)(ncell + 1));
  grow(gb.ids, ctx, sizeof(int32_t) * nb);
  grow(gb.sbox, ctx, sizeof(int4) * nb);
  grow(gb.smate, ctx, sizeof(int32_t) * nb);
  grow(gb.deg, ctx, sizeof(int32_t) * (nb + 1));
  grow(gb.ptr, ctx, sizeof(int32_t) * (nb + 1));
  // boxes and partners in one pinned staging copy
  const size_t in_bytes = sizeof(int4) * nb + sizeof(int32_t) * nb;
  if (!grow_pinned(gb.hin, in_bytes)) fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
  std::memcpy(gb.hin.p, lp.nd.data(), sizeof(int4) * nb);
  std::memcpy(static_cast<char*>(gb.hin.p) + sizeof(int4) * nb, lp.partner.data(),
              sizeof(int32_t) * nb);
  check_hip(hipMemcpyAsync(gb.box.p, gb.hin.p, sizeof(int4) * nb, hipMemcpyHostToDevice, s),
            "graph builder: upload boxes");
  check_hip(hipMemcpyAsync(gb.partner.p, static_cast<char*>(gb.hin.p) + sizeof(int4) * nb,
                           sizeof(int32_t) * nb, hipMemcpyHostToDevice, s),
            "graph builder: upload partners");
  const unsigned blocks = (unsigned)((nn + 255) / 256);
  const unsigned cblocks = (unsigned)std::min<int64_t>((ncell + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(cblocks), dim3(256), 0, s, gb.cnt.as<int32_t>(), ncell, 0);
  hipLaunchKernelGGL(cell_count_kernel, dim3(blocks), dim3(256), 0, s, gb.box.as<int4>(), nn, gp,
                     gb.cell_of.as<int32_t>(), gb.cnt.as<int32_t>());
  check_hip(hipGetLastError(), "graph builder: cell count");
  scan(gb, gb.cnt.as<int32_t>(), ncell, gb.start.as<int32_t>());
  check_hip(hipMemcpyAsync(gb.fill.p, gb.start.p, sizeof(int32_t) * (size_t)ncell,
                           hipMemcpyDeviceToDevice, s),
            "graph builder: cell fill positions");
  hipLaunchKernelGGL(cell_scatter_kernel, dim3(blocks), dim3(256), 0, s, gb.box.as<int4>(),
                     gb.partner.as<int32_t>(), nn, gb.cell_of.as<int32_t>(),
                     gb.fill.as<int32_t>(), gb.ids.as<int32_t>(), gb.sbox.as<int4>(),
                     gb.smate.as<int32_t>());
  const int64_t d2 = (int64_t)dmin * dmin;
  hipLaunchKernelGGL(neighbours_kernel<false>, dim3(blocks), dim3(256), 0, s, gb.sbox.as<int4>(),
                     gb.ids.as<int32_t>(), gb.smate.as<int32_t>(), gb.start.as<int32_t>(), nn, gp,
                     d2, gb.deg.as<int32_t>(), nullptr, nullptr);
  check_hip(hipGetLastError(), "graph builder: neighbour counts");
  scan(gb, gb.deg.as<int32_t>(), nn, gb.ptr.as<int32_t>());
  // the edge total decides the adjacency size
  int32_t total = 0;
  check_hip(hipMemcpyAsync(&total, gb.ptr.as<int32_t>() + nn, sizeof(int32_t),
                           hipMemcpyDeviceToHost, s),
            "graph builder: edge total");
  check_hip(hipStreamSynchronize(s), "graph builder: counts");
  grow(gb.adj, ctx, sizeof(int32_t) * (size_t)std::max(total, 1));
  hipLaunchKernelGGL(neighbours_kernel<true>, dim3(blocks), dim3(256), 0, s, gb.sbox.as<int4>(),
                     gb.ids.as<int32_t>(), gb.smate.as<int32_t>(), gb.start.as<int32_t>(), nn, gp,
                     d2, nullptr, gb.ptr.as<int32_t>(), gb.adj.as<int32_t>());
  check_hip(hipGetLastError(), "graph builder: neighbour lists");
  if (split && !device_split_pays(nn, total, k)) split = nullptr;   // the caller splits on the host
  if (split) enqueue_split(gb, nn, gb.ptr.as<int32_t>(), gb.adj.as<int32_t>(), k, simplify);
  const size_t split_words = split ? split_out_words(nn) : 0;
  const size_t out_bytes = sizeof(int32_t) * ((nb + 1) + (size_t)total + split_words);
  if (!grow_pinned(gb.hout, out_bytes)) fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
  int32_t* hptr = static_cast<int32_t*>(gb.hout.p);
  int32_t* hadj = hptr + nb + 1;
  int32_t* hsplit = hadj + total;
  if (split)
    check_hip(hipMemcpyAsync(hsplit, gb.split_ws.p, sizeof(int32_t) * split_words,
                             hipMemcpyDeviceToHost, s),
              "graph builder: download split");
  check_hip(hipMemcpyAsync(hptr, gb.ptr.p, sizeof(int32_t) * (nb + 1), hipMemcpyDeviceToHost, s),
            "graph builder: download offsets");
  if (total)
    check_hip(hipMemcpyAsync(hadj, gb.adj.p, sizeof(int32_t) * (size_t)total,
                             hipMemcpyDeviceToHost, s),
              "graph builder: download lists");
  check_hip(hipStreamSynchronize(s), "graph builder");
  for (size_t i = 0; i <= nb; ++i) g.ptr[i] = hptr[i];
  g.adj.assign(hadj, hadj + total);
  g.num_ce = total / 2;
  if (split) collect_split(hsplit, nn, *split);
  return split != nullptr;
}

}  // namespace mpld
