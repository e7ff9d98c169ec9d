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
// still on the device: split_kernel reproduces the host's FIFO peeling order,
// components ordered by smallest id and BFS local numbering exactly, level by
// level (see the comment above it).
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
// One workgroup of 1024 threads does the whole split, so that its many short
// rounds are separated by barriers instead of launches.  It reproduces the
// sequential definitions exactly:
//
// FIFO peeling (nodes of conflict degree < k, queue seeded in ascending id;
// a popped node lowers its neighbours' degrees in ascending id and queues
// those that drop below k).  The queue falls into levels: level 0 is the
// seed; level L+1 holds the nodes queued while level L is popped.  A node w
// outside levels 0..L with deg0(w) = d is queued when its (d - k + 1)-th
// neighbour is popped; if that neighbour (its trigger) is in level L, it is
// the one of rank (d - k + 1 - before) among w's level-L neighbours by queue
// position, `before` counting w's neighbours in earlier levels.  Level L+1 is
// then ordered by (trigger's queue position, w's position in the trigger's
// ascending list), i.e. one exclusive scan of per-trigger counts.
//
// Components: union-find with hooking of the larger root under the smaller
// (so each root is its component's smallest id), numbered by root id.  BFS
// local numbering from each root, neighbours in ascending id: a node of BFS
// level d+1 is reached from its level-d neighbour of smallest local position,
// and level d+1 is ordered per component by (parent's position, id) -- again
// one scan of per-parent counts, with per-component bases.
constexpr int kSplitThreads = 1024;

struct SplitArgs {
  int32_t n, k, simplify;
  const int32_t* ptr;   // n + 1 CSR offsets
  const int32_t* adj;   // ascending neighbour lists
  // outputs
  int32_t* counts;      // [0] removed, [1] components
  int32_t* queue;       // n: removal order
  int32_t* comp_of;     // n: component, -1 if removed
  int32_t* order;       // n: core nodes by component, local order
  int32_t* comp_ptr;    // n + 1
  int32_t* local;       // n: local index, -1 if removed
  // scratch, n each
  int32_t *qpos, *lvl, *stamp, *trig, *cand, *parent, *fa, *fb, *gex, *cnt, *cbase, *tail, *rootof;
};

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

__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving (parent[x] < x for every non-root, so every
// rewrite points x at one of its ancestors and the loop ends).
__device__ int32_t uf_find(int32_t* parent, int32_t x) {
  for (;;) {
    const int32_t p = ld_relaxed(parent + x);
    if (p == x) return x;
    const int32_t g = ld_relaxed(parent + p);
    if (g == p) return p;
    __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = g;
  }
}

// Hooks the larger of the two roots under the smaller; a failed CAS means
// that root was just hooked elsewhere: find again.
__device__ void uf_unite(int32_t* parent, int32_t a, int32_t b) {
  for (;;) {
    const int32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    const int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
    if (atomicCAS(parent + hi, hi, lo) == hi) return;
  }
}

__global__ __launch_bounds__(kSplitThreads) void split_kernel(SplitArgs a) {
  __shared__ int32_t wsum[kSplitThreads / 64];
  __shared__ int32_t ncand;
  const int32_t tid = (int32_t)threadIdx.x, T = kSplitThreads, n = a.n;
  const int32_t* __restrict__ ptr = a.ptr;
  const int32_t* __restrict__ adj = a.adj;
  for (int32_t v = tid; v < n; v += T) {
    a.qpos[v] = -1;
    a.lvl[v] = -1;
    a.stamp[v] = -1;
    a.trig[v] = -1;
    a.local[v] = -1;
    a.comp_of[v] = -1;
  }
  __syncthreads();

  // ---- FIFO peeling, level by level
  int32_t qn = 0;
  if (a.simplify) {
    for (int32_t base = 0; base < n; base += T) {   // level 0: degree < k, ascending
      const int32_t v = base + tid;
      const int32_t f = v < n && ptr[v + 1] - ptr[v] < a.k ? 1 : 0;
      int32_t total;
      const int32_t ex = wg_excl_scan(f, wsum, total);
      if (f) {
        a.queue[qn + ex] = v;
        a.qpos[v] = qn + ex;
        a.lvl[v] = 0;
      }
      qn += total;
    }
  }
  for (int32_t lo = 0, hi = qn, L = 0; lo < hi; ++L) {
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
          if (a.qpos[w] < 0 && a.trig[w] == u) {
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
    qn = next;
  }

  // ---- components over the core (never queued): union-find
  for (int32_t v = tid; v < n; v += T) a.parent[v] = a.lvl[v] < 0 ? v : -1;
  __syncthreads();
  for (int32_t v = tid; v < n; v += T) {
    if (a.lvl[v] >= 0) continue;
    for (int32_t t = ptr[v]; t < ptr[v + 1]; ++t) {
      const int32_t w = adj[t];
      if (w > v && a.lvl[w] < 0) uf_unite(a.parent, v, w);
    }
  }
  __syncthreads();
  // every core node's root, by read-only walks (a halving store here could
  // overwrite a root just written with an older ancestor), then stored
  for (int32_t v = tid; v < n; v += T)
    if (a.lvl[v] < 0) {
      int32_t r = v;
      for (int32_t p = a.parent[r]; p != r; p = a.parent[r]) r = p;
      a.fa[v] = r;
    }
  __syncthreads();
  for (int32_t v = tid; v < n; v += T)
    if (a.lvl[v] < 0) a.parent[v] = a.fa[v];
  __syncthreads();
  // numbered by root (= smallest id) ascending
  int32_t ncomp = 0;
  for (int32_t base = 0; base < n; base += T) {
    const int32_t v = base + tid;
    const int32_t f = v < n && a.lvl[v] < 0 && a.parent[v] == v ? 1 : 0;
    int32_t total;
    const int32_t ex = wg_excl_scan(f, wsum, total);
    if (f) {
      a.comp_of[v] = ncomp + ex;
      a.rootof[ncomp + ex] = v;
    }
    ncomp += total;
  }
  for (int32_t c = tid; c < ncomp; c += T) a.tail[c] = 0;
  __syncthreads();
  for (int32_t v = tid; v < n; v += T) {
    if (a.lvl[v] >= 0) continue;
    const int32_t c = a.comp_of[a.parent[v]];
    if (a.parent[v] != v) a.comp_of[v] = c;
    atomicAdd(a.tail + c, 1);
  }
  __syncthreads();
  int32_t core = 0;
  for (int32_t base = 0; base < ncomp; base += T) {
    const int32_t c = base + tid;
    const int32_t sz = c < ncomp ? a.tail[c] : 0;
    int32_t total;
    const int32_t ex = wg_excl_scan(sz, wsum, total);
    if (c < ncomp) a.comp_ptr[c] = core + ex;
    core += total;
  }
  if (tid == 0) a.comp_ptr[ncomp] = core;
  __syncthreads();

  // ---- BFS local numbering, all components at once
  for (int32_t v = tid; v < n; v += T) {
    a.stamp[v] = -1;
    a.trig[v] = -1;
  }
  for (int32_t c = tid; c < ncomp; c += T) {
    const int32_t r = a.rootof[c];
    a.fa[c] = r;
    a.local[r] = 0;
    a.order[a.comp_ptr[c]] = r;
    a.tail[c] = 1;
  }
  __syncthreads();
  int32_t* F = a.fa;
  int32_t* NF = a.fb;
  for (int32_t fn = ncomp, d = 0; fn > 0; ++d) {
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
    // children per frontier node; frontier is ordered by (component, position)
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
      const int32_t u = F[i], cu = a.comp_of[u];
      int32_t p = a.tail[cu] + a.gex[i] - a.cbase[cu], g = a.gex[i];
      if (a.cnt[i] == 0) continue;
      for (int32_t t = ptr[u]; t < ptr[u + 1]; ++t) {
        const int32_t w = adj[t];
        if (a.lvl[w] < 0 && a.local[w] < 0 && a.trig[w] == u) {
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
  if (tid == 0) {
    a.counts[0] = qn;
    a.counts[1] = ncomp;
  }
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

static void grow(DevBuf& b, mpld_context* ctx, size_t bytes) {
  if (b.bytes < bytes) b.alloc(ctx, bytes + bytes / 4);
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
// comp_ptr (n + 1), local (n) -- the part copied back, kSplitOut(n) words --
// then 13 scratch arrays of n.
static size_t split_out_words(int64_t n) { return 2 + 5 * (size_t)n + 1; }

// Enqueues split_kernel on the CSR at dptr / dadj (device, int32).
static void enqueue_split(GraphBuilder& gb, int32_t n, const int32_t* dptr, const int32_t* dadj,
                          int32_t k, bool simplify) {
  const size_t nn = (size_t)n;
  grow(gb.split_ws, gb.ctx, sizeof(int32_t) * (split_out_words(n) + 13 * nn));
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
  int32_t** scratch[] = {&a.qpos, &a.lvl, &a.stamp, &a.trig, &a.cand, &a.parent, &a.fa,
                         &a.fb, &a.gex, &a.cnt, &a.cbase, &a.tail, &a.rootof};
  for (int32_t** d : scratch) {
    *d = q;
    q += nn;
  }
  hipLaunchKernelGGL(split_kernel, dim3(1), dim3(kSplitThreads), 0, gb.stream, a);
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
  if (!gb.hin.reserve(in_bytes)) fail(MPLD_E_NOMEM, "device split: pinned host memory");
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
  if (!gb.hout.reserve(out_bytes)) fail(MPLD_E_NOMEM, "device split: pinned host memory");
  check_hip(hipMemcpyAsync(gb.hout.p, gb.split_ws.p, out_bytes, hipMemcpyDeviceToHost, st),
            "device split: download");
  check_hip(hipStreamSynchronize(st), "device split");
  collect_split(gb.hout.as<int32_t>(), nn, s);
}

void build_layout_graph_device(GraphBuilder& gb, const mpld_rect* rects, int32_t n, int32_t dmin,
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
    return;
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
  if (!gb.hin.reserve(in_bytes)) fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
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
  if (split) enqueue_split(gb, nn, gb.ptr.as<int32_t>(), gb.adj.as<int32_t>(), k, simplify);
  const size_t split_words = split ? split_out_words(nn) : 0;
  const size_t out_bytes = sizeof(int32_t) * ((nb + 1) + (size_t)total + split_words);
  if (!gb.hout.reserve(out_bytes)) fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
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
}

}  // namespace mpld
