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

// ---- host side --------------------------------------------------------------

struct GraphBuilder {
  mpld_context* ctx = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  DevBuf box, partner, cell_of, cnt, start, fill, ids, sbox, smate, deg, ptr, adj, sums, offs;
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

void build_layout_graph_device(GraphBuilder& gb, const mpld_rect* rects, int32_t n, int32_t dmin,
                               int32_t split_len, Graph& g, std::vector<int32_t>* se) {
  LayoutPrep lp;
  prepare_layout(rects, n, dmin, split_len, lp);
  const int32_t nn = (int32_t)lp.nd.size();
  g = Graph();
  g.n = nn;
  g.partner = lp.partner;
  g.ptr.assign((size_t)nn + 1, 0);
  if (se) *se = lp.se;
  if (nn == 0) return;
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
  const size_t out_bytes = sizeof(int32_t) * (nb + 1) + sizeof(int32_t) * (size_t)total;
  if (!gb.hout.reserve(out_bytes)) fail(MPLD_E_NOMEM, "graph builder: pinned host memory");
  int32_t* hptr = static_cast<int32_t*>(gb.hout.p);
  int32_t* hadj = hptr + nb + 1;
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
}

}  // namespace mpld
