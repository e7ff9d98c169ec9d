// noalloc.hip - mpld_solve_components_noalloc: mpld_solve_components for
// register-tier components (at most 64 nodes each) with every device buffer
// it needs - queue counter, per-component records, local colors, packed
// work items - in one fixed file-scope device array, and its host staging
// in static host memory, so that a call allocates nothing.
//
// The device array `scratch` exists once per GPU the library runs on.  In
// host code its name is only a host-side stand-in: its device address is
// looked up once per device with hipGetSymbolAddress (with that device
// current) and kept; only that address is handed to kernels and copies.
// Every call on a GPU shares that GPU's array and leaves its contents
// behind; calls that overlap on one GPU race (a process-wide mutex
// serialises the calls of one process).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "device_types.h"
#include "internal.h"
#include "mpld.h"
#include "runtime.h"

namespace mpld {

constexpr size_t kScratchBytes = MPLD_NOALLOC_SCRATCH_BYTES;
constexpr int32_t kNoallocMaxComps = MPLD_NOALLOC_MAX_COMPONENTS;
constexpr int kNoallocMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Clears `n` 32-bit words (a kernel, not a memset, so that a caller may
// capture the call in a HIP graph).
__global__ void noalloc_clear_kernel(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

namespace {

// Host staging, static: packed items, launch order, component offsets and
// the records read back.
struct NoallocStage {
  std::mutex mu;
  uint8_t items[kScratchBytes];
  int32_t order[kNoallocMaxComps];
  int32_t offs[kNoallocMaxComps];
  DevRecord recs[kNoallocMaxComps];
};
NoallocStage g_stage;

std::mutex g_addr_mu;
void* g_addr[kNoallocMaxDevices];

// Device address of `scratch` on the current device `dev`, looked up once.
uint8_t* scratch_on(int dev) {
  if (dev < 0 || dev >= kNoallocMaxDevices) fail(MPLD_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_addr_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(MPLD_E_DEVICE, "hipGetSymbolAddress gave a null scratch address");
    g_addr[dev] = p;
  }
  return static_cast<uint8_t*>(g_addr[dev]);
}

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

void solve_noalloc(mpld_context* ctx, const mpld_component* comps, int32_t count,
                   const mpld_options* opt, mpld_comp_record* out, int8_t* colors_out) {
  if (!ctx) fail(MPLD_E_INVALID, "context is NULL");
  check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (!opt || opt->struct_size != sizeof(mpld_options)) fail(MPLD_E_INVALID, "bad options");
  if (opt->k < 2 || opt->k > MPLD_MAX_K) fail(MPLD_E_INVALID, "k must be in [2, 8]");
  if (opt->node_budget < 1) fail(MPLD_E_INVALID, "node_budget must be >= 1");
  const uint32_t unsupported = MPLD_PLAIN | MPLD_FORCE_LDS | MPLD_FORCE_GLOBAL | MPLD_FORCE_DEVICE |
                               MPLD_SPLIT_HEAVY | MPLD_STITCH_ORDER | MPLD_MINIMIZE | MPLD_ROUNDTRIP;
  if (opt->flags & unsupported)
    fail(MPLD_E_UNSUPPORTED, "the allocation-free solve takes MPLD_TRACE_HASH and "
                             "MPLD_MARK_CONFLICTS only (register tier, direct launches)");
  if (count < 0 || (count > 0 && (!comps || !out || !colors_out)))
    fail(MPLD_E_INVALID, "bad component array");
  if (count > kNoallocMaxComps)
    fail(MPLD_E_INVALID, "more components than the allocation-free solve takes (" +
                             std::to_string(kNoallocMaxComps) + ")");
  // sizes: every component on the register tier
  int64_t total_nodes = 0;
  int32_t max_n = 1;
  for (int32_t c = 0; c < count; ++c) {
    const mpld_component& cp = comps[c];
    if (cp.n < 0 || cp.m < 0 || (cp.m > 0 && !cp.edges))
      fail(MPLD_E_INVALID, "component " + std::to_string(c) + " has a bad size or edge array");
    if (cp.n > 64)
      fail(MPLD_E_UNSUPPORTED, "the allocation-free solve takes components of at most 64 nodes; "
                               "component " + std::to_string(c) + " has " + std::to_string(cp.n));
    total_nodes += cp.n;
    max_n = std::max(max_n, cp.n);
  }
  const uint32_t width = reg_item_width(max_n);
  const size_t stride = kRegItemHead + 8u * (size_t)width;
  const size_t off_recs = 256, off_colors = off_recs + up256(sizeof(DevRecord) * (size_t)count),
               off_items = off_colors + up256((size_t)total_nodes),
               need = off_items + stride * (size_t)count;
  if (need > kScratchBytes)
    fail(MPLD_E_INVALID, "the components need " + std::to_string(need) +
                             " bytes of device scratch; the allocation-free solve has " +
                             std::to_string(kScratchBytes));
  if (count == 0) return;
  uint8_t* dev = scratch_on(ctx->device);

  std::lock_guard<std::mutex> lk(g_stage.mu);
  // offsets in input order; launch order = largest component first, ties by index
  int32_t off = 0;
  for (int32_t c = 0; c < count; ++c) {
    g_stage.offs[c] = off;
    off += comps[c].n;
    g_stage.order[c] = c;
  }
  std::sort(g_stage.order, g_stage.order + count, [&](int32_t a, int32_t b) {
    return comps[a].n != comps[b].n ? comps[a].n > comps[b].n : a < b;
  });
  for (int32_t i = 0; i < count; ++i) {
    const int32_t c = g_stage.order[i];
    const mpld_component& cp = comps[c];
    uint8_t* it = g_stage.items + stride * (size_t)i;
    DevDesc d{};
    d.n = cp.n;
    d.k = opt->k;
    d.budget = opt->node_budget;
    d.nbr_off = 0;
    d.out_off = g_stage.offs[c];
    d.comp = c;
    std::memcpy(it, &d, sizeof(DevDesc));
    uint64_t* mk = reinterpret_cast<uint64_t*>(it + kRegItemHead);
    std::memset(mk, 0, 8u * (size_t)width);
    for (int64_t e = 0; e < cp.m; ++e) {
      const int32_t a = cp.edges[2 * e], b = cp.edges[2 * e + 1];
      if (a < 0 || b < 0 || a >= cp.n || b >= cp.n || a == b)
        fail(MPLD_E_INVALID, "component " + std::to_string(c) + " edge " + std::to_string(e) +
                                 " is out of range or a self loop");
      if ((mk[a] >> b) & 1ull)
        fail(MPLD_E_INVALID, "component " + std::to_string(c) + " has a duplicate edge");
      mk[a] |= 1ull << b;
      mk[b] |= 1ull << a;
    }
  }

  hipStream_t s = ctx->stream;
  int32_t* counter = reinterpret_cast<int32_t*>(dev);
  DevRecord* recs = reinterpret_cast<DevRecord*>(dev + off_recs);
  int8_t* colors = reinterpret_cast<int8_t*>(dev + off_colors);
  uint8_t* items = dev + off_items;
  hipLaunchKernelGGL(noalloc_clear_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(dev),
                     64u);
  check_hip(hipGetLastError(), "clear the queue counter");
  check_hip(hipMemcpyAsync(items, g_stage.items, stride * (size_t)count, hipMemcpyHostToDevice, s),
            "upload items");
  const RegItems ri{items, width, (uint32_t)stride, 0u};
  const bool trace = opt->flags & MPLD_TRACE_HASH;
  const int cap = ctx->num_cus * ctx->reg_blocks_per_cu;
  const int grid = std::max(1, std::min((count + 3) / 4, cap));
  check_hip(launch_reg_batched(trace, opt->k, grid, 4, ri, count, counter, recs, colors, ~0ull, 0, 16u,
                               (opt->flags & MPLD_MARK_CONFLICTS) != 0, s),
            "register-tier launch");
  check_hip(hipMemcpyAsync(g_stage.recs, recs, sizeof(DevRecord) * (size_t)count,
                           hipMemcpyDeviceToHost, s), "download records");
  if (total_nodes)
    check_hip(hipMemcpyAsync(colors_out, colors, (size_t)total_nodes, hipMemcpyDeviceToHost, s),
              "download colors");
  check_hip(hipStreamSynchronize(s), "allocation-free solve");
  const bool colored_marked = opt->flags & MPLD_MARK_CONFLICTS;
  for (int32_t c = 0; c < count; ++c) {
    const DevRecord& dr = g_stage.recs[c];
    if (dr.status < 0 || dr.status > MPLD_BUDGET_EXHAUSTED)
      fail(MPLD_E_INTERNAL, "search reported a broken state");
    mpld_comp_record& r = out[c];
    r.size = comps[c].n;
    r.status = dr.status;
    r.nodes = (int64_t)dr.nodes;
    r.trace_hash = trace ? dr.hash : 0;
    r.depth_at_stop = dr.depth;
    r.stitches = r.status == MPLD_FEASIBLE || colored_marked ? 0 : -1;
    r.first_node = -1;
    r.num_edges = (int32_t)comps[c].m;
    r.conflicts = 0;
    r.min_nodes = 0;
    const int8_t* cc = colors_out + g_stage.offs[c];
    for (int64_t e = 0; e < comps[c].m; ++e) {
      const int8_t a = cc[comps[c].edges[2 * e]];
      r.conflicts += a >= 0 && a == cc[comps[c].edges[2 * e + 1]];
    }
  }
}

}  // namespace
}  // namespace mpld

extern "C" int32_t mpld_solve_components_noalloc(mpld_context* ctx, const mpld_component* comps,
                                                 int32_t count, const mpld_options* opt,
                                                 mpld_comp_record* out, int8_t* colors_out) {
  try {
    mpld::solve_noalloc(ctx, comps, count, opt, out, colors_out);
    mpld::set_last_error("");
    return MPLD_OK;
  } catch (const mpld::Error& e) {
    mpld::set_last_error(e.what);
    return e.code;
  } catch (...) {
    mpld::set_last_error("unexpected exception in the allocation-free solve");
    return MPLD_E_INTERNAL;
  }
}
