// measure.hip - measurements that put the search kernels' times in
// context: the LDS read rate used for the roofline of the LDS-tier kernels
// (every CU runs workgroups that read their LDS with ds_read_b64 or
// ds_read_b128; each wave reads contiguous bytes, so no bank conflicts; the
// bytes read over the kernel's time give the chip's achievable LDS read
// rate), and the time per launch of an empty kernel launched back to back
// (the fixed cost inside a step of one search launch).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "mpld.h"
#include "runtime.h"

namespace mpld {

constexpr int kLdsProbeThreads = 256;
constexpr int kLdsProbeUnroll = 16;

// 32 KB of LDS per workgroup (five workgroups, twenty waves, per CU).  Per
// iteration a lane reads kLdsProbeUnroll vectors at immediate offsets from
// a base that alternates between two halves; an empty asm statement with a
// memory clobber ends every iteration, so the compiler must read LDS again
// (it may not hoist the loads or fold the XORs across iterations), and the
// XOR of everything read is kept so that the loads are not removed.
template <typename V>
__global__ __launch_bounds__(kLdsProbeThreads) void lds_read_kernel(uint32_t iters,
                                                                    uint32_t* __restrict__ sink) {
  constexpr int kElems = 32768 / (int)sizeof(V);
  constexpr int kStride = (kElems - 2 * kLdsProbeThreads) / kLdsProbeUnroll;
  __shared__ V buf[kElems];
  for (int i = threadIdx.x; i < kElems; i += kLdsProbeThreads) {
    V v;
    uint32_t* w = reinterpret_cast<uint32_t*>(&v);
    for (int j = 0; j < (int)(sizeof(V) / 4); ++j) w[j] = (uint32_t)(i * 4 + j);
    buf[i] = v;
  }
  __syncthreads();
  uint32_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
    const V* p = buf + threadIdx.x + ((it & 1u) ? kLdsProbeThreads : 0);
#pragma unroll
    for (int j = 0; j < kLdsProbeUnroll; ++j) {
      const V v = p[j * kStride];
      const uint32_t* w = reinterpret_cast<const uint32_t*>(&v);
#pragma unroll
      for (int q = 0; q < (int)(sizeof(V) / 4); ++q) acc ^= w[q];
    }
    __asm__ volatile("" ::: "memory");
  }
  if (acc == 0x9e3779b9u) sink[blockIdx.x] = acc;   // never true for these contents in practice
}

// Does nothing: its back-to-back launches time dispatch and completion.
__global__ void empty_kernel() {}

// Each wave w reads the 64 bytes at in + 64 w (lanes 0..7) and lane 0
// writes 8 bytes to out[w]: the fixed cost of a launch whose waves touch
// device memory once each way, as every search wave loads its item and
// stores its record.
__global__ void touch_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), l = threadIdx.x & 63u;
  uint64_t v = l < 8u ? in[(uint64_t)w * 8u + l] : 0ull;
  v ^= __shfl_xor(v, 1);
  v ^= __shfl_xor(v, 2);
  v ^= __shfl_xor(v, 4);
  if (l == 0u) out[w] = v;
}

}  // namespace mpld

using namespace mpld;

extern "C" int32_t mpld_measure_lds_read_rate(mpld_context* ctx, int32_t bytes_per_lane,
                                              int32_t iters, double* gbytes_per_s,
                                              double* bytes_per_clock_per_cu) {
  try {
    if (!ctx || !gbytes_per_s) fail(MPLD_E_INVALID, "NULL argument");
    if (bytes_per_lane != 8 && bytes_per_lane != 16)
      fail(MPLD_E_INVALID, "bytes_per_lane must be 8 (ds_read_b64) or 16 (ds_read_b128)");
    if (iters < 1 || iters > (1 << 24)) fail(MPLD_E_INVALID, "iters must be in [1, 2^24]");
    check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    const int grid = ctx->num_cus * 5 * 8;   // five resident workgroups per CU, eight rounds
    DevBuf sink;
    sink.alloc(ctx, sizeof(uint32_t) * (size_t)grid);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {   // the first run warms up
      err = hipEventRecord(e0, s);
      if (bytes_per_lane == 8)
        hipLaunchKernelGGL((lds_read_kernel<uint2>), dim3(grid), dim3(kLdsProbeThreads), 0, s,
                           (uint32_t)iters, sink.as<uint32_t>());
      else
        hipLaunchKernelGGL((lds_read_kernel<uint4>), dim3(grid), dim3(kLdsProbeThreads), 0, s,
                           (uint32_t)iters, sink.as<uint32_t>());
      if (err == hipSuccess) err = hipGetLastError();
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    }
    // whatever failed, the sink is released only once the stream has
    // drained what was enqueued on it
    const hipError_t drained = hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    check_hip(err, "LDS read-rate kernel");
    check_hip(drained, "LDS read-rate drain");
    const double bytes = (double)grid * kLdsProbeThreads * (double)iters * kLdsProbeUnroll *
                         (double)bytes_per_lane;
    *gbytes_per_s = bytes / ((double)ms * 1e-3) / 1e9;
    if (bytes_per_clock_per_cu) {
      int khz = 0;
      check_hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, ctx->device), "clock rate");
      *bytes_per_clock_per_cu = khz > 0 ? *gbytes_per_s * 1e9 / ((double)khz * 1e3) / ctx->num_cus : 0.0;
    }
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (...) {
    set_last_error("unexpected exception in the LDS read-rate measurement");
    return MPLD_E_INTERNAL;
  }
}

extern "C" int32_t mpld_measure_launch_floor(mpld_context* ctx, int32_t grid, int32_t block,
                                             int32_t reps, double* us_per_launch) {
  try {
    if (!ctx || !us_per_launch) fail(MPLD_E_INVALID, "NULL argument");
    if (grid < 1 || grid > (1 << 20)) fail(MPLD_E_INVALID, "grid must be in [1, 2^20]");
    if (block < 64 || block > 1024 || block % 64 != 0)
      fail(MPLD_E_INVALID, "block must be a multiple of 64 in [64, 1024]");
    if (reps < 1 || reps > 100000) fail(MPLD_E_INVALID, "reps must be in [1, 100000]");
    check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(empty_kernel, dim3(grid), dim3(block), 0, s);   // warm-up
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int32_t r = 0; r < reps && err == hipSuccess; ++r) {
      hipLaunchKernelGGL(empty_kernel, dim3(grid), dim3(block), 0, s);
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    check_hip(err, "empty-kernel launches");
    *us_per_launch = (double)ms * 1e3 / reps;
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (...) {
    set_last_error("unexpected exception in the launch-floor measurement");
    return MPLD_E_INTERNAL;
  }
}

extern "C" int32_t mpld_measure_touch_floor(mpld_context* ctx, int32_t grid, int32_t block,
                                            int32_t reps, double* us_per_launch) {
  try {
    if (!ctx || !us_per_launch) fail(MPLD_E_INVALID, "NULL argument");
    if (grid < 1 || grid > (1 << 20)) fail(MPLD_E_INVALID, "grid must be in [1, 2^20]");
    if (block < 64 || block > 1024 || block % 64 != 0)
      fail(MPLD_E_INVALID, "block must be a multiple of 64 in [64, 1024]");
    if (reps < 1 || reps > 100000) fail(MPLD_E_INVALID, "reps must be in [1, 100000]");
    check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    const size_t waves = (size_t)grid * (size_t)(block / 64);
    DevBuf in, out;
    in.alloc(ctx, 64 * waves);
    out.alloc(ctx, 8 * waves);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    hipError_t err = hipMemsetAsync(in.p, 0, 64 * waves, s);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) {
      hipLaunchKernelGGL(touch_kernel, dim3(grid), dim3(block), 0, s, in.as<const uint64_t>(),
                         out.as<uint64_t>());   // warm-up
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int32_t r = 0; r < reps && err == hipSuccess; ++r) {
      hipLaunchKernelGGL(touch_kernel, dim3(grid), dim3(block), 0, s, in.as<const uint64_t>(),
                         out.as<uint64_t>());
      err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    // whatever failed, the buffers are released only once the stream has
    // drained what was enqueued on them
    const hipError_t drained = hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    check_hip(err, "touch-kernel launches");
    check_hip(drained, "touch-kernel drain");
    *us_per_launch = (double)ms * 1e3 / reps;
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (...) {
    set_last_error("unexpected exception in the touch-floor measurement");
    return MPLD_E_INTERNAL;
  }
}
