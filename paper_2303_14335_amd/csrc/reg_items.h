// reg_items.h - device-side access to the register-tier work items (the
// RegItems layout of device_types.h), shared by the register-tier kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_types.h"

namespace mpld {

__device__ __forceinline__ const DevDesc& item_desc(const RegItems& R, int32_t i) {
  return *reinterpret_cast<const DevDesc*>(R.base + (uint64_t)i * R.stride);
}
__device__ __forceinline__ uint64_t item_mask(const RegItems& R, int32_t i, uint32_t lane) {
  const uint64_t* m = reinterpret_cast<const uint64_t*>(R.base + (uint64_t)i * R.stride + kRegItemHead);
  return lane < R.width ? m[lane] : 0ull;   // zero past n
}
// Stitch partner (local id) of node `lane`, 0xff for none: byte `lane` of
// the item's partner block, which is 8-byte aligned and padded, so it is
// read as a 32-bit word.
__device__ __forceinline__ uint32_t item_partner(const RegItems& R, int32_t i, uint32_t lane) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(R.base + (uint64_t)i * R.stride + R.part_off);
  const bool in = lane < R.width;
  const uint32_t w = p[in ? lane >> 2 : 0u];   // word 0 always exists
  return in ? (w >> ((lane & 3u) * 8u)) & 0xffu : 0xffu;
}

}  // namespace mpld
