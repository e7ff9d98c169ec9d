// wave_ops.h - 64-lane wavefront reductions shared by the search kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpld {

__device__ __forceinline__ uint32_t rdlane(uint32_t x, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)lane);
}
__device__ __forceinline__ uint64_t rdlane64(uint32_t lo, uint32_t hi, uint32_t lane) {
  return (uint64_t)rdlane(lo, lane) | ((uint64_t)rdlane(hi, lane) << 32);
}
// v_writelane: `old` with lane `lane` replaced by the uniform `val`.
__device__ int mpld_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t wrlane(uint32_t old, uint32_t lane, uint32_t val) {
  return (uint32_t)mpld_writelane((int)val, (int)lane, (int)old);
}
// Index of the lowest set bit of a nonzero 64-bit mask.
__device__ __forceinline__ uint32_t low_bit(uint64_t x) { return (uint32_t)__builtin_ctzll(x); }
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  return (uint64_t)uniform((uint32_t)x) | ((uint64_t)uniform((uint32_t)(x >> 32)) << 32);
}


// Minimum over the wave: row_shr 1, 2, 4, 8 leave each row's minimum in its
// lane 15; row_bcast 15 and 31 fold the four rows into lane 63.  A lane
// with no source in a step reads all-ones, the identity of min, so the
// compiler fuses each step into one v_min_u32_dpp.  Every lane must be
// active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t m) {
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x111, 0xf, 0xf, false));
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x112, 0xf, 0xf, false));
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x114, 0xf, 0xf, false));
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x118, 0xf, 0xf, false));
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x142, 0xa, 0xf, false));
  m = min(m, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)m, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
}

// Sum over the wave, by the same steps as wave_min_u32 (a lane with no
// source reads 0, the identity of the sum); every lane must be active.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t m) {
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x111, 0xf, 0xf, false);
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x112, 0xf, 0xf, false);
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x114, 0xf, 0xf, false);
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x118, 0xf, 0xf, false);
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x142, 0xa, 0xf, false);
  m += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)m, 0x143, 0xc, 0xf, false);
  return (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
}

}  // namespace mpld
