// wave_ops.h - 64-lane wavefront reductions shared by the search kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpld {

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

}  // namespace mpld
