// sort_util.h -- 64-bit TopK keys and the LDS bitonic network shared by the
// TopK and rescoring kernels.
//
// key = ord(score) << 32 | (0xFFFFFFFF - id): unsigned order = score
// descending, then id ascending; ord() maps IEEE floats monotonically onto
// unsigned integers.  Key 0 never arises from a real entry (it would need a NaN
// score), so it pads.
#pragma once

#include "farm_internal.h"

namespace farm {

constexpr int kSortMax = 4096;

__device__ inline uint32_t ord_float(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ inline float unord_float(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(b);
}

__device__ inline uint64_t make_key(float score, uint32_t id) {
  return ((uint64_t)ord_float(score) << 32) | (uint64_t)(0xFFFFFFFFu - id);
}

// Descending bitonic sort of keys[0..P) (P a power of two) with a payload.
__device__ inline void bitonic_desc(uint64_t* keys, int32_t* idx, int P) {
  for (int k2 = 2; k2 <= P; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        int i = 2 * t - (t & (j - 1));
        int l = i + j;
        bool desc = (i & k2) == 0;
        uint64_t a = keys[i], b = keys[l];
        bool sw = desc ? (a < b) : (a > b);
        if (sw) {
          keys[i] = b;
          keys[l] = a;
          int32_t x = idx[i];
          idx[i] = idx[l];
          idx[l] = x;
        }
      }
      __syncthreads();
    }
  }
}

__device__ inline int pow2_at_least(int v) {
  int p = 2;
  while (p < v) p <<= 1;
  return p;
}


__device__ inline float key_score(uint64_t k) { return unord_float((uint32_t)(k >> 32)); }
__device__ inline uint32_t key_id(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFu); }

}  // namespace farm
