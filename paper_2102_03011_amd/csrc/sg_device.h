// Device helpers shared by the gather/filter kernels and the learned-filter kernels.
#ifndef SG_DEVICE_H
#define SG_DEVICE_H

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scene_gather.h"

namespace sg {

__device__ __forceinline__ float h2f(uint32_t bits16) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16 & 0xFFFFu)));
}

__device__ __forceinline__ uint32_t f2h(float v) {
  return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(v)));
}

constexpr uint32_t kInvalidDepth16 = 0x7E00u;  // binary16 quiet NaN

// Stored planes: SG_APRON rows above and below, SG_APRON columns left and
// SG_APRON_RIGHT columns right of the image.
__host__ __device__ __forceinline__ int stored_pitch(int width) {
  return width + SG_APRON + SG_APRON_RIGHT;
}
__host__ __device__ __forceinline__ int stored_rows(int height) { return height + 2 * SG_APRON; }

// Stored-plane index of image pixel (x, y).
__device__ __forceinline__ size_t padded_index(int x, int y, int pw) {
  return static_cast<size_t>(y + SG_APRON) * pw + (x + SG_APRON);
}

}  // namespace sg

#endif
