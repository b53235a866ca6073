// Device helpers shared by the gather/filter kernels and the learned-filter kernels.
#ifndef SG_DEVICE_H
#define SG_DEVICE_H

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scene_gather.h"

namespace sg {

// Global-memory pointers. A pointer read from a descriptor in memory (not a kernel
// argument) is generic to the compiler and its accesses become flat instructions;
// the device functions take pointers of the global address space, and every
// device buffer of this library is global memory.
template <typename T>
using gp = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gp<T> to_global(T* p) {
  return (gp<T>)p;
}

// 8-byte records through global pointers (the vector type's members take generic
// references only)
__device__ __forceinline__ uint2 ld2(gp<const uint2> p) {
  const uint64_t v = *reinterpret_cast<gp<const uint64_t>>(p);
  return make_uint2(static_cast<uint32_t>(v), static_cast<uint32_t>(v >> 32));
}
__device__ __forceinline__ void st2(gp<uint2> p, uint2 v) {
  *reinterpret_cast<gp<uint64_t>>(p) = static_cast<uint64_t>(v.x) | (static_cast<uint64_t>(v.y) << 32);
}
__device__ __forceinline__ void flag_or(gp<uint32_t> status, uint32_t bits) {
  __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float h2f(uint32_t bits16) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16 & 0xFFFFu)));
}

__device__ __forceinline__ uint32_t f2h(float v) {
  return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(v)));
}

constexpr uint32_t kInvalidDepth16 = 0x7E00u;  // binary16 quiet NaN

// Stored planes: SG_APRON rows above and below, SG_APRON columns left and
// SG_APRON_RIGHT columns right of the image. Every block read of the gather stays
// inside the plane: centres at most r outside the image, blocks 2r + 1 wide, block
// rows of depths read as whole 8-byte words (4 values) from their first column.
constexpr int right_apron_needed(int r) { return 4 * ((2 * r + 1 + 3) / 4) - 1; }
static_assert(SG_APRON >= 2 * SG_MAX_RADIUS, "apron must hold a block centred r outside the image");
static_assert(SG_APRON_RIGHT >= right_apron_needed(0) && SG_APRON_RIGHT >= right_apron_needed(1) &&
                  SG_APRON_RIGHT >= right_apron_needed(2) && SG_APRON_RIGHT >= right_apron_needed(3) &&
                  SG_MAX_RADIUS <= 3,
              "right apron must hold the 8-byte block-row reads of every radius");
__host__ __device__ __forceinline__ int stored_pitch(int width) {
  return width + SG_APRON + SG_APRON_RIGHT;
}
__host__ __device__ __forceinline__ int stored_rows(int height) { return height + 2 * SG_APRON; }

// Stored-plane index of image pixel (x, y), for x, y at most SG_APRON outside the
// image. A plane has fewer than 2^31 entries and both factors are below 2^24
// (W * H <= 2^22), so the 24-bit multiply is exact and the index is 32-bit.
__device__ __forceinline__ uint32_t padded_index(int x, int y, int pw) {
  return __umul24(static_cast<uint32_t>(y + SG_APRON), static_cast<uint32_t>(pw)) + static_cast<uint32_t>(x + SG_APRON);
}

// The block of stored (r, g, b, depth) pixels around plane entry `at`: each block
// row is fetched as 16-byte loads of two pixels and one 8-byte load of its last
// pixel (three load instructions per row at r = 1 instead of one per pixel; a
// wave's load touches about as many cache lines either way, and the vector memory
// path's cost goes with the lines each instruction touches).
typedef uint64_t __attribute__((ext_vector_type(2))) PixelPairV;
typedef PixelPairV __attribute__((aligned(8))) PixelPair;  // two stored pixels, 8-byte aligned

template <int R>
__device__ __forceinline__ void load_block_pixels(gp<const uint2> plane, uint32_t at, int pw,
                                                  uint2 (&px)[2 * R + 1][2 * R + 1]) {
  constexpr int kSide = 2 * R + 1;
#pragma unroll
  for (int dy = 0; dy < kSide; ++dy) {
    gp<const uint2> row = plane + (at + static_cast<uint32_t>((dy - R) * pw - R));
#pragma unroll
    for (int c = 0; c + 1 < kSide; c += 2) {
      const PixelPairV v = *reinterpret_cast<gp<const PixelPair>>(row + c);
      px[dy][c] = make_uint2(static_cast<uint32_t>(v.x), static_cast<uint32_t>(v.x >> 32));
      px[dy][c + 1] = make_uint2(static_cast<uint32_t>(v.y), static_cast<uint32_t>(v.y >> 32));
    }
    px[dy][kSide - 1] = ld2(row + (kSide - 1));
  }
}

}  // namespace sg

#endif
