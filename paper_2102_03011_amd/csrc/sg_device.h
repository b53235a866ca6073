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
// inside the plane: centres at most r outside the image, blocks 2r + 1 wide.
static_assert(SG_APRON >= 2 * SG_MAX_RADIUS, "apron must hold a block centred r outside the image");
static_assert(SG_APRON_RIGHT >= 2 * SG_MAX_RADIUS, "right apron must hold a block centred r outside the image");
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

// The depth plane pairs its stored rows: entry (P, X) is one 32-bit word holding
// the binary16 depths of stored rows 2P (low half) and 2P + 1 (high half) at
// stored column X, so one load of a block row of words brings two rows of depths.
// A plane has ceil(SH / 2) pair rows (SH = stored rows; for odd SH the last pair's
// high half is apron).
__host__ __device__ __forceinline__ int depth_pair_rows(int height) { return (stored_rows(height) + 1) / 2; }
__host__ __device__ __forceinline__ size_t depth_plane_elems(int width, int height) {
  return static_cast<size_t>(2) * stored_pitch(width) * depth_pair_rows(height);
}
// binary16 entry of image pixel (x, y) (at most SG_APRON outside the image)
__device__ __forceinline__ uint32_t depth_index(int x, int y, int pw) {
  const uint32_t row = static_cast<uint32_t>(y + SG_APRON);
  return 2u * (__umul24(row >> 1, static_cast<uint32_t>(pw)) + static_cast<uint32_t>(x + SG_APRON)) + (row & 1u);
}

// Depth of image pixel (x, y) of frame j (at most SG_APRON outside the image)
__device__ __forceinline__ float depth_at(gp<const uint16_t> depth, int width, int height, int j, int x, int y) {
  return h2f(depth[static_cast<size_t>(j) * depth_plane_elems(width, height) + depth_index(x, y, stored_pitch(width))]);
}

// The (2R + 1)^2 depths (binary16 bits) of the block around image pixel (u, v),
// read from one frame's depth plane (as 32-bit pair words): R + 1 pair rows of
// 2R + 1 words cover the block's rows, whichever row parity v has.
template <int R>
__device__ __forceinline__ void load_block_depths(gp<const uint32_t> plane, int u, int v, int pw,
                                                  uint32_t (&d)[2 * R + 1][2 * R + 1]) {
  constexpr int kSide = 2 * R + 1;
  const int top = v + SG_APRON - R;  // first stored row of the block
  const uint32_t sh = static_cast<uint32_t>(top & 1) * 16u;
  uint32_t wd[R + 1][kSide];
#pragma unroll
  for (int m = 0; m <= R; ++m) {
    gp<const uint32_t> row =
        plane + (__umul24(static_cast<uint32_t>((top >> 1) + m), static_cast<uint32_t>(pw)) +
                 static_cast<uint32_t>(u + SG_APRON - R));
#pragma unroll
    for (int c = 0; c < kSide; ++c) wd[m][c] = row[c];
  }
  // block row k is half (k + s) & 1 of pair word (k + s) >> 1, s = top & 1
#pragma unroll
  for (int c = 0; c < kSide; ++c)
#pragma unroll
    for (int k = 0; k < kSide; ++k) {
      const int m = k >> 1;
      const int m1 = m + 1 <= R ? m + 1 : m;  // the next pair row, when the block reaches it
      const uint64_t win = static_cast<uint64_t>(wd[m][c]) | (m1 > m ? static_cast<uint64_t>(wd[m1][c]) << 32 : 0ull);
      d[k][c] = static_cast<uint32_t>(win >> (sh + 16u * static_cast<uint32_t>(k & 1))) & 0xFFFFu;
    }
}

// The block of stored (r, g, b, depth) pixels around plane entry `at`: each block
// row is fetched as 16-byte loads of two pixels and one 8-byte load of its last
// pixel (two load instructions per row at r = 1 instead of three; a wave's 16-byte
// load touches about as many cache lines as an 8-byte one, and the vector memory
// path's cost goes with the (instruction, cache line) pairs it serves).
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
