// Device kernels of the scene-space gather + filter library (gfx950, wave64).
//
// Gather (Sec. 4): for every output pixel p of frame f with depth d_p, and every
// source frame J of the window, the point X = d_p K^-1 [x, y, 1] is mapped into J
// with the folded float32 map Y = d_p * (M [x, y, 1]) + k (M = K R K^-1, k = K t,
// (R, t) = (C^J)^-1 C^f), projected to (u, v) = (Y1, Y2) / Y3, and the source
// pixels of the (2r+1)^2 block around the rounded projection whose depth agrees
// with z = Y3 to a relative tolerance become members (the depth-guided form of the
// frustum test of Eq. 1-2). Pass 1 counts, a scan turns counts into CSR offsets,
// pass 2 repeats the identical arithmetic and writes the records.
//
// Filter (Sec. 5 Eq. 3, weight of Eq. 4): weighted mean of each set.
//
// All kernels are compiled with -ffp-contract=off; every fused multiply-add is
// written explicitly, so pass 1 and pass 2 make bit-identical decisions.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {

__device__ __forceinline__ float h2f(uint32_t bits16) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16 & 0xFFFFu)));
}

__device__ __forceinline__ uint32_t f2h(float v) {
  return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(v)));
}

// ---------------------------------------------------------------------------
// a1: staging. colour c (0-255) -> binary16(c / 255); depth -> binary16(depth).

__global__ __launch_bounds__(256) void k_stage(const uint8_t* __restrict__ rgb,
                                               const float* __restrict__ depth, int64_t n,
                                               uint2* __restrict__ rgbd,
                                               uint16_t* __restrict__ depth16) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float r = static_cast<float>(rgb[3 * i + 0]) / 255.0f;   // correctly rounded division
  const float g = static_cast<float>(rgb[3 * i + 1]) / 255.0f;
  const float b = static_cast<float>(rgb[3 * i + 2]) / 255.0f;
  const uint32_t d = f2h(depth[i]);
  rgbd[i] = make_uint2(f2h(r) | (f2h(g) << 16), f2h(b) | (d << 16));
  depth16[i] = static_cast<uint16_t>(d);
}

// ---------------------------------------------------------------------------
// a2: relative camera maps, float64 -> float32.
// One thread per (output frame fo, window slot s): J = f - w + s.
// Record layout (kRelStride floats): M row-major (9), k (3), unused (4).

__global__ __launch_bounds__(64) void k_pose_prep(const double* __restrict__ c2w, int n_frames,
                                                  int f0, int n_out, int w, double fx, double fy,
                                                  double cx, double cy, float* __restrict__ rel,
                                                  uint32_t* __restrict__ status) {
  const int slots = 2 * w + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && status != nullptr) *status = 0u;
  if (i >= n_out * slots) return;
  const int fo = i / slots, s = i - fo * slots;
  const int f = f0 + fo, j = f - w + s;
  float* out = rel + static_cast<size_t>(i) * kRelStride;
  double m[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double kt[3] = {0, 0, 0};
  if (j < 0 || j >= n_frames) {
    for (int e = 0; e < kRelStride; ++e) out[e] = 0.0f;
    return;
  }
  if (j != f) {
    const double* a = c2w + static_cast<size_t>(f) * 16;   // C^f
    const double* b = c2w + static_cast<size_t>(j) * 16;   // C^J
    // (C^J)^-1 C^f for rigid maps: R = Rj^T Rf, t = Rj^T (tf - tj)
    double r[9], t[3];
    for (int row = 0; row < 3; ++row) {
      for (int col = 0; col < 3; ++col) {
        double acc = 0.0;
        for (int e = 0; e < 3; ++e) acc = fma(b[e * 4 + row], a[e * 4 + col], acc);
        r[row * 3 + col] = acc;
      }
      double acc = 0.0;
      for (int e = 0; e < 3; ++e) acc = fma(b[e * 4 + row], a[e * 4 + 3] - b[e * 4 + 3], acc);
      t[row] = acc;
    }
    // M = K R K^-1 with K^-1 = [[1/fx, 0, -cx/fx], [0, 1/fy, -cy/fy], [0, 0, 1]]
    const double ifx = 1.0 / fx, ify = 1.0 / fy;
    double a3[9];  // R K^-1
    for (int row = 0; row < 3; ++row) {
      a3[row * 3 + 0] = r[row * 3 + 0] * ifx;
      a3[row * 3 + 1] = r[row * 3 + 1] * ify;
      a3[row * 3 + 2] = r[row * 3 + 2] - r[row * 3 + 0] * cx * ifx - r[row * 3 + 1] * cy * ify;
    }
    for (int col = 0; col < 3; ++col) {
      m[0 * 3 + col] = fx * a3[0 * 3 + col] + cx * a3[2 * 3 + col];
      m[1 * 3 + col] = fy * a3[1 * 3 + col] + cy * a3[2 * 3 + col];
      m[2 * 3 + col] = a3[2 * 3 + col];
    }
    kt[0] = fx * t[0] + cx * t[2];
    kt[1] = fy * t[1] + cy * t[2];
    kt[2] = t[2];
  }
  for (int e = 0; e < 9; ++e) out[e] = static_cast<float>(m[e]);
  for (int e = 0; e < 3; ++e) out[9 + e] = static_cast<float>(kt[e]);
  out[12] = 1.0f;  // slot valid
  out[13] = out[14] = out[15] = 0.0f;
}

// ---------------------------------------------------------------------------
// Shared projection (identical in both gather passes).

struct Projected {
  float z, tz, inv;
  int iu, iv;
};

__device__ __forceinline__ bool project(const float* __restrict__ m, float x, float y, float dp,
                                        float z_near, float tol, int width, int height, int r,
                                        Projected& o) {
  const float a0 = fmaf(m[0], x, fmaf(m[1], y, m[2]));
  const float a1 = fmaf(m[3], x, fmaf(m[4], y, m[5]));
  const float a2 = fmaf(m[6], x, fmaf(m[7], y, m[8]));
  const float y0 = fmaf(dp, a0, m[9]);
  const float y1 = fmaf(dp, a1, m[10]);
  const float z = fmaf(dp, a2, m[11]);
  if (!(z > z_near)) return false;
  const float inv = __builtin_amdgcn_rcpf(z);
  const float uh = floorf(y0 * inv + 0.5f);
  const float vh = floorf(y1 * inv + 0.5f);
  const float fr = static_cast<float>(r);
  if (!(uh >= -fr && uh <= static_cast<float>(width - 1) + fr && vh >= -fr &&
        vh <= static_cast<float>(height - 1) + fr))
    return false;
  o.z = z;
  o.tz = tol * z;
  o.inv = inv;
  o.iu = static_cast<int>(uh);
  o.iv = static_cast<int>(vh);
  return true;
}

__device__ __forceinline__ bool accept(float dq, const Projected& p) {
  return dq > 0.0f && fabsf(dq - p.z) <= p.tz;
}

// ---------------------------------------------------------------------------
// a3: gather pass 1 -- count members per output pixel.
// Block = 64 x 4 pixels (one wave per row segment), grid.z = output frame.

template <int R>
__global__ __launch_bounds__(256) void k_count(const uint16_t* __restrict__ depth,
                                               const float* __restrict__ rel, int width, int height,
                                               int n_frames, int f0, int w, float tol, float z_near,
                                               int64_t* __restrict__ counts) {
  const int x = blockIdx.x * kTileW + threadIdx.x;
  const int y = blockIdx.y * kTileH + threadIdx.y;
  const int fo = blockIdx.z;
  if (x >= width || y >= height) return;
  const int f = f0 + fo;
  const size_t plane = static_cast<size_t>(width) * height;
  const size_t self = static_cast<size_t>(y) * width + x;
  const float dp = h2f(depth[static_cast<size_t>(f) * plane + self]);
  int count = 0;
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
    for (int j = jlo; j <= jhi; ++j) {
      Projected p;
      if (!project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p))
        continue;
      const uint16_t* dj = depth + static_cast<size_t>(j) * plane;
#pragma unroll
      for (int dy = -R; dy <= R; ++dy) {
        const int row = p.iv + dy;
        if (row < 0 || row >= height) continue;
        const uint16_t* drow = dj + static_cast<size_t>(row) * width;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
          const int col = p.iu + dx;
          if (col < 0 || col >= width) continue;
          count += accept(h2f(drow[col]), p) ? 1 : 0;
        }
      }
    }
  }
  counts[static_cast<size_t>(fo) * plane + self] = count;
}

// ---------------------------------------------------------------------------
// a5: gather pass 2 -- write records in canonical order.

template <int R>
__global__ __launch_bounds__(256) void k_scatter(const uint2* __restrict__ rgbd,
                                                 const float* __restrict__ rel, int width,
                                                 int height, int n_frames, int f0, int w, float tol,
                                                 float z_near, const int64_t* __restrict__ offsets,
                                                 uint32_t* __restrict__ ids,
                                                 uint2* __restrict__ crho, int64_t capacity,
                                                 uint32_t* __restrict__ status) {
  const int x = blockIdx.x * kTileW + threadIdx.x;
  const int y = blockIdx.y * kTileH + threadIdx.y;
  const int fo = blockIdx.z;
  if (x >= width || y >= height) return;
  const int f = f0 + fo;
  const size_t plane = static_cast<size_t>(width) * height;
  const size_t self = static_cast<size_t>(y) * width + x;
  const size_t pix = static_cast<size_t>(fo) * plane + self;
  int64_t cur = offsets[pix];
  const int64_t end = offsets[pix + 1];
  if (cur < 0 || end < cur) {  // offsets not produced by the count pass
    atomicOr(status, SG_FLAG_INCONSISTENT);
    return;
  }
  if (end > capacity) {
    if (end > cur) atomicOr(status, SG_FLAG_CAPACITY);
    return;
  }
  const float dp = h2f(rgbd[static_cast<size_t>(f) * plane + self].y >> 16);
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
    for (int j = jlo; j <= jhi; ++j) {
      Projected p;
      if (!project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p))
        continue;
      const uint2* cj = rgbd + static_cast<size_t>(j) * plane;
      const uint32_t idj = static_cast<uint32_t>(j - f + w) << SG_ID_SHIFT;
#pragma unroll
      for (int dy = -R; dy <= R; ++dy) {
        const int row = p.iv + dy;
        if (row < 0 || row >= height) continue;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
          const int col = p.iu + dx;
          if (col < 0 || col >= width) continue;
          const uint32_t q = static_cast<uint32_t>(row * width + col);
          const uint2 px = cj[q];
          const float dq = h2f(px.y >> 16);
          if (accept(dq, p)) {
            if (cur < end) {
              const float rho = (dq - p.z) * p.inv;
              ids[cur] = idj | q;
              crho[cur] = make_uint2(px.x, (px.y & 0xFFFFu) | (f2h(rho) << 16));
            }
            ++cur;
          }
        }
      }
    }
  }
  if (cur != end) atomicOr(status, SG_FLAG_INCONSISTENT);
}

// ---------------------------------------------------------------------------
// a4: scan. counts live in offsets[1..P]; three phases turn them into an
// inclusive scan in place, and offsets[0] = 0.

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* lds, int64_t* total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t add = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const int64_t incl = lds[t];
  *total = lds[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int64_t* __restrict__ data,
                                                              int64_t n,
                                                              int64_t* __restrict__ partial) {
  __shared__ int64_t lds[kScanThreads];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int64_t s = 0;
  for (int e = threadIdx.x; e < kScanTile; e += kScanThreads) {
    const int64_t i = base + e;
    if (i < n) s += data[i];
  }
  int64_t total;
  block_exclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int64_t* __restrict__ partial,
                                                                int64_t nb) {
  __shared__ int64_t lds[kScanThreads];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? partial[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, lds, &total);
    if (i < nb) partial[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int64_t* __restrict__ offsets,
                                                             int64_t n,
                                                             const int64_t* __restrict__ partial) {
  __shared__ int64_t lds[kScanThreads];
  int64_t* data = offsets + 1;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  constexpr int kPer = kScanTile / kScanThreads;
  // each thread owns kPer consecutive elements
  int64_t vals[kPer];
  int64_t s = 0;
  const int64_t mine = base + static_cast<int64_t>(threadIdx.x) * kPer;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int64_t i = mine + e;
    vals[e] = i < n ? data[i] : 0;
    s += vals[e];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(s, lds, &total) + partial[blockIdx.x];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int64_t i = mine + e;
    run += vals[e];
    if (i < n) data[i] = run;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

// ---------------------------------------------------------------------------
// a6: filter. kGroup lanes per output pixel stride through its CSR segment;
// each lane accumulates in a fixed order, then a fixed butterfly reduces.

template <bool kColour, bool kTime>
__global__ __launch_bounds__(256) void k_filter(const uint2* __restrict__ rgbd, int width,
                                                int height, int f0, int w, int64_t n_pix,
                                                const int64_t* __restrict__ offsets,
                                                const uint32_t* __restrict__ ids,
                                                const uint2* __restrict__ crho, int64_t capacity,
                                                float a_d, float a_c, float a_t,
                                                float* __restrict__ out) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t pix = gid / kGroup;
  const int lane = static_cast<int>(gid % kGroup);
  const bool live = pix < n_pix;
  const size_t plane = static_cast<size_t>(width) * height;
  float cr = 0.f, cg = 0.f, cb = 0.f;
  int64_t s = 0, e = 0;
  int fo = 0;
  if (live) {
    fo = static_cast<int>(pix / static_cast<int64_t>(plane));
    const size_t self = static_cast<size_t>(pix - static_cast<int64_t>(fo) * plane);
    const uint2 ref = rgbd[static_cast<size_t>(f0 + fo) * plane + self];
    cr = h2f(ref.x);
    cg = h2f(ref.x >> 16);
    cb = h2f(ref.y);
    s = offsets[pix];
    e = offsets[pix + 1];
  }
  // a set that did not fit the arena (or malformed offsets) yields NaN, never a read past it
  const bool bad = live && (s < 0 || e < s || e > capacity);
  if (bad) s = e = 0;
  float wsum = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
  for (int64_t i = s + lane; i < e; i += kGroup) {
    const uint2 rec = crho[i];
    const float r = h2f(rec.x), g = h2f(rec.x >> 16), b = h2f(rec.y), rho = h2f(rec.y >> 16);
    float arg = a_d * rho * rho;
    if (kColour) {
      const float dr = r - cr, dg = g - cg, db = b - cb;
      arg = fmaf(a_c, fmaf(dr, dr, fmaf(dg, dg, db * db)), arg);
    }
    if (kTime) {
      const float dj = static_cast<float>(static_cast<int>(ids[i] >> SG_ID_SHIFT) - w);
      arg = fmaf(a_t, dj * dj, arg);
    }
    const float wt = __builtin_amdgcn_exp2f(arg);
    wsum += wt;
    ar = fmaf(wt, r, ar);
    ag = fmaf(wt, g, ag);
    ab = fmaf(wt, b, ab);
  }
#pragma unroll
  for (int off = kGroup / 2; off > 0; off >>= 1) {
    wsum += __shfl_xor(wsum, off, kGroup);
    ar += __shfl_xor(ar, off, kGroup);
    ag += __shfl_xor(ag, off, kGroup);
    ab += __shfl_xor(ab, off, kGroup);
  }
  if (live && lane == 0) {
    float* o = out + static_cast<size_t>(pix) * 3;
    if (bad) {
      o[0] = o[1] = o[2] = __builtin_nanf("");
    } else if (e > s) {
      const float inv = 1.0f / wsum;
      o[0] = ar * inv;
      o[1] = ag * inv;
      o[2] = ab * inv;
    } else {
      o[0] = cr;
      o[1] = cg;
      o[2] = cb;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_stage(const uint8_t* rgb, const float* depth, int64_t n, uint16_t* rgbd,
                        uint16_t* depth16, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_stage, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, rgb, depth, n,
                     reinterpret_cast<uint2*>(rgbd), depth16);
  return hipGetLastError();
}

hipError_t launch_pose_prep(const GatherJob& jb, hipStream_t st) {
  const int n = jb.n_out * (2 * jb.w + 1);
  hipLaunchKernelGGL(k_pose_prep, dim3((n + 63) / 64), dim3(64), 0, st, jb.c2w, jb.n_frames, jb.f0,
                     jb.n_out, jb.w, jb.fx, jb.fy, jb.cx, jb.cy, jb.rel, jb.status);
  return hipGetLastError();
}

template <int R>
static void count_r(const GatherJob& jb, dim3 g, hipStream_t st) {
  hipLaunchKernelGGL(k_count<R>, g, dim3(kTileW, kTileH), 0, st, jb.depth, jb.rel, jb.width,
                     jb.height, jb.n_frames, jb.f0, jb.w, jb.tol, jb.z_near, jb.offsets + 1);
}

template <int R>
static void scatter_r(const GatherJob& jb, dim3 g, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter<R>, g, dim3(kTileW, kTileH), 0, st,
                     reinterpret_cast<const uint2*>(jb.rgbd), jb.rel, jb.width, jb.height,
                     jb.n_frames, jb.f0, jb.w, jb.tol, jb.z_near, jb.offsets, jb.ids,
                     reinterpret_cast<uint2*>(jb.crho), jb.capacity, jb.status);
}

static dim3 gather_grid(const GatherJob& jb) {
  return dim3((jb.width + kTileW - 1) / kTileW, (jb.height + kTileH - 1) / kTileH, jb.n_out);
}

hipError_t launch_count(const GatherJob& jb, hipStream_t st) {
  const dim3 g = gather_grid(jb);
  switch (jb.radius) {
    case 0: count_r<0>(jb, g, st); break;
    case 1: count_r<1>(jb, g, st); break;
    case 2: count_r<2>(jb, g, st); break;
    default: count_r<3>(jb, g, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_scan(int64_t* offsets, int64_t n, int64_t* partial, hipStream_t st) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    // no pixels: offsets[0] = 0 still has to be written
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, st, offsets, n, partial);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st,
                     offsets + 1, n, partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partial, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(kScanThreads), 0, st,
                     offsets, n, partial);
  return hipGetLastError();
}

hipError_t launch_scatter(const GatherJob& jb, hipStream_t st) {
  const dim3 g = gather_grid(jb);
  switch (jb.radius) {
    case 0: scatter_r<0>(jb, g, st); break;
    case 1: scatter_r<1>(jb, g, st); break;
    case 2: scatter_r<2>(jb, g, st); break;
    default: scatter_r<3>(jb, g, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_filter(const FilterJob& fj, hipStream_t st) {
  const int64_t threads = fj.n_pix * kGroup;
  if (threads == 0) return hipSuccess;
  const dim3 g(static_cast<unsigned>((threads + 255) / 256));
  const uint2* rgbd = reinterpret_cast<const uint2*>(fj.rgbd);
  const uint2* crho = reinterpret_cast<const uint2*>(fj.crho);
  if (fj.use_colour && fj.use_time)
    hipLaunchKernelGGL((k_filter<true, true>), g, dim3(256), 0, st, rgbd, fj.width, fj.height, fj.f0,
                       fj.w, fj.n_pix, fj.offsets, fj.ids, crho, fj.capacity, fj.a_d, fj.a_c, fj.a_t, fj.out);
  else if (fj.use_colour)
    hipLaunchKernelGGL((k_filter<true, false>), g, dim3(256), 0, st, rgbd, fj.width, fj.height,
                       fj.f0, fj.w, fj.n_pix, fj.offsets, fj.ids, crho, fj.capacity, fj.a_d, fj.a_c,
                       fj.a_t, fj.out);
  else if (fj.use_time)
    hipLaunchKernelGGL((k_filter<false, true>), g, dim3(256), 0, st, rgbd, fj.width, fj.height,
                       fj.f0, fj.w, fj.n_pix, fj.offsets, fj.ids, crho, fj.capacity, fj.a_d, fj.a_c,
                       fj.a_t, fj.out);
  else
    hipLaunchKernelGGL((k_filter<false, false>), g, dim3(256), 0, st, rgbd, fj.width, fj.height,
                       fj.f0, fj.w, fj.n_pix, fj.offsets, fj.ids, crho, fj.capacity, fj.a_d, fj.a_c,
                       fj.a_t, fj.out);
  return hipGetLastError();
}

}  // namespace sg
