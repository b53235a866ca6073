// Depth-agnostic frustum gather (Sec. 4, Eq. 1-2).
//
// The paper rasterises, per output pixel p and window frame J, the convex hull of
// p's frustum projected into J, an epipolar band that can cross the whole image,
// and tests every pixel in it. Its dual is what the GPU runs here: a source pixel
// q of J reaches only the output pixels within L1 distance l/2 of its point p'(q)
// carried into the output view. Per window frame:
//   carry   -- every q: p'(q), z'(q) in float32; q is kept when its depth is valid
//              and near <= z' <= far, and filed under its nearest output pixel
//              b(q) = round(p'(q)) on a grid extended by the bucket radius rb
//              (a member has |p - b(q)|_1 < l/2 + 1, so rb = ceil(l/2 + 1) - 1);
//              the bucket's counter hands q its slot (the order inside a bucket is
//              arbitrary);
//   bucket  -- after a scan of the counters, q is filed at its bucket's start plus
//              its slot, with p'(q), z'(q) (computed again, the same float32
//              arithmetic) and its stored colour, so a row of buckets is one
//              contiguous range of records and the scatter reads no source plane;
//   count / scatter -- each output pixel reads the buckets within L1 distance rb,
//              applies Eq. 2, and (scatter) orders its members of J by q in a small
//              per-thread sort, so the records come out in canonical order whatever
//              order the buckets hold.
// The member counts are scanned into the caller's CSR offsets between the passes.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <climits>
#include <type_traits>

#include "scene_frustum.h"
#include "sg_device.h"
#include "sg_internal.h"
#include "sg_validate.h"

namespace sg {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// 16-byte stores at 8- and 4-byte aligned positions (global memory takes unaligned
// dword accesses)
typedef uint32_t u32x4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));

constexpr int kMapFloats = 16;  // per window frame: M (3x3, row-major), k (3), padding
constexpr int kThreads = 256;

// a filed source pixel: p' = (x, y), z', q, and its stored r, g, b, depth (binary16)
struct __attribute__((aligned(32))) Filed {
  float x, y, z;
  int32_t q;
  uint32_t rg, bd;
  uint32_t pad[2];
};
static_assert(sizeof(Filed) == 32, "two 16-byte words per record");
// The count pass reads p' only: the bucket pass also writes it to an array of its
// own (8 B per record), so the count stages a quarter of the bytes.

int bucket_radius(float l) { return static_cast<int>(ceilf(0.5f * l + 1.0f)) - 1; }

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

struct FrustumLayout {
  int jlo, n_j, rb;
  int64_t n_pix, n_buckets;  // per window frame
  size_t maps, slots, counts, boff, items, xy, partial, total;
};

FrustumLayout frustum_layout(const sg_clip* c, int32_t f, const sg_frustum_params* p) {
  FrustumLayout l{};
  l.jlo = f - p->window > 0 ? f - p->window : 0;
  const int jhi = f + p->window < c->num_frames - 1 ? f + p->window : c->num_frames - 1;
  l.n_j = jhi - l.jlo + 1;
  l.rb = bucket_radius(p->l);
  l.n_pix = static_cast<int64_t>(c->width) * c->height;
  l.n_buckets = static_cast<int64_t>(c->width + 2 * l.rb) * (c->height + 2 * l.rb);
  const int64_t scan_a = (l.n_j * l.n_buckets + kScanTile - 1) / kScanTile;
  const int64_t scan_b = (l.n_pix + kScanTile - 1) / kScanTile;
  size_t at = 0;
  l.maps = at;
  at += align_up(static_cast<size_t>(l.n_j) * kMapFloats * sizeof(float));
  l.slots = at;
  at += align_up(static_cast<size_t>(l.n_j) * l.n_pix * sizeof(int2));
  l.counts = at;
  at += align_up(static_cast<size_t>(l.n_j) * l.n_buckets * sizeof(uint32_t));
  l.boff = at;
  at += align_up((static_cast<size_t>(l.n_j) * l.n_buckets + 1) * sizeof(int64_t));
  l.items = at;
  at += align_up(static_cast<size_t>(l.n_j) * l.n_pix * sizeof(Filed));
  l.xy = at;
  at += align_up(static_cast<size_t>(l.n_j) * l.n_pix * sizeof(uint2));
  l.partial = at;
  at += align_up(static_cast<size_t>((scan_a > scan_b ? scan_a : scan_b) + 1) * sizeof(int64_t));
  l.total = at;
  return l;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(T* __restrict__ p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = T(0);
}

// Scan of the 32-bit bucket counters into the 64-bit bucket offsets (offsets[0] =
// 0, offsets[1 + i] = counts[0] + ... + counts[i]): block sums over kScanTile
// counters, a scan of the block sums, then each block's scan plus its start.
__device__ __forceinline__ int64_t block_scan_excl(int64_t v, int64_t* lds, int64_t* total) {
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

__global__ __launch_bounds__(kScanThreads) void k_count_sums(const uint32_t* __restrict__ counts, int64_t n,
                                                             int64_t* __restrict__ partial) {
  __shared__ int64_t lds[kScanThreads];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  int64_t s = 0;
  for (int e = threadIdx.x; e < kScanTile; e += kScanThreads) {
    const int64_t i = base + e;
    if (i < n) s += counts[i];
  }
  int64_t total;
  block_scan_excl(s, lds, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_count_sums_scan(int64_t* __restrict__ partial, int64_t nb) {
  __shared__ int64_t lds[kScanThreads];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? partial[i] : 0;
    int64_t total;
    const int64_t ex = block_scan_excl(v, lds, &total);
    if (i < nb) partial[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_count_offsets(const uint32_t* __restrict__ counts, int64_t n,
                                                                const int64_t* __restrict__ partial,
                                                                int64_t* __restrict__ offsets) {
  __shared__ int64_t lds[kScanThreads];
  constexpr int kPer = kScanTile / kScanThreads;
  const int64_t mine = static_cast<int64_t>(blockIdx.x) * kScanTile + static_cast<int64_t>(threadIdx.x) * kPer;
  uint32_t vals[kPer];
  int64_t s = 0;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    vals[e] = mine + e < n ? counts[mine + e] : 0u;
    s += vals[e];
  }
  int64_t total;
  int64_t run = block_scan_excl(s, lds, &total) + partial[blockIdx.x];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    run += vals[e];
    if (mine + e < n) offsets[1 + mine + e] = run;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

// (C^f)^-1 C^J in float64 (rigid: the inverse rotation is the transpose), folded
// with K: a pixel (x, y) of J with depth d goes to Y = d M (x, y, 1) + k, z' = Y_3,
// p' = (Y_1, Y_2) / Y_3. J = f gives exactly M = I, k = 0.
__global__ __launch_bounds__(64) void k_frustum_pose(const double* __restrict__ c2w, int f, int jlo, int n_j,
                                                     double fx, double fy, double cx, double cy,
                                                     float* __restrict__ maps, uint32_t* __restrict__ status) {
  if (threadIdx.x == 0) *status = 0u;  // the count pass starts a new set of flags
  for (int jn = threadIdx.x; jn < n_j; jn += 64) {
    const int j = jlo + jn;
    float* m = maps + jn * kMapFloats;
    for (int i = 0; i < kMapFloats; ++i) m[i] = 0.0f;
    if (j == f) {
      m[0] = m[4] = m[8] = 1.0f;
      continue;
    }
    const double* a = c2w + static_cast<size_t>(f) * 16;
    const double* b = c2w + static_cast<size_t>(j) * 16;
    double r[3][3], t[3], am[3][3];
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) r[i][k] = a[i] * b[k] + a[4 + i] * b[4 + k] + a[8 + i] * b[8 + k];
      t[i] = a[i] * (b[3] - a[3]) + a[4 + i] * (b[7] - a[7]) + a[8 + i] * (b[11] - a[11]);
    }
    for (int i = 0; i < 3; ++i) {  // R K^-1
      am[i][0] = r[i][0] / fx;
      am[i][1] = r[i][1] / fy;
      am[i][2] = r[i][2] - r[i][0] * cx / fx - r[i][1] * cy / fy;
    }
    for (int k = 0; k < 3; ++k) {  // K R K^-1
      m[k] = static_cast<float>(fx * am[0][k] + cx * am[2][k]);
      m[3 + k] = static_cast<float>(fy * am[1][k] + cy * am[2][k]);
      m[6 + k] = static_cast<float>(am[2][k]);
    }
    m[9] = static_cast<float>(fx * t[0] + cx * t[2]);
    m[10] = static_cast<float>(fy * t[1] + cy * t[2]);
    m[11] = static_cast<float>(t[2]);
  }
}

// p'(q), z'(q) of source pixel (x, y) of window frame jn; its bucket, or -1 when q is
// not kept (invalid depth, z' outside [near, far], or p' beyond the extended grid).
// The carry and bucket passes both call it, so both see the same floats.
__device__ __forceinline__ int carry_point(gp<const uint16_t> depth, gp<const float> m, int width, int height,
                                           int jn_plane_frame, int x, int y, int rb, float near_z, float far_z,
                                           float& px, float& py, float& z) {
  const int pw = stored_pitch(width);
  const float d = h2f(depth[static_cast<size_t>(jn_plane_frame) * depth_plane_elems(width, height) + depth_index(x, y, pw)]);
  px = py = z = 0.0f;
  if (!(d > 0.0f && d < INFINITY)) return -1;
  const float fx = static_cast<float>(x), fy = static_cast<float>(y);
  const float y0 = fmaf(d, fmaf(m[0], fx, fmaf(m[1], fy, m[2])), m[9]);
  const float y1 = fmaf(d, fmaf(m[3], fx, fmaf(m[4], fy, m[5])), m[10]);
  z = fmaf(d, fmaf(m[6], fx, fmaf(m[7], fy, m[8])), m[11]);
  if (!(z >= near_z && z <= far_z)) return -1;
  px = y0 / z;
  py = y1 / z;
  const float ex = px + 0.5f, ey = py + 0.5f;
  // NaN fails every comparison; the bounds keep b inside the extended grid
  if (!(ex >= static_cast<float>(-rb) && ex < static_cast<float>(width + rb) && ey >= static_cast<float>(-rb) &&
        ey < static_cast<float>(height + rb)))
    return -1;
  const int bx = static_cast<int>(floorf(ex)), by = static_cast<int>(floorf(ey));
  return (by + rb) * (width + 2 * rb) + (bx + rb);
}

// grid (pixels / 256, window frames): the bucket of every q and its slot in it
__global__ __launch_bounds__(kThreads) void k_frustum_carry(const uint16_t* __restrict__ depth,
                                                            const float* __restrict__ maps, int width, int height,
                                                            int jlo, int rb, float near_z, float far_z, int64_t n_pix,
                                                            int64_t n_buckets, int2* __restrict__ slots,
                                                            unsigned int* __restrict__ bcount) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= n_pix) return;
  const int jn = blockIdx.y;
  const int y = static_cast<int>(q / width), x = static_cast<int>(q - static_cast<int64_t>(y) * width);
  float px, py, z;
  const int b = carry_point(to_global(depth), to_global(maps) + jn * kMapFloats, width, height, jlo + jn, x, y, rb,
                            near_z, far_z, px, py, z);
  int slot = 0;
  if (b >= 0)
    slot = static_cast<int>(atomicAdd(bcount + static_cast<int64_t>(jn) * n_buckets + b, 1u));
  slots[static_cast<int64_t>(jn) * n_pix + q] = make_int2(b, slot);
}

// grid (pixels / 256, window frames): file every kept q at its bucket's start plus its
// slot, so the count and scatter passes read each bucket's candidates contiguously
__global__ __launch_bounds__(kThreads) void k_frustum_bucket(const uint2* __restrict__ rgbd,
                                                             const uint16_t* __restrict__ depth,
                                                             const float* __restrict__ maps, int width, int height,
                                                             int jlo, int rb, float near_z, float far_z,
                                                             const int2* __restrict__ slots,
                                                             const int64_t* __restrict__ boff, int64_t n_pix,
                                                             int64_t n_buckets, Filed* __restrict__ filed,
                                                             uint2* __restrict__ fxy) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= n_pix) return;
  const int jn = blockIdx.y;
  const int2 bs = slots[static_cast<int64_t>(jn) * n_pix + q];
  if (bs.x < 0) return;
  const int y = static_cast<int>(q / width), x = static_cast<int>(q - static_cast<int64_t>(y) * width);
  float px, py, z;
  carry_point(to_global(depth), to_global(maps) + jn * kMapFloats, width, height, jlo + jn, x, y, rb, near_z, far_z,
              px, py, z);
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const uint2 c = ld2(to_global(rgbd) + static_cast<size_t>(jlo + jn) * pplane + padded_index(x, y, pw));
  const int64_t at = to_global(boff)[static_cast<int64_t>(jn) * n_buckets + bs.x] + bs.y;
  gp<u32x4> out = reinterpret_cast<gp<u32x4>>(to_global(filed) + at);
  out[0] = u32x4{__float_as_uint(px), __float_as_uint(py), __float_as_uint(z), static_cast<uint32_t>(q)};
  out[1] = u32x4{c.x, c.y, 0u, 0u};
  st2(to_global(fxy) + at, make_uint2(__float_as_uint(px), __float_as_uint(py)));
}

// Calls fn(q, z', k) for every q filed (at index k) within L1 distance rb of output
// pixel (x, y) in window frame jn and passing Eq. 2 (kXy: positions from the p'
// array only, fn gets q = z' = 0).
template <bool kXy, typename Fn>
__device__ __forceinline__ void for_members(const Filed* __restrict__ filed_, const uint2* __restrict__ fxy_,
                                            const int64_t* __restrict__ boff, int width, int rb, float half,
                                            int64_t n_buckets, int jn, int x, int y, Fn&& fn) {
  gp<const u32x4> filed = reinterpret_cast<gp<const u32x4>>(to_global(filed_));
  gp<const uint2> fxy = to_global(fxy_);
  gp<const int64_t> bj = to_global(boff) + static_cast<int64_t>(jn) * n_buckets;
  const int ew = width + 2 * rb;
  const float fx = static_cast<float>(x), fy = static_cast<float>(y);
  for (int dy = -rb; dy <= rb; ++dy) {
    const int span = rb - (dy < 0 ? -dy : dy);
    const int64_t row = static_cast<int64_t>(y + dy + rb) * ew + (x + rb);
    // the buckets of this row are adjacent: one contiguous range of filed records
    const int64_t k0 = bj[row - span], k1 = bj[row + span + 1];
    for (int64_t k = k0; k < k1; ++k) {
      u32x4 w;
      if (kXy) {
        const uint2 v = ld2(fxy + k);
        w = u32x4{v.x, v.y, 0u, 0u};
      } else {
        w = filed[2 * k];
      }
      if (fabsf(fx - __uint_as_float(w[0])) + fabsf(fy - __uint_as_float(w[1])) < half)
        fn(static_cast<int32_t>(w[3]), __uint_as_float(w[2]), k);
    }
  }
}

// Count and scatter run on 16 x 16 tiles of output pixels, one thread each. Per
// window frame the workgroup first copies the buckets its pixels can reach (kTile +
// 2 rb rows of kTile + 2 rb buckets; each row is one contiguous range of filed
// records) into LDS with loads spread over all its threads, then every thread reads
// its 2 rb (rb + 1) + 1 buckets from there. A frame whose reachable records do not
// fit (more than kStageCap: points of a wide depth range crowding into few buckets)
// is read from global memory by every thread instead, as for_members does.
constexpr int kTile = 16;
constexpr int kMaxRb = 4;  // bucket_radius(SG_MAX_FRUSTUM_L)
constexpr int kStageSide = kTile + 2 * kMaxRb;
constexpr int kStageCap = 768;
constexpr int kBoundsPerThread = (kStageSide * (kStageSide + 1) + kThreads - 1) / kThreads;
static_assert(kThreads == kTile * kTile, "one thread per pixel of a tile");

// records staged per window frame (kColour: with their colours, for the scatter)
template <bool kColour>
struct StageLds {
  // x, y, z', q (scatter) or x, y (count) of the staged rows' records, row after row
  typename std::conditional<kColour, u32x4, uint2>::type rec[kStageCap];
  uint2 col[kColour ? kStageCap : 1];       // their r, g, b, depth
  int32_t loc[kStageSide][kStageSide + 1];  // rec index of bucket (row, column); [r][ncols] = row end
  int32_t base[kStageSide + 1];             // rec index of each row's first record; [nrows] = total
  int64_t first[kStageSide];                // filed index of each row's first record
  int32_t base_next[kStageSide + 1];        // the same for the next window frame (whole tile)
  int64_t first_next[kStageSide];
};

struct TileGeom {
  int tx0, ty0;       // first output pixel of the tile = first staged bucket (extended grid)
  int nrows, ncols;   // staged bucket rows and columns that exist in the extended grid
};

__device__ __forceinline__ TileGeom tile_geom(int width, int height, int rb) {
  const int tiles_x = (width + kTile - 1) / kTile;
  const int nt = tiles_x * ((height + kTile - 1) / kTile);
  // whole tile rows per XCD: the dispatcher hands consecutive workgroups to the
  // eight XCDs in turn, so workgroup b runs on XCD b % 8
  const int bl = static_cast<int>(blockIdx.x);
  const int full = (nt / (8 * tiles_x)) * (8 * tiles_x);
  int tl = bl;
  if (bl < full) {
    const int xcd = bl & 7, i = bl >> 3;
    const int q = i / tiles_x, p = i - q * tiles_x;
    tl = (q * 8 + xcd) * tiles_x + p;
  }
  TileGeom g;
  g.tx0 = (tl % tiles_x) * kTile;
  g.ty0 = (tl / tiles_x) * kTile;
  g.nrows = min(kTile + 2 * rb, height + 2 * rb - g.ty0);
  g.ncols = min(kTile + 2 * rb, width + 2 * rb - g.tx0);
  return g;
}

// The first and end filed index of staged row t (threads t < nrows) of a window
// frame: loaded one frame ahead, while the workgroup works on the frame before.
struct RowSpan {
  int64_t a, e;
};
__device__ __forceinline__ RowSpan row_span(gp<const int64_t> bj, int ew, const TileGeom& g, int r0, int r1) {
  const int t = threadIdx.x;
  RowSpan r{0, 0};
  if (t < r1 - r0) {
    const int64_t row = static_cast<int64_t>(g.ty0 + r0 + t) * ew + g.tx0;
    r.a = bj[row];
    r.e = bj[row + g.ncols];
  }
  return r;
}

// Stages the tile's bucket rows [r0, r1) of one window frame (rs: this thread's
// row_span of those rows); false (nothing staged) when their records number more
// than kStageCap. Every thread of the workgroup calls it; it ends on a barrier
// either way, and the caller puts one between its last read of the staged records
// and the next call.
template <bool kColour>
__device__ bool stage_rows(gp<const u32x4> filed, gp<const uint2> fxy, gp<const int64_t> bj, int ew,
                           const TileGeom& g, int r0, int r1, RowSpan rs, StageLds<kColour>& s) {
  const int t = threadIdx.x;
  const int nr = r1 - r0;
  if (t < nr) {
    s.first[t] = rs.a;
    s.base[t + 1] = static_cast<int32_t>(min(rs.e - rs.a, static_cast<int64_t>(kStageCap) + 1));
  }
  __syncthreads();
  if (t == 0) {  // row starts (at most kStageSide rows; clamped counts cannot overflow)
    int acc = 0;
    s.base[0] = 0;
    for (int r = 0; r < nr; ++r) {
      acc = min(acc + s.base[r + 1], kStageCap + 1);
      s.base[r + 1] = acc;
    }
  }
  __syncthreads();
  const int total = s.base[nr];
  if (total > kStageCap) {  // uniform: every thread read the same LDS word
    __syncthreads();        // ... before the next call rewrites it
    return false;
  }
  // bucket starts relative to the staged rows, and the records, loads issued together
  int64_t gb[kBoundsPerThread];
  int ib[kBoundsPerThread];
#pragma unroll
  for (int k = 0; k < kBoundsPerThread; ++k) {
    const int i = t + k * kThreads;
    ib[k] = i < nr * (g.ncols + 1) ? i : -1;
    if (ib[k] >= 0) {
      const int r = i / (g.ncols + 1), c = i - r * (g.ncols + 1);
      gb[k] = bj[static_cast<int64_t>(g.ty0 + r0 + r) * ew + g.tx0 + c];
    }
  }
  constexpr int kRecPerThread = kStageCap / kThreads;
  static_assert(kRecPerThread * kThreads == kStageCap, "whole records per thread");
  typename std::conditional<kColour, u32x4, uint2>::type v[kRecPerThread];
  uint2 cv[kRecPerThread];
#pragma unroll
  for (int k = 0; k < kRecPerThread; ++k) {
    const int i = t + k * kThreads;
    if (i < total) {
      int lo = 0, hi = nr - 1;  // row r with base[r] <= i < base[r + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.base[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const int64_t at = s.first[lo] + (i - s.base[lo]);
      if constexpr (kColour) {
        v[k] = filed[2 * at];
        const u32x4 w = filed[2 * at + 1];
        cv[k] = make_uint2(w[0], w[1]);
      } else {
        v[k] = ld2(fxy + at);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kBoundsPerThread; ++k) {
    if (ib[k] >= 0) {
      const int r = ib[k] / (g.ncols + 1), c = ib[k] - r * (g.ncols + 1);
      s.loc[r][c] = s.base[r] + static_cast<int32_t>(gb[k] - s.first[r]);
    }
  }
#pragma unroll
  for (int k = 0; k < kRecPerThread; ++k)
    if (t + k * kThreads < total) {
      s.rec[t + k * kThreads] = v[k];
      if constexpr (kColour) s.col[t + k * kThreads] = cv[k];
    }
  __syncthreads();
  return true;
}

// for_members over the staged records of rows [r0, ...): fn(q, z', staged index)
// (thread's pixel (x, y) = (tx0 + tx, ty0 + ty)).
template <bool kColour, typename Fn>
__device__ __forceinline__ void for_members_staged(const StageLds<kColour>& s, int r0, int rb, float half, int tx,
                                                   int ty, int x, int y, Fn&& fn) {
  const float fx = static_cast<float>(x), fy = static_cast<float>(y);
  for (int dy = -rb; dy <= rb; ++dy) {
    const int span = rb - (dy < 0 ? -dy : dy);
    const int r = ty + dy + rb - r0;
    const int k0 = s.loc[r][tx + rb - span], k1 = s.loc[r][tx + rb + span + 1];
    for (int k = k0; k < k1; ++k) {
      if constexpr (kColour) {
        const u32x4 w = s.rec[k];
        if (fabsf(fx - __uint_as_float(w[0])) + fabsf(fy - __uint_as_float(w[1])) < half)
          fn(static_cast<int32_t>(w[3]), __uint_as_float(w[2]), k);
      } else {
        const uint2 w = s.rec[k];
        if (fabsf(fx - __uint_as_float(w.x)) + fabsf(fy - __uint_as_float(w.y)) < half) fn(0, 0.0f, k);
      }
    }
  }
}

// A window frame whose reachable records outgrow the stage: halves, quarters, ...
// of the tile's pixel rows one after the other (pixel rows [r0, r0 + n) need staged
// bucket rows [r0, r0 + n + 2 rb)), body(staged, r0, mine) for each part; a single
// pixel row that still does not fit runs body with staged = false (read from
// global memory). Every thread calls it, and body runs for every thread of the
// workgroup (mine: the thread's pixel row belongs to the part); body may not use
// barriers.
template <bool kColour, typename Body>
__device__ __forceinline__ void for_frame_split(gp<const u32x4> filed, gp<const uint2> fxy, gp<const int64_t> bj,
                                                int ew, int rb, int height, const TileGeom& g, int ty,
                                                StageLds<kColour>& s, Body&& body) {
  const int prows = min(kTile, height - g.ty0);  // pixel rows of the tile inside the image
  uint32_t todo = (1u << prows) - 1u;            // pixel rows not yet done (uniform)
#pragma unroll 1
  for (int np = kTile / 2; np >= 1 && todo != 0u; np >>= 1) {
#pragma unroll 1
    for (int r0 = 0; r0 < kTile; r0 += np) {
      const uint32_t part = ((1u << np) - 1u) << r0;
      if ((todo & part) == 0u) continue;  // done, or no pixel rows
      const int r1 = min(g.nrows, r0 + np + 2 * rb);
      const bool mine = ty >= r0 && ty < r0 + np;
      if (stage_rows(filed, fxy, bj, ew, g, r0, r1, row_span(bj, ew, g, r0, r1), s)) {
        body(true, r0, mine);
        __syncthreads();
        todo &= ~part;
      } else if (np == 1) {
        body(false, r0, mine);
        todo &= ~part;
      }
    }
  }
}

// The next window frame's records, loaded into registers while the workgroup
// works on the current one, then written to the stage.
template <bool kColour>
struct Prefetch {
  using Rec = typename std::conditional<kColour, u32x4, uint2>::type;
  static constexpr int kPer = kStageCap / kThreads;
  int total;
  int64_t gb[kBoundsPerThread];
  Rec v[kPer];
  uint2 cv[kColour ? kPer : 1];
};

// Row starts of the next frame (rs: thread t's row span, t < nrows): the rows are
// held by wave 0, whose saturating prefix sum over them needs no barrier.
template <bool kColour>
__device__ __forceinline__ void plan_next(RowSpan rs, const TileGeom& g, StageLds<kColour>& s) {
  const int t = threadIdx.x;
  if (t < 64) {
    static_assert(kStageSide <= 32, "the rows fit in half a wave");
    const int c = t < g.nrows ? static_cast<int>(min(rs.e - rs.a, static_cast<int64_t>(kStageCap) + 1)) : 0;
    int incl = c;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int o = __shfl_up(incl, off, 64);
      if (t >= off) incl = min(incl + o, kStageCap + 1);
    }
    if (t < g.nrows) {
      s.first_next[t] = rs.a;
      s.base_next[t + 1] = incl;
    }
    if (t == 0) s.base_next[0] = 0;
  }
}

// Issues the loads of the next frame's bucket starts and records (after plan_next
// and a barrier); pf.total > kStageCap: nothing issued.
template <bool kColour>
__device__ __forceinline__ void issue_next(gp<const u32x4> filed, gp<const uint2> fxy, gp<const int64_t> bj, int ew,
                                           const TileGeom& g, const StageLds<kColour>& s, Prefetch<kColour>& pf) {
  const int t = threadIdx.x;
  pf.total = s.base_next[g.nrows];
  if (pf.total > kStageCap) return;  // uniform
#pragma unroll
  for (int k = 0; k < kBoundsPerThread; ++k) {
    const int i = t + k * kThreads;
    if (i < g.nrows * (g.ncols + 1)) {
      const int r = i / (g.ncols + 1), c = i - r * (g.ncols + 1);
      pf.gb[k] = bj[static_cast<int64_t>(g.ty0 + r) * ew + g.tx0 + c];
    }
  }
#pragma unroll
  for (int k = 0; k < Prefetch<kColour>::kPer; ++k) {
    const int i = t + k * kThreads;
    if (i < pf.total) {
      int lo = 0, hi = g.nrows - 1;  // row r with base[r] <= i < base[r + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.base_next[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const int64_t at = s.first_next[lo] + (i - s.base_next[lo]);
      if constexpr (kColour) {
        pf.v[k] = filed[2 * at];
        const u32x4 w = filed[2 * at + 1];
        pf.cv[k] = make_uint2(w[0], w[1]);
      } else {
        pf.v[k] = ld2(fxy + at);
      }
    }
  }
}

// Writes the prefetched frame into the stage (after a barrier past the last read
// of the current one).
template <bool kColour>
__device__ __forceinline__ void commit_next(const TileGeom& g, StageLds<kColour>& s, const Prefetch<kColour>& pf) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBoundsPerThread; ++k) {
    const int i = t + k * kThreads;
    if (i < g.nrows * (g.ncols + 1)) {
      const int r = i / (g.ncols + 1), c = i - r * (g.ncols + 1);
      s.loc[r][c] = s.base_next[r] + static_cast<int32_t>(pf.gb[k] - s.first_next[r]);
    }
  }
#pragma unroll
  for (int k = 0; k < Prefetch<kColour>::kPer; ++k)
    if (t + k * kThreads < pf.total) {
      s.rec[t + k * kThreads] = pf.v[k];
      if constexpr (kColour) s.col[t + k * kThreads] = pf.cv[k];
    }
}

// Runs body(jn, staged, r0, mine) for every window frame jn of the tile: a frame
// whose reachable records fit the stage is staged whole (body(jn, true, 0, true));
// one that does not fit goes by for_frame_split. kPrefetch: a frame's records are
// loaded into registers while the workgroup works on the frame before (the
// scatter, whose frames take long enough to hide the loads); otherwise only the
// row spans are loaded a frame ahead (the count, whose occupancy the registers
// would cost more than the loads). Every thread calls it; body may not use
// barriers.
template <bool kPrefetch, bool kColour, typename Body>
__device__ __forceinline__ void for_frames(gp<const u32x4> filed, gp<const uint2> fxy, gp<const int64_t> boff,
                                           int64_t n_buckets, int n_j, int ew, int rb, int height, const TileGeom& g,
                                           int ty, StageLds<kColour>& s, Body&& body) {
  if constexpr (!kPrefetch) {
    RowSpan next = row_span(boff, ew, g, 0, g.nrows);
#pragma unroll 1
    for (int jn = 0; jn < n_j; ++jn) {
      gp<const int64_t> bj = boff + static_cast<int64_t>(jn) * n_buckets;
      const RowSpan rs = next;
      if (jn + 1 < n_j) next = row_span(bj + n_buckets, ew, g, 0, g.nrows);
      if (stage_rows(filed, fxy, bj, ew, g, 0, g.nrows, rs, s)) {
        body(jn, true, 0, true);
        __syncthreads();
      } else {
        for_frame_split(filed, fxy, bj, ew, rb, height, g, ty, s,
                        [&](bool staged, int r0, bool mine) { body(jn, staged, r0, mine); });
      }
    }
    return;
  }
  Prefetch<kColour> pf;
  RowSpan sp = row_span(boff, ew, g, 0, g.nrows);
  plan_next(sp, g, s);
  __syncthreads();
  issue_next(filed, fxy, boff, ew, g, s, pf);
  if (n_j > 1) sp = row_span(boff + n_buckets, ew, g, 0, g.nrows);
  bool cur_ok = pf.total <= kStageCap;
  if (cur_ok) commit_next(g, s, pf);
  __syncthreads();
#pragma unroll 1
  for (int jn = 0; jn < n_j; ++jn) {
    gp<const int64_t> bj = boff + static_cast<int64_t>(jn) * n_buckets;
    const bool more = jn + 1 < n_j;
    if (more) plan_next(sp, g, s);
    __syncthreads();  // the next frame's row starts are visible
    bool next_ok = false;
    if (more) {
      issue_next(filed, fxy, bj + n_buckets, ew, g, s, pf);
      next_ok = pf.total <= kStageCap;
    }
    if (jn + 2 < n_j) sp = row_span(bj + 2 * n_buckets, ew, g, 0, g.nrows);
    if (cur_ok) {
      body(jn, true, 0, true);
    } else {
      for_frame_split(filed, fxy, bj, ew, rb, height, g, ty, s,
                      [&](bool staged, int r0, bool mine) { body(jn, staged, r0, mine); });
    }
    __syncthreads();  // every thread is done with this frame's stage
    if (next_ok) commit_next(g, s, pf);
    __syncthreads();
    cur_ok = next_ok;
  }
}

// grid: 16 x 16 tiles of the output frame
__global__ __launch_bounds__(kThreads) void k_frustum_count(const uint2* __restrict__ fxy,
                                                            const int64_t* __restrict__ boff, int width, int height,
                                                            int n_j, int rb, float half, int64_t n_buckets,
                                                            int64_t* __restrict__ counts) {
  __shared__ StageLds<false> s;
  const TileGeom g = tile_geom(width, height, rb);
  const int tx = static_cast<int>(threadIdx.x) % kTile, ty = static_cast<int>(threadIdx.x) / kTile;
  const int x = g.tx0 + tx, y = g.ty0 + ty;
  const bool in = x < width && y < height;
  const int ew = width + 2 * rb;
  int64_t n = 0;
  for_frames<false>(nullptr, to_global(fxy), to_global(boff), n_buckets, n_j, ew, rb, height, g, ty, s,
             [&](int jn, bool staged, int r0, bool mine) {
               if (!in || !mine) return;
               if (staged)
                 for_members_staged(s, r0, rb, half, tx, ty, x, y, [&](int32_t, float, int) { ++n; });
               else
                 for_members<true>(nullptr, fxy, boff, width, rb, half, n_buckets, jn, x, y,
                                   [&](int32_t, float, int64_t) { ++n; });
             });
  if (in) to_global(counts)[static_cast<int64_t>(y) * width + x] = n;
}

// Members of one (p, J) pair held per thread while they are ordered: up to
// kSortSlots keys (q << 10 | staged index, so the order of the keys is that of q) in
// registers, put in order by a sorting network.
constexpr int kSortSlots = 16;
constexpr int kIdxBits = 10;
static_assert(kStageCap <= (1 << kIdxBits) && SG_ID_SHIFT + kIdxBits <= 32, "key = q, staged index");

// Bitonic sorting network over keys k[0 .. N) (ascending; N a power of two); fully
// unrolled, so every compare-exchange is one minimum and one maximum.
template <int N>
__device__ __forceinline__ void sort_keys(uint32_t (&k)[kSortSlots]) {
  static_assert(N <= kSortSlots && (N & (N - 1)) == 0, "power of two within the slots");
#pragma unroll
  for (int size = 2; size <= N; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ stride;
        if (l > i) {
          const uint32_t a = k[i], b = k[l];
          const bool up = (i & size) == 0;
          k[i] = up ? min(a, b) : max(a, b);
          k[l] = up ? max(a, b) : min(a, b);
        }
      }
}

// Records held per lane between window frames (odd: the lanes' appends at one slot
// index fall in different LDS banks), written out as runs.
constexpr int kBufSlots = 9;
constexpr int kRunLanes = 16;  // lanes writing one run (>= kBufSlots)
static_assert(kBufSlots <= kRunLanes && (kBufSlots & 1) == 1, "a run fits its lane group; odd stride");

struct RecordBuf {
  uint32_t rec[3 * 64 * kBufSlots];  // lane l, slot i: colour + rho (2 words), id at 3 (l kBufSlots + i)
  int n[64];
  int64_t dst[64];
};

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Writes the nflush buffered records of every lane (0: the lane keeps its
// records) to [cur, cur + nflush) of its segment; every lane of the wave calls
// it. The flushing lanes' (count, destination) pairs are compacted into a list,
// and each group of kRunLanes lanes writes one list entry's run, so a store
// instruction writes 64 / kRunLanes runs instead of 64 scattered pieces.
__device__ __forceinline__ void flush_records(int nflush, int64_t& cur, int& fill, RecordBuf& b, gp<uint32_t> ids,
                                              gp<uint2> crho) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const uint64_t flushing = __ballot(nflush > 0);
  const int n_list = __popcll(flushing);
  if (nflush > 0) {
    const int rank = __popcll(flushing & ((static_cast<uint64_t>(1) << lane) - 1));
    b.n[rank] = (lane << 8) | nflush;
    b.dst[rank] = cur;
  }
  wave_fence();
  const int sub = lane % kRunLanes, grp = lane / kRunLanes;
  for (int base = 0; base < n_list; base += 64 / kRunLanes) {
    const int e = base + grp;
    if (e < n_list) {
      const int on = b.n[e];
      const int own = on >> 8, cnt = on & 0xFF;
      if (sub < cnt) {
        const int64_t dst = b.dst[e] + sub;
        const uint32_t* slot = b.rec + 3 * (own * kBufSlots + sub);
        st2(crho + dst, make_uint2(slot[0], slot[1]));
        ids[dst] = slot[2];
      }
    }
  }
  wave_fence();
  cur += nflush;
  fill -= nflush;
}

// Scatter: per output pixel and window frame, one pass over the staged buckets
// collects the members' keys and a sorting network orders them by q; the records
// (colour and carried depth from the staged records, no source plane is read) go
// to a per-lane buffer in LDS, written out in runs when a lane's buffer cannot take
// the next frame's members. A pair with more members than the buffer holds is
// written directly after the lane's buffer (by repeated minimum past kSortSlots
// members, as is every pair of a half-tile read from global memory).
__global__ __launch_bounds__(kThreads) void k_frustum_scatter(
    const uint16_t* __restrict__ depth_, const Filed* __restrict__ filed, const int64_t* __restrict__ boff,
    int width, int height, int f, int w, int jlo, int n_j, int rb, float half, int64_t n_buckets,
    const int64_t* __restrict__ offsets_, uint32_t* __restrict__ ids_, uint2* __restrict__ crho_, int64_t capacity,
    uint32_t* __restrict__ status_) {
  __shared__ StageLds<true> s;
  __shared__ RecordBuf s_buf[kThreads / 64];
  const int t = threadIdx.x, lane = t & 63;
  RecordBuf& buf = s_buf[t >> 6];
  const TileGeom g = tile_geom(width, height, rb);
  const int tx = t % kTile, ty = t / kTile;
  const int x = g.tx0 + tx, y = g.ty0 + ty;
  const int ew = width + 2 * rb;
  gp<uint32_t> status = to_global(status_);
  // a thread outside the image, or whose segment cannot be written, only joins the
  // staging and its wave's flushes (every thread reaches every barrier)
  bool live = x < width && y < height;
  const int64_t p = static_cast<int64_t>(y) * width + x;
  int64_t start = 0, end = 0;
  if (live) {
    start = to_global(offsets_)[p];
    end = to_global(offsets_)[p + 1];
    if (start < 0 || end < start) {
      flag_or(status, SG_FLAG_INCONSISTENT);
      live = false;
    } else if (end > capacity) {
      if (end > start) flag_or(status, SG_FLAG_CAPACITY);
      live = false;
    }
  }
  const float dp = live ? depth_at(to_global(depth_), width, height, f, x, y) : 0.0f;
  const bool has_ref = dp > 0.0f && dp < INFINITY;
  gp<uint32_t> ids = to_global(ids_);
  gp<uint2> crho = to_global(crho_);
  gp<const u32x4> filed4 = reinterpret_cast<gp<const u32x4>>(to_global(filed));
  int64_t cur = start;  // segment position of the buffer's first record
  int fill = 0;         // records in the buffer
  int64_t found = 0;    // members met (the count pass's total when nothing changed)
  // one record from a member's stored colour (r, g, b, depth) and carried depth z
  auto make = [&](uint32_t id, uint2 c, float z, uint32_t (&r)[3]) {
    const float rho = has_ref ? (z - dp) / dp : __builtin_nanf("");
    r[0] = c.x;
    r[1] = (c.y & 0xFFFFu) | (f2h(rho) << 16);
    r[2] = id;
  };
  // direct writes at cur (the buffer is empty), never past the segment
  auto emit = [&](uint32_t id, uint2 c, float z) {
    if (cur < end) {
      uint32_t r[3];
      make(id, c, z, r);
      st2(crho + cur, make_uint2(r[0], r[1]));
      ids[cur] = r[2];
    }
    ++cur;
  };
  auto emit_by_minimum = [&](uint32_t id_j, auto&& members, auto&& colour) {
    int32_t last = -1;
    for (;;) {  // the smallest member above the last emitted
      int32_t best = INT_MAX;
      float best_z = 0.0f;
      int64_t best_k = 0;
      members([&](int32_t q, float z, int64_t k) {
        if (q > last && q < best) {
          best = q;
          best_z = z;
          best_k = k;
        }
      });
      if (best == INT_MAX) break;
      emit(id_j | static_cast<uint32_t>(best), colour(best_k), best_z);
      last = best;
    }
  };
  for_frames<true>(filed4, nullptr, to_global(boff), n_buckets, n_j, ew, rb, height, g, ty, s,
             [&](int jn, bool staged, int r0, bool mine) {
      const uint32_t id_j = static_cast<uint32_t>(jlo + jn - f + w) << SG_ID_SHIFT;
      const bool act = live && mine;
      uint32_t keys[kSortSlots];
#pragma unroll
      for (int i = 0; i < kSortSlots; ++i) keys[i] = 0xFFFFFFFFu;
      int n = 0;
      auto members = [&](auto&& fn) { for_members_staged(s, r0, rb, half, tx, ty, x, y, fn); };
      if (act && staged)
        members([&](int32_t q, float, int k) {  // keys pushed in front (static register indices)
#pragma unroll
          for (int i = kSortSlots - 1; i > 0; --i) keys[i] = keys[i - 1];
          keys[0] = (static_cast<uint32_t>(q) << kIdxBits) | static_cast<uint32_t>(k);
          ++n;
        });
      const bool buffered = act && staged && n <= kBufSlots;
      // a lane whose buffer cannot take this frame's members writes it out first
      // (all of it when the members go out directly)
      const int nflush = act && (!buffered || fill + n > kBufSlots) ? fill : 0;
      if (__any(nflush > 0)) flush_records(nflush, cur, fill, buf, ids, crho);
      if (act && staged && n <= kSortSlots) {
        if (__any(n > kSortSlots / 2))
          sort_keys<kSortSlots>(keys);
        else
          sort_keys<kSortSlots / 2>(keys);
      }
      if (buffered) {
        found += n;
        const int64_t room = end - cur - fill;  // fewer only when the planes changed since pass 1
        uint32_t* slot = buf.rec + 3 * (lane * kBufSlots + fill);
#pragma unroll
        for (int i = 0; i < kBufSlots; ++i)
          if (i < n && i < room) {
            const uint32_t key = keys[i];
            const int k = static_cast<int>(key & ((1u << kIdxBits) - 1u));
            uint32_t r[3];
            make(id_j | (key >> kIdxBits), s.col[k], __uint_as_float(s.rec[k][2]), r);
            slot[3 * i] = r[0];
            slot[3 * i + 1] = r[1];
            slot[3 * i + 2] = r[2];
          }
        fill += static_cast<int>(min(static_cast<int64_t>(n), max(room, static_cast<int64_t>(0))));
      } else if (act && staged && n <= kSortSlots) {
        found += n;
#pragma unroll
        for (int i = 0; i < kSortSlots; ++i)
          if (i < n) {
            const uint32_t key = keys[i];
            const int k = static_cast<int>(key & ((1u << kIdxBits) - 1u));
            emit(id_j | (key >> kIdxBits), s.col[k], __uint_as_float(s.rec[k][2]));
          }
      } else if (act && staged) {
        found += n;
        emit_by_minimum(id_j, [&](auto&& fn) { members([&](int32_t q, float z, int k) { fn(q, z, k); }); },
                        [&](int64_t k) { return s.col[k]; });
      } else if (act) {
        const int64_t before = cur;
        emit_by_minimum(
            id_j,
            [&](auto&& fn) { for_members<false>(filed, nullptr, boff, width, rb, half, n_buckets, jn, x, y, fn); },
            [&](int64_t k) {
              const u32x4 c = filed4[2 * k + 1];
              return make_uint2(c[0], c[1]);
            });
        found += cur - before;
      }
    });
  const int nflush = fill;
  if (__any(nflush > 0)) flush_records(nflush, cur, fill, buf, ids, crho);
  if (live && found != end - start) flag_or(status, SG_FLAG_INCONSISTENT);
}

sg_status check_frustum(const sg_clip* clip, int32_t f, const sg_frustum_params* p) {
  sg_status s = check_clip(clip, true);
  if (s != SG_OK) return s;
  if (p == nullptr) return SG_E_INVALID;
  if (f < 0 || f >= clip->num_frames) return SG_E_INVALID;
  if (p->window < 0) return SG_E_INVALID;
  if (p->window > SG_MAX_WINDOW) return SG_E_UNSUPPORTED;
  if (!(p->l > 0.0f) || !isfinite(p->l)) return SG_E_INVALID;
  if (p->l > SG_MAX_FRUSTUM_L) return SG_E_UNSUPPORTED;
  if (!(p->near_z > 0.0f) || !isfinite(p->far_z) || !(p->far_z > p->near_z)) return SG_E_INVALID;
  return SG_OK;
}

struct FrustumCall {
  FrustumLayout l;
  float* maps;
  int2* slots;
  uint32_t* counts;
  int64_t* boff;
  Filed* filed;
  uint2* xy;
  int64_t* partial;
};

sg_status frustum_prepare(const sg_clip* clip, int32_t f, const sg_frustum_params* p, const sg_sample_sets* sets,
                          void* ws, size_t ws_bytes, bool need_arena, FrustumCall* c) {
  sg_status s = check_frustum(clip, f, p);
  if (s != SG_OK) return s;
  if (sets == nullptr || sets->offsets == nullptr || sets->status == nullptr || ws == nullptr) return SG_E_INVALID;
  if (need_arena && (sets->capacity < 0 || (sets->capacity > 0 && (sets->ids == nullptr || sets->crho == nullptr))))
    return SG_E_INVALID;
  c->l = frustum_layout(clip, f, p);
  if (ws_bytes < c->l.total) return SG_E_INVALID;
  char* base = static_cast<char*>(ws);
  c->maps = reinterpret_cast<float*>(base + c->l.maps);
  c->slots = reinterpret_cast<int2*>(base + c->l.slots);
  c->counts = reinterpret_cast<uint32_t*>(base + c->l.counts);
  c->boff = reinterpret_cast<int64_t*>(base + c->l.boff);
  c->filed = reinterpret_cast<Filed*>(base + c->l.items);
  c->xy = reinterpret_cast<uint2*>(base + c->l.xy);
  c->partial = reinterpret_cast<int64_t*>(base + c->l.partial);
  return SG_OK;
}

dim3 tile_grid(const sg_clip* clip) {
  return dim3(static_cast<unsigned>(((clip->width + kTile - 1) / kTile) * ((clip->height + kTile - 1) / kTile)));
}

unsigned zero_blocks(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return static_cast<unsigned>(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace
}  // namespace sg

using sg::hip_status;

extern "C" {

sg_status scene_frustum_workspace_size(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                                       size_t* bytes) {
  const sg_status s = sg::check_frustum(clip, f, params);
  if (s != SG_OK) return s;
  if (bytes == nullptr) return SG_E_INVALID;
  *bytes = sg::frustum_layout(clip, f, params).total;
  return SG_OK;
}

sg_status scene_frustum_count(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                              sg_sample_sets* sets, void* workspace, size_t workspace_bytes, void* stream) {
  sg::FrustumCall c{};
  sg_status s = sg::frustum_prepare(clip, f, params, sets, workspace, workspace_bytes, false, &c);
  if (s != SG_OK) return s;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const sg::FrustumLayout& l = c.l;
  const int64_t n_bk = static_cast<int64_t>(l.n_j) * l.n_buckets;
  const dim3 per_pixel(static_cast<unsigned>((l.n_pix + sg::kThreads - 1) / sg::kThreads));
  const dim3 per_pixel_frame(per_pixel.x, static_cast<unsigned>(l.n_j));
  const float half = 0.5f * params->l;
  hipLaunchKernelGGL(sg::k_zero<uint32_t>, dim3(sg::zero_blocks(n_bk)), dim3(sg::kThreads), 0, st, c.counts, n_bk);
  hipLaunchKernelGGL(sg::k_frustum_pose, dim3(1), dim3(64), 0, st, clip->cam_to_world, f, l.jlo, l.n_j, clip->fx,
                     clip->fy, clip->cx, clip->cy, c.maps, sets->status);
  hipLaunchKernelGGL(sg::k_frustum_carry, per_pixel_frame, dim3(sg::kThreads), 0, st, clip->depth, c.maps,
                     clip->width, clip->height, l.jlo, l.rb, params->near_z, params->far_z, l.n_pix, l.n_buckets,
                     c.slots, c.counts);
  {
    const int64_t nb = (n_bk + sg::kScanTile - 1) / sg::kScanTile;
    hipLaunchKernelGGL(sg::k_count_sums, dim3(static_cast<unsigned>(nb)), dim3(sg::kScanThreads), 0, st, c.counts,
                       n_bk, c.partial);
    hipLaunchKernelGGL(sg::k_count_sums_scan, dim3(1), dim3(sg::kScanThreads), 0, st, c.partial, nb);
    hipLaunchKernelGGL(sg::k_count_offsets, dim3(static_cast<unsigned>(nb)), dim3(sg::kScanThreads), 0, st,
                       c.counts, n_bk, c.partial, c.boff);
    if ((s = hip_status(hipGetLastError())) != SG_OK) return s;
  }
  hipLaunchKernelGGL(sg::k_frustum_bucket, per_pixel_frame, dim3(sg::kThreads), 0, st,
                     reinterpret_cast<const uint2*>(clip->rgbd), clip->depth, c.maps, clip->width, clip->height,
                     l.jlo, l.rb, params->near_z, params->far_z, c.slots, c.boff, l.n_pix, l.n_buckets, c.filed, c.xy);
  hipLaunchKernelGGL(sg::k_frustum_count, sg::tile_grid(clip), dim3(sg::kThreads), 0, st, c.xy, c.boff,
                     clip->width, clip->height, l.n_j, l.rb, half, l.n_buckets, sets->offsets + 1);
  return hip_status(sg::launch_scan(sets->offsets, l.n_pix, c.partial, st));
}

sg_status scene_frustum_scatter(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                                sg_sample_sets* sets, void* workspace, size_t workspace_bytes, void* stream) {
  sg::FrustumCall c{};
  const sg_status s = sg::frustum_prepare(clip, f, params, sets, workspace, workspace_bytes, true, &c);
  if (s != SG_OK) return s;
  const sg::FrustumLayout& l = c.l;
  hipLaunchKernelGGL(sg::k_frustum_scatter, sg::tile_grid(clip), dim3(sg::kThreads), 0,
                     static_cast<hipStream_t>(stream), clip->depth,
                     c.filed, c.boff, clip->width, clip->height, f, params->window, l.jlo, l.n_j, l.rb,
                     0.5f * params->l, l.n_buckets,
                     sets->offsets, sets->ids, reinterpret_cast<uint2*>(sets->crho), sets->capacity, sets->status);
  return hip_status(hipGetLastError());
}

}  // extern "C"
