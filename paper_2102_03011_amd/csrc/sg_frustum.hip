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

int bucket_radius(float l) { return static_cast<int>(ceilf(0.5f * l + 1.0f)) - 1; }

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

struct FrustumLayout {
  int jlo, n_j, rb;
  int64_t n_pix, n_buckets;  // per window frame
  size_t maps, slots, boff, items, partial, total;
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
  l.boff = at;
  at += align_up((static_cast<size_t>(l.n_j) * l.n_buckets + 1) * sizeof(int64_t));
  l.items = at;
  at += align_up(static_cast<size_t>(l.n_j) * l.n_pix * sizeof(Filed));
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
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const float d = h2f(depth[static_cast<size_t>(jn_plane_frame) * pplane + padded_index(x, y, pw)]);
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
                                                            unsigned long long* __restrict__ bcount) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (q >= n_pix) return;
  const int jn = blockIdx.y;
  const int y = static_cast<int>(q / width), x = static_cast<int>(q - static_cast<int64_t>(y) * width);
  float px, py, z;
  const int b = carry_point(to_global(depth), to_global(maps) + jn * kMapFloats, width, height, jlo + jn, x, y, rb,
                            near_z, far_z, px, py, z);
  int slot = 0;
  if (b >= 0)
    slot = static_cast<int>(atomicAdd(bcount + 1 + static_cast<int64_t>(jn) * n_buckets + b, 1ull));
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
                                                             int64_t n_buckets, Filed* __restrict__ filed) {
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
}

// Calls fn(q, z', k) for every q filed (at index k) within L1 distance rb of output
// pixel (x, y) in window frame jn and passing Eq. 2.
template <typename Fn>
__device__ __forceinline__ void for_members(const Filed* __restrict__ filed_, const int64_t* __restrict__ boff,
                                            int width, int rb, float half, int64_t n_buckets, int jn, int x, int y,
                                            Fn&& fn) {
  gp<const u32x4> filed = reinterpret_cast<gp<const u32x4>>(to_global(filed_));
  gp<const int64_t> bj = to_global(boff) + static_cast<int64_t>(jn) * n_buckets;
  const int ew = width + 2 * rb;
  const float fx = static_cast<float>(x), fy = static_cast<float>(y);
  for (int dy = -rb; dy <= rb; ++dy) {
    const int span = rb - (dy < 0 ? -dy : dy);
    const int64_t row = static_cast<int64_t>(y + dy + rb) * ew + (x + rb);
    // the buckets of this row are adjacent: one contiguous range of filed records
    const int64_t k0 = bj[row - span], k1 = bj[row + span + 1];
    for (int64_t k = k0; k < k1; ++k) {
      const u32x4 w = filed[2 * k];
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
constexpr int kStageCap = 1024;
constexpr int kBoundsPerThread = (kStageSide * (kStageSide + 1) + kThreads - 1) / kThreads;
static_assert(kThreads == kTile * kTile, "one thread per pixel of a tile");

// records staged per window frame (kColour: with their colours, for the scatter)
template <bool kColour>
struct StageLds {
  u32x4 rec[kStageCap];                     // x, y, z', q of the staged rows, row after row
  uint2 col[kColour ? kStageCap : 1];       // their r, g, b, depth
  int32_t loc[kStageSide][kStageSide + 1];  // rec index of bucket (row, column); [r][ncols] = row end
  int32_t base[kStageSide + 1];             // rec index of each row's first record; [nrows] = total
  int64_t first[kStageSide];                // filed index of each row's first record
};

struct TileGeom {
  int tx0, ty0;       // first output pixel of the tile = first staged bucket (extended grid)
  int nrows, ncols;   // staged bucket rows and columns that exist in the extended grid
};

__device__ __forceinline__ TileGeom tile_geom(int width, int height, int rb) {
  const int tiles_x = (width + kTile - 1) / kTile;
  TileGeom g;
  g.tx0 = (static_cast<int>(blockIdx.x) % tiles_x) * kTile;
  g.ty0 = (static_cast<int>(blockIdx.x) / tiles_x) * kTile;
  g.nrows = min(kTile + 2 * rb, height + 2 * rb - g.ty0);
  g.ncols = min(kTile + 2 * rb, width + 2 * rb - g.tx0);
  return g;
}

// The first and end filed index of staged row t (threads t < nrows) of a window
// frame: loaded one frame ahead, while the workgroup works on the frame before.
struct RowSpan {
  int64_t a, e;
};
__device__ __forceinline__ RowSpan row_span(gp<const int64_t> bj, int ew, const TileGeom& g) {
  const int t = threadIdx.x;
  RowSpan r{0, 0};
  if (t < g.nrows) {
    const int64_t row = static_cast<int64_t>(g.ty0 + t) * ew + g.tx0;
    r.a = bj[row];
    r.e = bj[row + g.ncols];
  }
  return r;
}

// Stages window frame jn's reachable records (rs: this thread's row_span of jn);
// false (nothing staged) when they number more than kStageCap. Every thread of the
// workgroup calls it; it ends on a barrier either way, and the caller puts one
// between its last read of the staged records and the next call.
template <bool kColour>
__device__ bool stage_frame(gp<const u32x4> filed, gp<const int64_t> bj, int ew, const TileGeom& g, RowSpan rs,
                            StageLds<kColour>& s) {
  const int t = threadIdx.x;
  if (t < g.nrows) {
    s.first[t] = rs.a;
    s.base[t + 1] = static_cast<int32_t>(min(rs.e - rs.a, static_cast<int64_t>(kStageCap) + 1));
  }
  __syncthreads();
  if (t == 0) {  // row starts (at most kStageSide rows; clamped counts cannot overflow)
    int acc = 0;
    s.base[0] = 0;
    for (int r = 0; r < g.nrows; ++r) {
      acc = min(acc + s.base[r + 1], kStageCap + 1);
      s.base[r + 1] = acc;
    }
  }
  __syncthreads();
  const int total = s.base[g.nrows];
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
    ib[k] = i < g.nrows * (g.ncols + 1) ? i : -1;
    if (ib[k] >= 0) {
      const int r = i / (g.ncols + 1), c = i - r * (g.ncols + 1);
      gb[k] = bj[static_cast<int64_t>(g.ty0 + r) * ew + g.tx0 + c];
    }
  }
  constexpr int kRecPerThread = kStageCap / kThreads;
  static_assert(kRecPerThread * kThreads == kStageCap, "whole records per thread");
  u32x4 v[kRecPerThread];
  uint2 cv[kRecPerThread];
#pragma unroll
  for (int k = 0; k < kRecPerThread; ++k) {
    const int i = t + k * kThreads;
    if (i < total) {
      int lo = 0, hi = g.nrows - 1;  // row r with base[r] <= i < base[r + 1]
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.base[mid] <= i) lo = mid; else hi = mid - 1;
      }
      const int64_t at = s.first[lo] + (i - s.base[lo]);
      v[k] = filed[2 * at];
      if (kColour) {
        const u32x4 w = filed[2 * at + 1];
        cv[k] = make_uint2(w[0], w[1]);
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
      if (kColour) s.col[t + k * kThreads] = cv[k];
    }
  __syncthreads();
  return true;
}

// for_members over the staged records: fn(q, z', staged index) (thread's pixel
// (x, y) = (tx0 + tx, ty0 + ty)).
template <bool kColour, typename Fn>
__device__ __forceinline__ void for_members_staged(const StageLds<kColour>& s, int rb, float half, int tx, int ty,
                                                   int x, int y, Fn&& fn) {
  const float fx = static_cast<float>(x), fy = static_cast<float>(y);
  for (int dy = -rb; dy <= rb; ++dy) {
    const int span = rb - (dy < 0 ? -dy : dy);
    const int r = ty + dy + rb;
    const int k0 = s.loc[r][tx + rb - span], k1 = s.loc[r][tx + rb + span + 1];
    for (int k = k0; k < k1; ++k) {
      const u32x4 w = s.rec[k];
      if (fabsf(fx - __uint_as_float(w[0])) + fabsf(fy - __uint_as_float(w[1])) < half)
        fn(static_cast<int32_t>(w[3]), __uint_as_float(w[2]), k);
    }
  }
}

// grid: 16 x 16 tiles of the output frame
__global__ __launch_bounds__(kThreads) void k_frustum_count(const Filed* __restrict__ filed,
                                                            const int64_t* __restrict__ boff, int width, int height,
                                                            int n_j, int rb, float half, int64_t n_buckets,
                                                            int64_t* __restrict__ counts) {
  __shared__ StageLds<false> s;
  const TileGeom g = tile_geom(width, height, rb);
  const int tx = static_cast<int>(threadIdx.x) % kTile, ty = static_cast<int>(threadIdx.x) / kTile;
  const int x = g.tx0 + tx, y = g.ty0 + ty;
  const bool in = x < width && y < height;
  const int ew = width + 2 * rb;
  gp<const u32x4> filed4 = reinterpret_cast<gp<const u32x4>>(to_global(filed));
  int64_t n = 0;
  RowSpan next = row_span(to_global(boff), ew, g);
  for (int jn = 0; jn < n_j; ++jn) {
    gp<const int64_t> bj = to_global(boff) + static_cast<int64_t>(jn) * n_buckets;
    const RowSpan rs = next;
    if (jn + 1 < n_j) next = row_span(bj + n_buckets, ew, g);
    if (stage_frame(filed4, bj, ew, g, rs, s)) {
      if (in) for_members_staged(s, rb, half, tx, ty, x, y, [&](int32_t, float, int) { ++n; });
      __syncthreads();
    } else if (in) {
      for_members(filed, boff, width, rb, half, n_buckets, jn, x, y, [&](int32_t, float, int64_t) { ++n; });
    }
  }
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

// Scatter: per output pixel and window frame, one pass over the staged buckets
// collects the members' keys, a sorting network orders them by q, and they are
// written in canonical order from the staged records (no source plane is read). A
// pair with more than kSortSlots members (dense occluders), and every pair of a
// frame read from global memory, is emitted by repeated minimum instead, one pass
// over the buckets per member.
__global__ __launch_bounds__(kThreads) void k_frustum_scatter(
    const uint16_t* __restrict__ depth_, const Filed* __restrict__ filed, const int64_t* __restrict__ boff,
    int width, int height, int f, int w, int jlo, int n_j, int rb, float half, int64_t n_buckets,
    const int64_t* __restrict__ offsets_, uint32_t* __restrict__ ids_, uint2* __restrict__ crho_, int64_t capacity,
    uint32_t* __restrict__ status_) {
  __shared__ StageLds<true> s;
  const int t = threadIdx.x;
  const TileGeom g = tile_geom(width, height, rb);
  const int tx = t % kTile, ty = t / kTile;
  const int x = g.tx0 + tx, y = g.ty0 + ty;
  const int ew = width + 2 * rb;
  gp<uint32_t> status = to_global(status_);
  // a thread outside the image, or whose segment cannot be written, only joins the
  // staging (every thread reaches every barrier)
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
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const float dp = live ? h2f(to_global(depth_)[static_cast<size_t>(f) * pplane + padded_index(x, y, pw)]) : 0.0f;
  const bool has_ref = dp > 0.0f && dp < INFINITY;
  gp<uint32_t> ids = to_global(ids_);
  gp<uint2> crho = to_global(crho_);
  gp<const u32x4> filed4 = reinterpret_cast<gp<const u32x4>>(to_global(filed));
  int64_t cur = start;
  // one record from a member's stored colour (r, g, b, depth) and carried depth z
  auto make = [&](uint32_t id, uint2 c, float z, uint32_t (&r)[3]) {
    const float rho = has_ref ? (z - dp) / dp : __builtin_nanf("");
    r[0] = c.x;
    r[1] = (c.y & 0xFFFFu) | (f2h(rho) << 16);
    r[2] = id;
  };
  auto emit = [&](uint32_t id, uint2 c, float z) {
    if (cur < end) {  // a count that changed since pass 1 never writes past the segment
      uint32_t r[3];
      make(id, c, z, r);
      st2(crho + cur, make_uint2(r[0], r[1]));
      ids[cur] = r[2];
    }
    ++cur;
  };
  // the sorted keys key[0 .. n), four at a time: a whole group goes out as two
  // 16-byte colour stores and one 16-byte id store (a segment position is 8-byte
  // aligned in crho, 4-byte in ids)
  auto emit_sorted = [&](uint32_t id_j, const uint32_t (&keys)[kSortSlots], int n) {
#pragma unroll
    for (int a0 = 0; a0 < kSortSlots; a0 += 4) {
      if (a0 >= n) break;
      const int c = min(4, n - a0);
      uint32_t r[4][3];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < c) {
          const uint32_t key = keys[a0 + i];
          const int k = static_cast<int>(key & ((1u << kIdxBits) - 1u));
          make(id_j | (key >> kIdxBits), s.col[k], __uint_as_float(s.rec[k][2]), r[i]);
        }
      const int64_t room = end - cur;
      if (c == 4 && room >= 4) {
        gp<u32x4a8> cr = reinterpret_cast<gp<u32x4a8>>(crho + cur);
        cr[0] = u32x4a8{r[0][0], r[0][1], r[1][0], r[1][1]};
        cr[1] = u32x4a8{r[2][0], r[2][1], r[3][0], r[3][1]};
        *reinterpret_cast<gp<u32x4a4>>(ids + cur) = u32x4a4{r[0][2], r[1][2], r[2][2], r[3][2]};
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i < c && i < room) {
            st2(crho + cur + i, make_uint2(r[i][0], r[i][1]));
            ids[cur + i] = r[i][2];
          }
      }
      cur += c;
    }
  };
  // repeated minimum over one pair's members; colour(k) gives a member's stored colour
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
  RowSpan next = row_span(to_global(boff), ew, g);
  for (int jn = 0; jn < n_j; ++jn) {
    const uint32_t id_j = static_cast<uint32_t>(jlo + jn - f + w) << SG_ID_SHIFT;
    gp<const int64_t> bj = to_global(boff) + static_cast<int64_t>(jn) * n_buckets;
    const RowSpan rs = next;
    if (jn + 1 < n_j) next = row_span(bj + n_buckets, ew, g);
    if (stage_frame(filed4, bj, ew, g, rs, s)) {
      if (live) {
        auto members = [&](auto&& fn) { for_members_staged(s, rb, half, tx, ty, x, y, fn); };
        // keys pushed in front (static register indices); UINT32_MAX pads the rest
        uint32_t keys[kSortSlots];
#pragma unroll
        for (int i = 0; i < kSortSlots; ++i) keys[i] = 0xFFFFFFFFu;
        int n = 0;
        members([&](int32_t q, float, int k) {
#pragma unroll
          for (int i = kSortSlots - 1; i > 0; --i) keys[i] = keys[i - 1];
          keys[0] = (static_cast<uint32_t>(q) << kIdxBits) | static_cast<uint32_t>(k);
          ++n;
        });
        if (n <= kSortSlots) {
          if (__any(n > kSortSlots / 2))
            sort_keys<kSortSlots>(keys);
          else
            sort_keys<kSortSlots / 2>(keys);
          emit_sorted(id_j, keys, n);
        } else {
          emit_by_minimum(id_j, [&](auto&& fn) { members([&](int32_t q, float z, int k) { fn(q, z, k); }); },
                          [&](int64_t k) { return s.col[k]; });
        }
      }
      __syncthreads();
    } else if (live) {
      emit_by_minimum(
          id_j, [&](auto&& fn) { for_members(filed, boff, width, rb, half, n_buckets, jn, x, y, fn); },
          [&](int64_t k) {
            const u32x4 c = filed4[2 * k + 1];
            return make_uint2(c[0], c[1]);
          });
    }
  }
  if (live && cur != end) flag_or(status, SG_FLAG_INCONSISTENT);
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
  int64_t* boff;
  Filed* filed;
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
  c->boff = reinterpret_cast<int64_t*>(base + c->l.boff);
  c->filed = reinterpret_cast<Filed*>(base + c->l.items);
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
  hipLaunchKernelGGL(sg::k_zero<int64_t>, dim3(sg::zero_blocks(n_bk + 1)), dim3(sg::kThreads), 0, st, c.boff,
                     n_bk + 1);
  hipLaunchKernelGGL(sg::k_frustum_pose, dim3(1), dim3(64), 0, st, clip->cam_to_world, f, l.jlo, l.n_j, clip->fx,
                     clip->fy, clip->cx, clip->cy, c.maps, sets->status);
  hipLaunchKernelGGL(sg::k_frustum_carry, per_pixel_frame, dim3(sg::kThreads), 0, st, clip->depth, c.maps,
                     clip->width, clip->height, l.jlo, l.rb, params->near_z, params->far_z, l.n_pix, l.n_buckets,
                     c.slots, reinterpret_cast<unsigned long long*>(c.boff));
  if ((s = hip_status(sg::launch_scan(c.boff, n_bk, c.partial, st))) != SG_OK) return s;
  hipLaunchKernelGGL(sg::k_frustum_bucket, per_pixel_frame, dim3(sg::kThreads), 0, st,
                     reinterpret_cast<const uint2*>(clip->rgbd), clip->depth, c.maps, clip->width, clip->height,
                     l.jlo, l.rb, params->near_z, params->far_z, c.slots, c.boff, l.n_pix, l.n_buckets, c.filed);
  hipLaunchKernelGGL(sg::k_frustum_count, sg::tile_grid(clip), dim3(sg::kThreads), 0, st, c.filed, c.boff,
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
