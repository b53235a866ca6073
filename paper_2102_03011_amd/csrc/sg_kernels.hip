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
// Stored planes carry an apron (SG_APRON rows above and below, SG_APRON columns
// on the left, SG_APRON_RIGHT on the right) holding an invalid depth (binary16
// NaN) and zero colour, so a block around any projection that passed the bounds
// test can be read without per-pixel bounds checks: out-of-image block pixels
// read the apron and fail the depth test. The wider right apron lets each block
// row be fetched as whole 8-byte words.
//
// All kernels are compiled with -ffp-contract=off; every fused multiply-add is
// written explicitly, so pass 1 and pass 2 make bit-identical decisions.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#include "sg_device.h"
#include "sg_internal.h"

namespace sg {

// Block rows are fetched as 8-byte words (four binary16 depths) starting at the
// row's first column: kRowWords words cover the 2R + 1 columns.
template <int R>
struct RowLoad {
  static constexpr int kWords = (2 * R + 1 + 3) / 4;
};

template <int R>
__device__ __forceinline__ void load_block_depths(const uint16_t* centre, int pw,
                                                  uint32_t (&d)[2 * R + 1][2 * R + 1]) {
  constexpr int kW = RowLoad<R>::kWords;
#pragma unroll
  for (int dy = -R; dy <= R; ++dy) {
    const uint16_t* rowp = centre + dy * pw - R;
    uint64_t w[kW];
#pragma unroll
    for (int c = 0; c < kW; ++c) __builtin_memcpy(&w[c], rowp + 4 * c, 8);
#pragma unroll
    for (int o = 0; o <= 2 * R; ++o)
      d[dy + R][o] = static_cast<uint32_t>(w[o / 4] >> (16 * (o % 4))) & 0xFFFFu;
  }
}

// ---------------------------------------------------------------------------
// a1: staging. colour c (0-255) -> binary16(c / 255); depth -> binary16(depth).
// One thread per stored (padded) pixel; apron pixels get NaN depth, zero colour.

__global__ __launch_bounds__(256) void k_stage(const uint8_t* __restrict__ rgb,
                                               const float* __restrict__ depth, int n_frames,
                                               int width, int height, uint2* __restrict__ rgbd,
                                               uint16_t* __restrict__ depth16) {
  const int pw = stored_pitch(width), ph = stored_rows(height);
  const int64_t pplane = static_cast<int64_t>(pw) * ph;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= pplane * n_frames) return;
  const int64_t n = i / pplane;
  const int64_t r = i - n * pplane;
  const int py = static_cast<int>(r / pw), px = static_cast<int>(r - static_cast<int64_t>(py) * pw);
  const int x = px - SG_APRON, y = py - SG_APRON;
  if (x < 0 || x >= width || y < 0 || y >= height) {
    rgbd[i] = make_uint2(0u, kInvalidDepth16 << 16);
    depth16[i] = static_cast<uint16_t>(kInvalidDepth16);
    return;
  }
  const int64_t s = (n * height + y) * static_cast<int64_t>(width) + x;
  const float cr = static_cast<float>(rgb[3 * s + 0]) / 255.0f;   // correctly rounded division
  const float cg = static_cast<float>(rgb[3 * s + 1]) / 255.0f;
  const float cb = static_cast<float>(rgb[3 * s + 2]) / 255.0f;
  const uint32_t d = f2h(depth[s]);
  rgbd[i] = make_uint2(f2h(cr) | (f2h(cg) << 16), f2h(cb) | (d << 16));
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
// Shared projection and depth test (identical in both gather passes).

struct Projected {
  float z, inv;
  int iu, iv;
  uint32_t lo16, range16;  // accepted binary16 depth bit patterns: lo16 .. lo16 + range16
};

// Depth test |D^J(q) - z| <= tol * z, as an interval of binary16 values: with
// lo = z - tol z and hi = z + tol z (float32), a stored depth d is kept iff
// lo <= d <= hi and d is positive and finite. For positive binary16 values the
// bit pattern orders like the value, so the test becomes one unsigned compare
// (NaN, infinities, zero and negatives all fall outside).
__device__ __forceinline__ void depth_interval(float z, float tol, Projected& o) {
  const float tz = tol * z;
  const float lo = z - tz, hi = z + tz;
  uint32_t l = 1u;  // smallest positive binary16
  if (lo > 0.0f) {
    l = f2h(lo);
    if (h2f(l) < lo) ++l;  // round up
  }
  uint32_t h = f2h(hi);
  if (h2f(h) > hi) --h;    // round down (an infinite result steps back to 65504)
  if (h >= l) {
    o.lo16 = l;
    o.range16 = h - l;
  } else {
    o.lo16 = 0x10000u;     // no 16-bit pattern reaches this
    o.range16 = 0u;
  }
}

__device__ __forceinline__ bool accept16(uint32_t d16, const Projected& p) {
  return d16 - p.lo16 <= p.range16;
}

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
  const float uh = floorf(fmaf(y0, inv, 0.5f));
  const float vh = floorf(fmaf(y1, inv, 0.5f));
  const float fr = static_cast<float>(r);
  if (!(uh >= -fr && uh <= static_cast<float>(width - 1) + fr && vh >= -fr &&
        vh <= static_cast<float>(height - 1) + fr))
    return false;
  o.z = z;
  o.inv = inv;
  o.iu = static_cast<int>(uh);
  o.iv = static_cast<int>(vh);
  depth_interval(z, tol, o);
  return true;
}

// Tile of a gather workgroup: 1-D dispatch index -> (tile x, tile y, output frame),
// x fastest. Consecutive workgroups are dispatched round-robin over the XCDs, so
// at any moment every XCD works on the same band of rows and the shared memory-side
// cache serves the source lines all of them miss in their own L2.
struct Tile {
  int tx, ty, fo;
};

__device__ __forceinline__ Tile tile_of_block(int tiles_x, int tiles_y) {
  const int b = static_cast<int>(blockIdx.x);
  Tile t;
  t.tx = b % tiles_x;
  const int rest = b / tiles_x;
  t.ty = rest % tiles_y;
  t.fo = rest / tiles_y;
  return t;
}

// ---------------------------------------------------------------------------
// a3: gather pass 1 -- count members per output pixel.
// Block = 64 x 4 pixels (one wave per row segment), grid.z = output frame.
// Per source frame the (2r+1)^2 depths are loaded unconditionally (apron makes
// every address valid), so all loads of a block are in flight together.

template <int R>
__global__ __launch_bounds__(256) void k_count(const uint16_t* __restrict__ depth,
                                               const float* __restrict__ rel, int width, int height,
                                               int n_frames, int f0, int w, float tol, float z_near,
                                               int64_t* __restrict__ counts) {
  const Tile tile = tile_of_block((width + kTileW - 1) / kTileW, (height + kTileH - 1) / kTileH);
  const int x = tile.tx * kTileW + threadIdx.x;
  const int y = tile.ty * kTileH + threadIdx.y;
  const int fo = tile.fo;
  if (x >= width || y >= height) return;
  const int f = f0 + fo;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const float dp = h2f(depth[static_cast<size_t>(f) * pplane + padded_index(x, y, pw)]);
  int count = 0;
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
    for (int j = jlo; j <= jhi; ++j) {
      Projected p;
      if (!project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p))
        continue;
      uint32_t d[2 * R + 1][2 * R + 1];
      load_block_depths<R>(depth + static_cast<size_t>(j) * pplane + padded_index(p.iu, p.iv, pw), pw, d);
#pragma unroll
      for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
        for (int dx = 0; dx <= 2 * R; ++dx) count += accept16(d[dy][dx], p) ? 1 : 0;
    }
  }
  counts[static_cast<size_t>(fo) * width * height + static_cast<size_t>(y) * width + x] = count;
}

// ---------------------------------------------------------------------------
// a5: gather pass 2 -- write records in canonical order.
//
// Each wave owns 64 consecutive output pixels of one row, so their CSR segments
// are adjacent in memory. Per source frame each lane reads its whole block of
// stored (r, g, b, depth) pixels in one round trip, decides membership from the
// depth channel exactly as pass 1 does from the depth plane (same binary16 bits,
// same test), and appends its accepted records to a per-lane buffer in LDS
// (kSlots entries, odd stride: conflict-free appends). When some lane's buffer
// could overflow on the next source frame, the wave flushes every lane holding at
// least kMinRun records: a group of kRunLanes lanes writes each flushed lane's
// run, so a store instruction writes 64 / kRunLanes contiguous runs instead of 64
// scattered 8-byte pieces. Records reach global memory in the order they are
// found, which is the canonical order.

template <int R>
struct ScatterShape {
  static constexpr int kCand = (2 * R + 1) * (2 * R + 1);
  // Odd number of slots per lane (LDS: 12 B per slot, 256 lanes per workgroup).
  // A flush is triggered when some lane has fewer than kCand free slots and empties
  // every lane holding >= kMinRun records, so afterwards each lane has room for a
  // whole block again: kMinRun - 1 <= kSlots - kCand.
  static constexpr int kSlots = R == 3 ? 51 : (R == 2 ? 41 : 15);
  static constexpr int kMinRun = R == 3 ? 2 : (R == 2 ? 12 : 7);
  static constexpr int kRunLanes = kSlots <= 16 ? 16 : 64;  // lanes writing one run
  static_assert(kMinRun - 1 <= kSlots - kCand, "flush must leave room for one block");
  static_assert((kSlots & 1) == 1, "odd stride keeps LDS accesses conflict-free");
  static_assert(kSlots <= kRunLanes, "a run fits its lane group");
  using Mask = typename std::conditional<(kCand > 32), uint64_t, uint32_t>::type;
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Write the n buffered records of every lane (n = 0 for lanes that keep theirs)
// to [cur, cur + n) of that lane's segment. Only lanes with n > 0 take part: their
// (count, destination) pairs are compacted into a list (ballot + rank), and each
// group of kRunLanes lanes writes one list entry's run, so the store instructions
// stay dense however few lanes flush.
template <int R>
__device__ __forceinline__ void flush_runs(int n, int64_t& cur, int& fill, const uint2* s_rec,
                                           const uint32_t* s_id, int* s_n, int64_t* s_dst,
                                           uint32_t* __restrict__ ids, uint2* __restrict__ crho) {
  constexpr int kSlots = ScatterShape<R>::kSlots;
  constexpr int kRun = ScatterShape<R>::kRunLanes;
  constexpr int kPer = 64 / kRun;
  const int lane = threadIdx.x;
  const uint64_t flushing = __ballot(n > 0);
  const int n_list = __popcll(flushing);
  if (n > 0) {
    const int rank = __popcll(flushing & ((static_cast<uint64_t>(1) << lane) - 1));
    s_n[rank] = (lane << 8) | n;  // owner lane, count (count <= kSlots < 256)
    s_dst[rank] = cur;
  }
  wave_lds_fence();
  const int sub = lane % kRun, grp = lane / kRun;
  for (int base = 0; base < n_list; base += kPer) {
    const int e = base + grp;
    if (e < n_list) {
      const int on = s_n[e];
      const int own = on >> 8, cnt = on & 0xFF;
      if (sub < cnt) {
        const int64_t dst = s_dst[e] + sub;
        crho[dst] = s_rec[own * kSlots + sub];
        ids[dst] = s_id[own * kSlots + sub];
      }
    }
  }
  wave_lds_fence();
  cur += n;
  fill -= n;
}

template <int R>
__global__ __launch_bounds__(256) void k_scatter(const uint2* __restrict__ rgbd,
                                                 const uint16_t* __restrict__ depth,
                                                 const float* __restrict__ rel, int width,
                                                 int height, int n_frames, int f0, int w, float tol,
                                                 float z_near, const int64_t* __restrict__ offsets,
                                                 uint32_t* __restrict__ ids,
                                                 uint2* __restrict__ crho, int64_t capacity,
                                                 uint32_t* __restrict__ status) {
  using Shape = ScatterShape<R>;
  using Mask = typename Shape::Mask;
  constexpr int kSlots = Shape::kSlots;
  constexpr int kSide = 2 * R + 1;
  __shared__ uint2 s_rec_all[kTileH][kTileW * kSlots];
  __shared__ uint32_t s_id_all[kTileH][kTileW * kSlots];
  __shared__ int s_n_all[kTileH][kTileW];
  __shared__ int64_t s_dst_all[kTileH][kTileW];
  const int lane = threadIdx.x, wv = threadIdx.y;
  uint2* s_rec = s_rec_all[wv];
  uint32_t* s_id = s_id_all[wv];
  int* s_n = s_n_all[wv];
  int64_t* s_dst = s_dst_all[wv];

  const Tile tile = tile_of_block((width + kTileW - 1) / kTileW, (height + kTileH - 1) / kTileH);
  const int x = tile.tx * kTileW + lane;
  const int y = tile.ty * kTileH + wv;
  const int fo = tile.fo;
  const int f = f0 + fo;
  const bool in = x < width && y < height;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  int64_t cur = 0, end = 0, start = 0;
  bool active = false;
  float dp = 0.0f;
  if (in) {
    const size_t pix = static_cast<size_t>(fo) * width * height + static_cast<size_t>(y) * width + x;
    start = cur = offsets[pix];
    end = offsets[pix + 1];
    if (cur < 0 || end < cur) {  // offsets not produced by the count pass
      atomicOr(status, SG_FLAG_INCONSISTENT);
    } else if (end > capacity) {
      if (end > cur) atomicOr(status, SG_FLAG_CAPACITY);
    } else {
      dp = h2f(depth[static_cast<size_t>(f) * pplane + padded_index(x, y, pw)]);
      active = dp > z_near && dp < INFINITY;
    }
  }
  int fill = 0;
  int found = 0;
  const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
  const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
  const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
  uint2* my_rec = s_rec + lane * kSlots;
  uint32_t* my_id = s_id + lane * kSlots;
  for (int j = jlo; j <= jhi; ++j) {
    Projected p;
    if (active && project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p)) {
      const uint2* cj = rgbd + static_cast<size_t>(j) * pplane + padded_index(p.iu, p.iv, pw);
      uint2 px[kSide][kSide];
#pragma unroll
      for (int dy = 0; dy < kSide; ++dy)
#pragma unroll
        for (int dx = 0; dx < kSide; ++dx) px[dy][dx] = cj[(dy - R) * pw + (dx - R)];
      Mask mask = 0;
#pragma unroll
      for (int k = 0; k < kSide * kSide; ++k)
        mask |= static_cast<Mask>(accept16(px[k / kSide][k % kSide].y >> 16, p) ? 1 : 0) << k;
      const int n = __popc(static_cast<uint32_t>(mask)) +
                    (sizeof(Mask) > 4 ? __popc(static_cast<uint32_t>(static_cast<uint64_t>(mask) >> 32)) : 0);
      found += n;
      // keep only as many records as the segment has room for (fewer only when
      // the planes changed since the count pass; flagged at the end)
      int kept = n;
      const int64_t room = end - cur - fill;
      if (n > room) {
        Mask keep = 0;
        int left = static_cast<int>(room);
        for (int k = 0; k < kSide * kSide && left > 0; ++k)
          if ((mask >> k) & 1) {
            keep |= static_cast<Mask>(1) << k;
            --left;
          }
        mask = keep;
        kept = static_cast<int>(room);
      }
      // id = ((J - f + w) << 22) | q; q < 2^22, so the OR is an add of a
      // per-(p, J) base and a per-candidate constant
      const uint32_t id0 = (static_cast<uint32_t>(j - f + w) << SG_ID_SHIFT) +
                           static_cast<uint32_t>((p.iv - R) * width + (p.iu - R));
      uint2* rec = my_rec + fill;
      uint32_t* idp = my_id + fill;
#pragma unroll
      for (int k = 0; k < kSide * kSide; ++k) {
        if ((mask >> k) & 1) {
          const int dy = k / kSide, dx = k % kSide;
          const uint2 v = px[dy][dx];
          // rho = (d - z) / z = d * (1 / z) - 1, d = the record's own stored depth
          const float rho = fmaf(h2f(v.y >> 16), p.inv, -1.0f);
          *rec++ = make_uint2(v.x, (v.y & 0xFFFFu) | (f2h(rho) << 16));
          *idp++ = id0 + static_cast<uint32_t>(dy * width + dx);
        }
      }
      fill += kept;
    }
    if (__any(fill > kSlots - Shape::kCand))
      flush_runs<R>(fill >= Shape::kMinRun ? fill : 0, cur, fill, s_rec, s_id, s_n, s_dst, ids, crho);
  }
  if (__any(fill > 0)) flush_runs<R>(fill, cur, fill, s_rec, s_id, s_n, s_dst, ids, crho);
  if (active && found != end - start) atomicOr(status, SG_FLAG_INCONSISTENT);
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
    const int64_t self = pix - static_cast<int64_t>(fo) * plane;
    const int y = static_cast<int>(self / width), x = static_cast<int>(self - static_cast<int64_t>(y) * width);
    const int pw = stored_pitch(width);
    const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
    const uint2 ref = rgbd[static_cast<size_t>(f0 + fo) * pplane + padded_index(x, y, pw)];
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

hipError_t launch_stage(const uint8_t* rgb, const float* depth, int n_frames, int width, int height,
                        uint16_t* rgbd, uint16_t* depth16, hipStream_t st) {
  const int64_t n = static_cast<int64_t>(stored_pitch(width)) * stored_rows(height) * n_frames;
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_stage, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, rgb, depth,
                     n_frames, width, height, reinterpret_cast<uint2*>(rgbd), depth16);
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
                     reinterpret_cast<const uint2*>(jb.rgbd), jb.depth, jb.rel, jb.width, jb.height,
                     jb.n_frames, jb.f0, jb.w, jb.tol, jb.z_near, jb.offsets, jb.ids,
                     reinterpret_cast<uint2*>(jb.crho), jb.capacity, jb.status);
}

static dim3 gather_grid(const GatherJob& jb) {
  const int64_t nb = static_cast<int64_t>((jb.width + kTileW - 1) / kTileW) *
                     ((jb.height + kTileH - 1) / kTileH) * jb.n_out;
  return dim3(static_cast<unsigned>(nb));
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
#define SG_FILTER_LAUNCH(C, T)                                                                  \
  hipLaunchKernelGGL((k_filter<C, T>), g, dim3(256), 0, st, rgbd, fj.width, fj.height, fj.f0, \
                     fj.w, fj.n_pix, fj.offsets, fj.ids, crho, fj.capacity, fj.a_d, fj.a_c,    \
                     fj.a_t, fj.out)
  if (fj.use_colour && fj.use_time)
    SG_FILTER_LAUNCH(true, true);
  else if (fj.use_colour)
    SG_FILTER_LAUNCH(true, false);
  else if (fj.use_time)
    SG_FILTER_LAUNCH(false, true);
  else
    SG_FILTER_LAUNCH(false, false);
#undef SG_FILTER_LAUNCH
  return hipGetLastError();
}

}  // namespace sg
