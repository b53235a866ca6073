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
// read the apron and fail the depth test. The depth plane pairs stored rows (one
// 32-bit word per column holds two rows), so the count pass reads a 3 x 3 block
// of depths with two row loads.
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

// ---------------------------------------------------------------------------
// a1: staging. colour c (0-255) -> binary16(c / 255); depth -> binary16(depth).
// One thread per stored (padded) pixel; apron pixels get NaN depth, zero colour.
// The depth goes to its row-paired entry; with an odd number of stored rows the
// threads of the last row also fill the unused high half of the last pair.

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
  uint16_t* dn = depth16 + static_cast<size_t>(n) * depth_plane_elems(width, height);
  const uint32_t di = depth_index(x, y, pw);
  if ((ph & 1) && py == ph - 1) dn[di + 1] = static_cast<uint16_t>(kInvalidDepth16);
  if (x < 0 || x >= width || y < 0 || y >= height) {
    rgbd[i] = make_uint2(0u, kInvalidDepth16 << 16);
    dn[di] = static_cast<uint16_t>(kInvalidDepth16);
    return;
  }
  const int64_t s = (n * height + y) * static_cast<int64_t>(width) + x;
  const float cr = static_cast<float>(rgb[3 * s + 0]) / 255.0f;   // correctly rounded division
  const float cg = static_cast<float>(rgb[3 * s + 1]) / 255.0f;
  const float cb = static_cast<float>(rgb[3 * s + 2]) / 255.0f;
  const uint32_t d = f2h(depth[s]);
  rgbd[i] = make_uint2(f2h(cr) | (f2h(cg) << 16), f2h(cb) | (d << 16));
  dn[di] = static_cast<uint16_t>(d);
}

// ---------------------------------------------------------------------------
// a2: relative camera maps, float64 -> float32.
// One thread per (output frame fo, window slot s): J = f - w + s.
// Record layout (kRelStride floats): M row-major (9), k (3), unused (4).

__device__ __forceinline__ void pose_prep_one(gp<const double> c2w, int n_frames, int f0, int w,
                                              double fx, double fy, double cx, double cy, gp<float> rel,
                                              int i) {
  const int slots = 2 * w + 1;
  const int fo = i / slots, s = i - fo * slots;
  const int f = f0 + fo, j = f - w + s;
  gp<float> out = rel + static_cast<size_t>(i) * kRelStride;
  double m[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double kt[3] = {0, 0, 0};
  if (j < 0 || j >= n_frames) {
    for (int e = 0; e < kRelStride; ++e) out[e] = 0.0f;
    return;
  }
  if (j != f) {
    gp<const double> a = c2w + static_cast<size_t>(f) * 16;   // C^f
    gp<const double> b = c2w + static_cast<size_t>(j) * 16;   // C^J
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

__global__ __launch_bounds__(64) void k_pose_prep(const double* __restrict__ c2w, int n_frames,
                                                  int f0, int n_out, int w, double fx, double fy,
                                                  double cx, double cy, float* __restrict__ rel,
                                                  uint32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && status != nullptr) *status = 0u;
  if (i >= n_out * (2 * w + 1)) return;
  pose_prep_one(to_global(c2w), n_frames, f0, w, fx, fy, cx, cy, to_global(rel), i);
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

__device__ __forceinline__ bool project(gp<const float> m, float x, float y, float dp,
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

// Frame j's depth plane as pair words (dplane binary16 entries per frame, an even
// number, so every plane starts 4-byte aligned when the first one does).
__device__ __forceinline__ gp<const uint32_t> depth_words(gp<const uint16_t> depth, int j, size_t dplane) {
  return reinterpret_cast<gp<const uint32_t>>(depth + static_cast<size_t>(j) * dplane);
}

// Members of output pixel (x, y) of output frame f; relf = the relative maps of f.
template <int R>
__device__ __forceinline__ int count_pixel(gp<const uint16_t> depth, gp<const float> relf,
                                           int width, int height, int n_frames, int f, int w, float tol,
                                           float z_near, int x, int y) {
  const int pw = stored_pitch(width);
  const size_t dplane = depth_plane_elems(width, height);
  const float dp = h2f(depth[static_cast<size_t>(f) * dplane + depth_index(x, y, pw)]);
  int count = 0;
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    for (int j = jlo; j <= jhi; ++j) {
      Projected p;
      if (!project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p))
        continue;
      uint32_t d[2 * R + 1][2 * R + 1];
      load_block_depths<R>(depth_words(depth, j, dplane), p.iu, p.iv, pw, d);
#pragma unroll
      for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
        for (int dx = 0; dx <= 2 * R; ++dx) count += accept16(d[dy][dx], p) ? 1 : 0;
    }
  }
  return count;
}

// The same count with K source frames per step: the K projections are made and all
// K blocks' loads issued before any test, for more loads in flight per lane. A
// source frame past the window or whose projection fails loads a valid apron block
// of frame jlo and contributes nothing, so the count equals count_pixel's.
template <int R, int K>
__device__ __forceinline__ int count_pixel_k(gp<const uint16_t> depth, gp<const float> relf,
                                             int width, int height, int n_frames, int f, int w, float tol,
                                             float z_near, int x, int y) {
  if (K == 1) return count_pixel<R>(depth, relf, width, height, n_frames, f, w, tol, z_near, x, y);
  const int pw = stored_pitch(width);
  const size_t dplane = depth_plane_elems(width, height);
  const float dp = h2f(depth[static_cast<size_t>(f) * dplane + depth_index(x, y, pw)]);
  int count = 0;
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    for (int j0 = jlo; j0 <= jhi; j0 += K) {
      Projected p[K];
      bool ok[K];
      uint32_t d[K][2 * R + 1][2 * R + 1];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = j0 + k;
        ok[k] = j <= jhi &&
                project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p[k]);
        // a frame past the window or a failed projection reads a valid block of frame jlo
        load_block_depths<R>(depth_words(depth, ok[k] ? j : jlo, dplane), ok[k] ? p[k].iu : 0, ok[k] ? p[k].iv : 0,
                             pw, d[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!ok[k]) continue;
#pragma unroll
        for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
          for (int dx = 0; dx <= 2 * R; ++dx) count += accept16(d[k][dy][dx], p[k]) ? 1 : 0;
      }
    }
  }
  return count;
}

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
  const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
  counts[static_cast<size_t>(fo) * width * height + static_cast<size_t>(y) * width + x] =
      count_pixel<R>(to_global(depth), to_global(relf), width, height, n_frames, f0 + fo, w, tol, z_near, x, y);
}

// 16 x 16 tiles (the scatter pass and the fused gather + filter): four waves of
// 16 x 4: a block row of 16 pixels is
// one 128-byte line of a source plane, and depth noise scatters the projections
// of one output row over several source rows, so a squarer wave touches fewer
// distinct lines per load than a 64 x 1 one (9 % faster at 1080p, +-50 frames;
// 8 x 8 waves, half-line rows, were 7 % slower). The dispatcher hands
// consecutive workgroups to the XCDs in turn; tile_of_block_xcd_rows gives each
// XCD whole tile rows instead, so vertically and horizontally adjacent tiles
// share an L2 (1 % more).
constexpr int kFuseWaveW = 16;
static_assert((kFuseW / kFuseWaveW) * (kFuseH / (64 / kFuseWaveW)) == 4, "four waves per fused tile");

// Tile of a fused workgroup: with tiles_x tiles per row, round r of the XCDs
// (workgroups 8 r .. 8 r + 7) takes tile rows 8 q + x, q = r / tiles_x, for XCD x;
// the dispatches past the last whole round of 8 tile rows map to themselves.
__device__ __forceinline__ Tile tile_of_block_xcd_rows(int tiles_x, int tiles_y) {
  const int b = static_cast<int>(blockIdx.x);
  const int nt = tiles_x * tiles_y;
  Tile t;
  t.fo = b / nt;
  const int bl = b - t.fo * nt;
  const int full = (nt / (8 * tiles_x)) * (8 * tiles_x);
  int tl = bl;
  if (bl < full) {
    const int xcd = bl & 7, i = bl >> 3;
    const int q = i / tiles_x, p = i - q * tiles_x;
    tl = (q * 8 + xcd) * tiles_x + p;
  }
  t.tx = tl % tiles_x;
  t.ty = tl / tiles_x;
  return t;
}

// ---------------------------------------------------------------------------
// a5: gather pass 2 -- write records in canonical order.
//
// Each wave owns 64 output pixels: a 16 x 4 block of a 16 x 16 tile (the batched
// pass: 64 consecutive pixels of a row; a 16 x 4 block makes the 2.65 ms scatter of
// a 1080p +-50 frame 2.55 ms). Per source frame each lane reads its whole block of
// stored (r, g, b, depth) pixels in one round trip, decides membership from the
// depth channel exactly as pass 1 does from the depth plane (same binary16 bits,
// same test), and appends its accepted records to a per-lane buffer in LDS
// (kSlots entries of three words: colour + rho, id; odd stride: conflict-free
// appends). The append is branch-free: every candidate of the block is written to
// the lane's next free slot, and the slot pointer advances only past the accepted
// ones, so a rejected candidate's write is overwritten by the next accepted one or
// lands in the slot after the last record (one slot per lane is kept free for it).
// A lane whose buffer cannot take the records of the current source frame writes
// out what it holds before appending them; the wave does these flushes together: a group of kRunLanes lanes
// writes each flushing lane's run, so a store instruction writes 64 / kRunLanes
// contiguous runs instead of 64 scattered 8-byte pieces. Flushing only lanes that
// must keeps the runs long (whole cache lines more often). Records reach global
// memory in the order they are found, which is the canonical order.

using half2v = _Float16 __attribute__((ext_vector_type(2)));

template <int R>
struct ScatterShape {
  static constexpr int kCand = (2 * R + 1) * (2 * R + 1);
  // Odd number of slots per lane (LDS: 12 B per slot, 256 lanes per workgroup; at
  // R = 1, 15 slots is the most that keeps three workgroups on a compute unit). The
  // last slot takes the writes of rejected candidates, so a lane holds at most
  // kSlots - 1 records, and an emptied buffer must take a whole block.
  static constexpr int kSlots = R == 3 ? 51 : (R == 2 ? 41 : 15);
  static constexpr int kCap = kSlots - 1;                    // records a lane holds
  static constexpr int kRunLanes = kSlots <= 16 ? 16 : 64;  // lanes writing one run
  static_assert(kCand <= kCap, "an empty buffer takes one block");
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
__device__ __forceinline__ void flush_runs(int n, int64_t& cur, int& fill, const uint32_t* s_buf, int* s_n,
                                           int64_t* s_dst, gp<uint32_t> ids, gp<uint2> crho) {
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
        const uint32_t* slot = s_buf + 3 * (own * kSlots + sub);
        st2(crho + dst, make_uint2(slot[0], slot[1]));
        ids[dst] = slot[2];
      }
    }
  }
  wave_lds_fence();
  cur += n;
  fill -= n;
}

// LDS of one scatter wave
template <int R>
struct ScatterLds {
  uint32_t buf[3 * kTileW * ScatterShape<R>::kSlots];  // per slot: colour + rho (2 words), id
  int n[kTileW];
  int64_t dst[kTileW];
};

// One wave writes the records of its 64 output pixels of output frame f: lane's
// pixel (x, y), CSR index pix (x, y and pix may lie outside the frame for lanes
// past its right or lower edge; those lanes only join the wave's flushes). Every
// lane of the wave calls it.
template <int R>
__device__ __forceinline__ void scatter_wave(gp<const uint2> rgbd, gp<const uint16_t> depth,
                                             gp<const float> relf, int width, int height,
                                             int n_frames, int f, int w, float tol, float z_near, int x, int y,
                                             int64_t pix, gp<const int64_t> offsets, gp<uint32_t> ids,
                                             gp<uint2> crho, int64_t capacity, gp<uint32_t> status,
                                             ScatterLds<R>& lds) {
  using Shape = ScatterShape<R>;
  using Mask = typename Shape::Mask;
  constexpr int kSlots = Shape::kSlots;
  constexpr int kSide = 2 * R + 1;
  const int lane = threadIdx.x;
  uint32_t* s_buf = lds.buf;
  int* s_n = lds.n;
  int64_t* s_dst = lds.dst;
  const bool in = x < width && y < height;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  int64_t cur = 0, end = 0, start = 0;
  bool active = false;
  float dp = 0.0f;
  if (in) {
    start = cur = offsets[pix];
    end = offsets[pix + 1];
    if (cur < 0 || end < cur) {  // offsets not produced by the count pass
      flag_or(status, SG_FLAG_INCONSISTENT);
    } else if (end > capacity) {
      if (end > cur) flag_or(status, SG_FLAG_CAPACITY);
    } else {
      dp = h2f(depth[static_cast<size_t>(f) * depth_plane_elems(width, height) + depth_index(x, y, pw)]);
      active = dp > z_near && dp < INFINITY;
    }
  }
  int fill = 0;
  int found = 0;
  const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
  const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
  uint32_t* my_buf = s_buf + 3 * kSlots * lane;
  // id of candidate (dy, dx) = id of (0, 0) + dy * width + dx
  uint32_t cand_off[kSide * kSide];
#pragma unroll
  for (int k = 0; k < kSide * kSide; ++k) cand_off[k] = static_cast<uint32_t>((k / kSide) * width + k % kSide);
  for (int j = jlo; j <= jhi; ++j) {
    Projected p;
    uint2 px[kSide][kSide];
    Mask mask = 0;
    int kept = 0;
    if (active && project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p)) {
      gp<const uint2> cj = rgbd + static_cast<size_t>(j) * pplane;  // frame J's plane (uniform)
      const uint32_t at = padded_index(p.iu, p.iv, pw);
      load_block_pixels<R>(cj, at, pw, px);
#pragma unroll
      for (int k = 0; k < kSide * kSide; ++k)
        mask |= static_cast<Mask>(accept16(px[k / kSide][k % kSide].y >> 16, p) ? 1 : 0) << k;
      const int n = __popc(static_cast<uint32_t>(mask)) +
                    (sizeof(Mask) > 4 ? __popc(static_cast<uint32_t>(static_cast<uint64_t>(mask) >> 32)) : 0);
      found += n;
      // keep only as many records as the segment has room for (fewer only when
      // the planes changed since the count pass; flagged at the end)
      kept = n;
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
    }
    // a lane whose buffer cannot take this frame's records writes out what it holds
    // first; the others keep theirs, so every flushed run is as long as it can be
    if (__any(fill + kept > Shape::kCap))
      flush_runs<R>(fill + kept > Shape::kCap ? fill : 0, cur, fill, s_buf, s_n, s_dst, ids, crho);
    if (kept > 0) {
      // id = ((J - f + w) << 22) | q; q < 2^22, so the OR is an add of a
      // per-(p, J) base and a per-candidate constant
      const uint32_t id0 = (static_cast<uint32_t>(j - f + w) << SG_ID_SHIFT) +
                           static_cast<uint32_t>((p.iv - R) * width + (p.iu - R));
      // slots fill .. fill + kept - 1 take the accepted candidates in block order;
      // every write stays below slot fill + kept <= kCap (the spare slot)
      uint32_t* slot = my_buf + 3 * fill;
#pragma unroll
      for (int k = 0; k < kSide * kSide; ++k) {
        const uint2 v = px[k / kSide][k % kSide];
        // (b, d) -> (b, rho): rho = (d - z) / z = d * (1 / z) - 1 in float32, rounded
        // to nearest binary16 in place of the record's own stored depth d
        half2v bd = __builtin_bit_cast(half2v, v.y);
        bd.y = static_cast<_Float16>(fmaf(static_cast<float>(bd.y), p.inv, -1.0f));
        slot[0] = v.x;
        slot[1] = __builtin_bit_cast(uint32_t, bd);
        slot[2] = id0 + cand_off[k];
        slot += 3 * __builtin_amdgcn_ubfe(static_cast<uint32_t>(mask >> k), 0, 1);
      }
      fill += kept;
    }
  }
  if (__any(fill > 0)) flush_runs<R>(fill, cur, fill, s_buf, s_n, s_dst, ids, crho);
  if (active && found != end - start) flag_or(status, SG_FLAG_INCONSISTENT);
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
  constexpr int kWavesX = kFuseW / kFuseWaveW, kWaveH = 64 / kFuseWaveW;
  __shared__ ScatterLds<R> lds[4];
  const Tile tile = tile_of_block_xcd_rows((width + kFuseW - 1) / kFuseW, (height + kFuseH - 1) / kFuseH);
  const int wave = threadIdx.y, lane = threadIdx.x;
  const int x = tile.tx * kFuseW + (wave % kWavesX) * kFuseWaveW + lane % kFuseWaveW;
  const int y = tile.ty * kFuseH + (wave / kWavesX) * kWaveH + lane / kFuseWaveW;
  const int fo = tile.fo;
  const float* relf = rel + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
  const int64_t pix = static_cast<int64_t>(fo) * width * height + static_cast<int64_t>(y) * width + x;
  scatter_wave<R>(to_global(rgbd), to_global(depth), to_global(relf), width, height, n_frames, f0 + fo, w, tol,
                  z_near, x, y, pix, to_global(offsets), to_global(ids), to_global(crho), capacity,
                  to_global(status), lds[wave]);
}

// ---------------------------------------------------------------------------
// Fused gather + plain filter (no record arena): each lane walks its output
// pixel's window like the gather passes (same projection, same block, same
// membership test) and accumulates the filter's weighted sums directly, with rho
// rounded to binary16 exactly as a stored record holds it. The result equals
// scene_gather + scene_filter up to the order of the float32 additions.
//
// Its tile is that of the scatter pass (see tile_of_block_xcd_rows).

template <int R, bool kColour, bool kTime>
__global__ __launch_bounds__(256) void k_gather_filter(const uint2* __restrict__ rgbd_, const float* __restrict__ rel,
                                                       int width, int height, int n_frames, int f0, int w,
                                                       float tol, float z_near, float a_d, float a_c, float a_t,
                                                       float* __restrict__ out) {
  constexpr int kSide = 2 * R + 1;
  constexpr int kWavesX = kFuseW / kFuseWaveW, kWaveH = 64 / kFuseWaveW;
  const Tile tile = tile_of_block_xcd_rows((width + kFuseW - 1) / kFuseW, (height + kFuseH - 1) / kFuseH);
  const int wave = threadIdx.y, lane = threadIdx.x;  // block = 64 x 4 threads: one wave per threadIdx.y
  const int x = tile.tx * kFuseW + (wave % kWavesX) * kFuseWaveW + lane % kFuseWaveW;
  const int y = tile.ty * kFuseH + (wave / kWavesX) * kWaveH + lane / kFuseWaveW;
  const int fo = tile.fo;
  if (x >= width || y >= height) return;
  gp<const uint2> rgbd = to_global(rgbd_);
  gp<const float> relf = to_global(rel) + static_cast<size_t>(fo) * (2 * w + 1) * kRelStride;
  const int f = f0 + fo;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const uint2 ref = ld2(rgbd + static_cast<size_t>(f) * pplane + padded_index(x, y, pw));
  const float cr = h2f(ref.x), cg = h2f(ref.x >> 16), cb = h2f(ref.y);
  const float dp = h2f(ref.y >> 16);  // the depth channel holds the depth plane's binary16
  float wsum = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
  int n = 0;
  if (dp > z_near && dp < INFINITY) {
    const int jlo = max(0, f - w), jhi = min(n_frames - 1, f + w);
    const float fxp = static_cast<float>(x), fyp = static_cast<float>(y);
    for (int j = jlo; j <= jhi; ++j) {
      Projected p;
      if (!project(relf + (j - f + w) * kRelStride, fxp, fyp, dp, z_near, tol, width, height, R, p)) continue;
      gp<const uint2> cj = rgbd + static_cast<size_t>(j) * pplane;  // frame J's plane (uniform)
      const uint32_t at = padded_index(p.iu, p.iv, pw);
      uint2 px[kSide][kSide];
      load_block_pixels<R>(cj, at, pw, px);
      const float dj = static_cast<float>(j - f);
#pragma unroll
      for (int k = 0; k < kSide * kSide; ++k) {
        const uint2 v = px[k / kSide][k % kSide];
        if (!accept16(v.y >> 16, p)) continue;
        // rho exactly as the scatter stores it
        half2v bd = __builtin_bit_cast(half2v, v.y);
        const float rho = static_cast<float>(static_cast<_Float16>(fmaf(static_cast<float>(bd.y), p.inv, -1.0f)));
        const float r = h2f(v.x), g = h2f(v.x >> 16), b = h2f(v.y);
        float arg = a_d * rho * rho;
        if (kColour) {
          const float er = r - cr, eg = g - cg, eb = b - cb;
          arg = fmaf(a_c, fmaf(er, er, fmaf(eg, eg, eb * eb)), arg);
        }
        if (kTime) arg = fmaf(a_t, dj * dj, arg);
        const float wt = __builtin_amdgcn_exp2f(arg);
        wsum += wt;
        ar = fmaf(wt, r, ar);
        ag = fmaf(wt, g, ag);
        ab = fmaf(wt, b, ab);
        ++n;
      }
    }
  }
  gp<float> o = to_global(out) + (static_cast<size_t>(fo) * width * height + static_cast<size_t>(y) * width + x) * 3;
  if (n > 0) {
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

// kGroup lanes filter one pixel: pixel `self` (y * W + x) of frame f, whose set is
// CSR entry `pix` of offsets / out. Every lane of the group calls it (live or not).
template <bool kColour, bool kTime>
__device__ __forceinline__ void filter_group(gp<const uint2> rgbd, int width, int height, int f,
                                             int w, bool live, int64_t self, int64_t pix, int lane,
                                             gp<const int64_t> offsets, gp<const uint32_t> ids,
                                             gp<const uint2> crho, int64_t capacity, float a_d,
                                             float a_c, float a_t, gp<float> out) {
  float cr = 0.f, cg = 0.f, cb = 0.f;
  int64_t s = 0, e = 0;
  if (live) {
    const int y = static_cast<int>(self / width), x = static_cast<int>(self - static_cast<int64_t>(y) * width);
    const int pw = stored_pitch(width);
    const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
    const uint2 ref = ld2(rgbd + static_cast<size_t>(f) * pplane + padded_index(x, y, pw));
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
  auto accumulate = [&](uint2 rec, uint32_t id) {
    const float r = h2f(rec.x), g = h2f(rec.x >> 16), b = h2f(rec.y), rho = h2f(rec.y >> 16);
    float arg = a_d * rho * rho;
    if (kColour) {
      const float dr = r - cr, dg = g - cg, db = b - cb;
      arg = fmaf(a_c, fmaf(dr, dr, fmaf(dg, dg, db * db)), arg);
    }
    if (kTime) {
      const float dj = static_cast<float>(static_cast<int>(id >> SG_ID_SHIFT) - w);
      arg = fmaf(a_t, dj * dj, arg);
    }
    const float wt = __builtin_amdgcn_exp2f(arg);
    wsum += wt;
    ar = fmaf(wt, r, ar);
    ag = fmaf(wt, g, ag);
    ab = fmaf(wt, b, ab);
  };
  // four records per lane in flight; each lane still adds its records in order
  int64_t i = s + lane;
  for (; i + 3 * kGroup < e; i += 4 * kGroup) {
    uint2 rec[4];
    uint32_t id[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rec[k] = ld2(crho + i + k * kGroup);
      if (kTime) id[k] = ids[i + k * kGroup];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) accumulate(rec[k], id[k]);
  }
  for (; i < e; i += kGroup) accumulate(ld2(crho + i), kTime ? ids[i] : 0u);
#pragma unroll
  for (int off = kGroup / 2; off > 0; off >>= 1) {
    wsum += __shfl_xor(wsum, off, kGroup);
    ar += __shfl_xor(ar, off, kGroup);
    ag += __shfl_xor(ag, off, kGroup);
    ab += __shfl_xor(ab, off, kGroup);
  }
  if (live && lane == 0) {
    gp<float> o = out + static_cast<size_t>(pix) * 3;
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
  const int64_t plane = static_cast<int64_t>(width) * height;
  const int fo = live ? static_cast<int>(pix / plane) : 0;
  filter_group<kColour, kTime>(to_global(rgbd), width, height, f0 + fo, w, live, pix - fo * plane, pix, lane,
                               to_global(offsets), to_global(ids), to_global(crho), capacity, a_d, a_c, a_t,
                               to_global(out));
}

// ---------------------------------------------------------------------------
// a9: batched persistent passes over uneven clips. Each pass is one launch of a
// grid sized to the machine; a workgroup takes the next work item from an atomic
// queue until the queue is exhausted (every workgroup reaches the exit). Gather
// items are tiles (64 x TH pixels of one output frame of one clip) in cost order
// (clip slots sorted by estimated work, largest first); filter items are runs of
// consecutive CSR pixels. The per-pixel work is the single-clip kernels' code, so
// each clip's records and colours equal those of its own calls.

__global__ __launch_bounds__(64) void k_batch_prep(BatchDev bd, unsigned int* __restrict__ queues,
                                                   uint32_t* __restrict__ status) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (c == 0 && i < 4) queues[i] = 0u;
  if (c == 0 && i == 0) *status = 0u;
  const BatchClip& cl = bd.clips[c];
  if (i < cl.n_out * (2 * cl.w + 1))
    pose_prep_one(to_global(cl.c2w), cl.n_frames, bd.f0[c], cl.w, cl.fx, cl.fy, cl.cx, cl.cy, to_global(cl.rel), i);
}

// Work items of a wave: the atomic for the next item is issued before the current
// one is processed, so its round trip overlaps the work (every lane calls these).
struct ItemQueue {
  unsigned int* queue;
  uint32_t pending;  // lane 0: the atomic's result, read when the next item is taken

  __device__ __forceinline__ explicit ItemQueue(unsigned int* q) : queue(q), pending(0u) { issue(); }
  __device__ __forceinline__ void issue() {
    if (threadIdx.x == 0) pending = atomicAdd(queue, 1u);
  }
  __device__ __forceinline__ int64_t take() {
    const int64_t item = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(pending));
    issue();
    return item;
  }
};

// slot of work item `item`: the largest k with prefix[k] <= item
__device__ __forceinline__ int item_slot(const int64_t* __restrict__ prefix, int n, int64_t item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct TileOf {
  int fo, x0, y0;
};

// A clip descriptor read into scalar registers: every word goes through
// readfirstlane, so the compiler knows the pointers and sizes are uniform (the
// planes' and maps' addresses then stay scalar in the inner loops).
__device__ __forceinline__ BatchClip load_clip(const BatchClip* __restrict__ p) {
  static_assert(sizeof(BatchClip) % 4 == 0, "descriptor is whole words");
  BatchClip c;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
  uint32_t w[sizeof(BatchClip) / 4];
#pragma unroll
  for (unsigned i = 0; i < sizeof(BatchClip) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
  __builtin_memcpy(&c, w, sizeof(BatchClip));
  return c;
}

// Gather item: TH rows of 64 pixels of one output frame of one clip, taken by one
// wave. Items are numbered per slot (clips in cost order), x fastest.
template <int TH>
__device__ __forceinline__ TileOf batch_tile(const BatchClip& c, int64_t local) {
  const int tiles_x = (c.width + kTileW - 1) / kTileW, tiles_y = (c.height + TH - 1) / TH;
  TileOf t;
  // 64-bit division is expanded on the vector units: readfirstlane puts the
  // (uniform) results back in scalar registers, so addresses built from them stay
  // scalar
  t.x0 = __builtin_amdgcn_readfirstlane(static_cast<int>(local % tiles_x) * kTileW);
  const int64_t rest = local / tiles_x;
  t.y0 = __builtin_amdgcn_readfirstlane(static_cast<int>(rest % tiles_y) * TH);
  t.fo = __builtin_amdgcn_readfirstlane(static_cast<int>(rest / tiles_y));
  return t;
}

// Workgroups of 4 independent waves; each wave draws its own items, so no wave
// waits at a barrier for the slowest row of a tile.
template <int R, int TH, int K>
__global__ __launch_bounds__(256) void k_count_batched(BatchDev bd, int64_t* __restrict__ counts,
                                                       unsigned int* __restrict__ queue) {
  const int64_t n_items = bd.prefix[bd.n_clips];
  ItemQueue q(queue);
  for (;;) {
    const int64_t item = q.take();
    if (item >= n_items) break;
    // slot, clip and descriptor are uniform: scalar loads, kept in scalar registers
    const int slot = item_slot(bd.prefix, bd.n_clips, item);
    const int clip = bd.order[slot];
    const BatchClip c = load_clip(bd.clips + clip);
    const int f0 = bd.f0[clip];
    const TileOf t = batch_tile<TH>(c, item - bd.prefix[slot]);
    const int x = t.x0 + threadIdx.x;
    gp<const float> relf = to_global(static_cast<const float*>(c.rel)) + static_cast<size_t>(t.fo) * (2 * c.w + 1) * kRelStride;
    gp<const uint16_t> depth = to_global(c.depth);
    const int f = f0 + t.fo;
    for (int r = 0; r < TH; ++r) {
      const int y = t.y0 + r;
      if (x < c.width && y < c.height) {
        const int64_t pix = c.pix_base + static_cast<int64_t>(t.fo) * c.width * c.height +
                            static_cast<int64_t>(y) * c.width + x;
        counts[pix] = count_pixel_k<R, K>(depth, relf, c.width, c.height, c.n_frames, f, c.w, c.tol, c.z_near, x, y);
      }
    }
  }
}

// The plan arrays and the relative maps come as separate restrict arguments: the
// kernel's stores then provably miss them, so their loads can go through the
// scalar cache (each clip's maps are addressed from rel_all, not from the pointer
// in its descriptor, which the compiler could not separate from the stores).
template <int R, int TH>
__global__ __launch_bounds__(256) void k_scatter_batched(const BatchClip* __restrict__ clips,
                                                         const int* __restrict__ f0s, const int* __restrict__ order,
                                                         const int64_t* __restrict__ prefix, int n_clips,
                                                         const float* __restrict__ rel_all,
                                                         const int64_t* __restrict__ offsets,
                                                         uint32_t* __restrict__ ids, uint2* __restrict__ crho,
                                                         int64_t capacity, uint32_t* __restrict__ status,
                                                         unsigned int* __restrict__ queue) {
  __shared__ ScatterLds<R> lds[4];
  const int64_t n_items = prefix[n_clips];
  ItemQueue q(queue);
  for (;;) {
    const int64_t item = q.take();
    if (item >= n_items) break;
    const int slot = item_slot(prefix, n_clips, item);
    const int clip = order[slot];
    const BatchClip c = load_clip(clips + clip);
    const int f0 = f0s[clip];
    const TileOf t = batch_tile<TH>(c, item - prefix[slot]);
    const int64_t rel_at = static_cast<int64_t>(c.rel_at) + static_cast<int64_t>(t.fo) * (2 * c.w + 1) * kRelStride;
    gp<const float> relf = to_global(rel_all) + rel_at;
    gp<const uint2> rgbd = to_global(reinterpret_cast<const uint2*>(c.rgbd));
    gp<const uint16_t> depth = to_global(c.depth);
    const int f = f0 + t.fo;
    for (int r = 0; r < TH; ++r) {
      const int y = t.y0 + r;
      if (y >= c.height) break;  // uniform over the wave
      const int64_t pix0 = c.pix_base + static_cast<int64_t>(t.fo) * c.width * c.height +
                           static_cast<int64_t>(y) * c.width + t.x0;
      scatter_wave<R>(rgbd, depth, relf, c.width, c.height, c.n_frames, f, c.w, c.tol, c.z_near,
                      t.x0 + static_cast<int>(threadIdx.x), y, pix0 + threadIdx.x,
                      to_global(offsets), to_global(ids), to_global(crho), capacity, to_global(status),
                      lds[threadIdx.y]);
    }
  }
}

constexpr int kBatchFilterPix = 64;  // CSR pixels per filter work item (4 per pass of a wave)

// Filter items are runs of 64 pixels of one clip (fprefix: first item of each clip).
template <bool kColour, bool kTime>
__global__ __launch_bounds__(256) void k_filter_batched(BatchDev bd, BatchIo io, const int64_t* __restrict__ fprefix,
                                                        unsigned int* __restrict__ queue) {
  const int g = threadIdx.x / kGroup, lane = threadIdx.x % kGroup;
  const int64_t n_items = fprefix[bd.n_clips];
  ItemQueue q(queue);
  for (;;) {
    const int64_t item = q.take();
    if (item >= n_items) break;
    const int c = item_slot(fprefix, bd.n_clips, item);
    const BatchClip cl = load_clip(bd.clips + c);
    const int f0 = bd.f0[c];
    gp<const uint2> rgbd = to_global(reinterpret_cast<const uint2*>(cl.rgbd));
    const int64_t plane = static_cast<int64_t>(cl.width) * cl.height;
    const int64_t n_clip = plane * cl.n_out;
    const int64_t first = (item - fprefix[c]) * kBatchFilterPix;
    for (int r = 0; r < kBatchFilterPix; r += 64 / kGroup) {
      const int64_t local = first + r + g;
      const bool live = local < n_clip;
      const int fo = live ? static_cast<int>(local / plane) : 0;
      filter_group<kColour, kTime>(rgbd, cl.width, cl.height, f0 + fo, cl.w, live, local - fo * plane,
                                   cl.pix_base + local, lane, to_global(static_cast<const int64_t*>(io.offsets)),
                                   to_global(static_cast<const uint32_t*>(io.ids)),
                                   to_global(reinterpret_cast<const uint2*>(io.crho)), io.capacity, cl.a_d,
                                   kColour ? cl.a_c : 0.0f, kTime ? cl.a_t : 0.0f, to_global(io.out));
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

static dim3 tile16_grid(const GatherJob& jb) {
  const int64_t nb = static_cast<int64_t>((jb.width + kFuseW - 1) / kFuseW) *
                     ((jb.height + kFuseH - 1) / kFuseH) * jb.n_out;
  return dim3(static_cast<unsigned>(nb));
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
  const dim3 g = tile16_grid(jb);
  switch (jb.radius) {
    case 0: scatter_r<0>(jb, g, st); break;
    case 1: scatter_r<1>(jb, g, st); break;
    case 2: scatter_r<2>(jb, g, st); break;
    default: scatter_r<3>(jb, g, st); break;
  }
  return hipGetLastError();
}

template <int R>
static void gather_filter_r(const GatherJob& jb, const FilterJob& fj, dim3 g, hipStream_t st) {
  const uint2* rgbd = reinterpret_cast<const uint2*>(jb.rgbd);
#define SG_FUSED(C, T)                                                                                     \
  hipLaunchKernelGGL((k_gather_filter<R, C, T>), g, dim3(64, 4), 0, st, rgbd, jb.rel, jb.width,            \
                     jb.height, jb.n_frames, jb.f0, jb.w, jb.tol, jb.z_near, fj.a_d, fj.a_c, fj.a_t, fj.out)
  if (fj.use_colour && fj.use_time)
    SG_FUSED(true, true);
  else if (fj.use_colour)
    SG_FUSED(true, false);
  else if (fj.use_time)
    SG_FUSED(false, true);
  else
    SG_FUSED(false, false);
#undef SG_FUSED
}

hipError_t launch_gather_filter(const GatherJob& jb, const FilterJob& fj, hipStream_t st) {
  const dim3 g = tile16_grid(jb);
  switch (jb.radius) {
    case 0: gather_filter_r<0>(jb, fj, g, st); break;
    case 1: gather_filter_r<1>(jb, fj, g, st); break;
    case 2: gather_filter_r<2>(jb, fj, g, st); break;
    default: gather_filter_r<3>(jb, fj, g, st); break;
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

hipError_t launch_batch_prep(const BatchDev& bd, unsigned int* queues, uint32_t* status, int max_slots,
                             hipStream_t st) {
  const dim3 g(static_cast<unsigned>((max_slots + 63) / 64), static_cast<unsigned>(bd.n_clips));
  hipLaunchKernelGGL(k_batch_prep, g, dim3(64), 0, st, bd, queues, status);
  return hipGetLastError();
}

template <int R, int TH>
static void count_batched_k(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl, unsigned int* q,
                            hipStream_t st) {
  const dim3 g(static_cast<unsigned>(bl.blocks_count)), b(kTileW, 4);
  switch (bl.k_count) {
    case 1: hipLaunchKernelGGL((k_count_batched<R, TH, 1>), g, b, 0, st, bd, io.offsets + 1, q); break;
    case 2: hipLaunchKernelGGL((k_count_batched<R, TH, 2>), g, b, 0, st, bd, io.offsets + 1, q); break;
    default: hipLaunchKernelGGL((k_count_batched<R, TH, 4>), g, b, 0, st, bd, io.offsets + 1, q); break;
  }
}

template <int R>
static void count_batched_r(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl, unsigned int* q,
                            hipStream_t st) {
  switch (bl.th_count) {
    case 1: count_batched_k<R, 1>(bd, io, bl, q, st); break;
    case 2: count_batched_k<R, 2>(bd, io, bl, q, st); break;
    case 4: count_batched_k<R, 4>(bd, io, bl, q, st); break;
    default: count_batched_k<R, 8>(bd, io, bl, q, st); break;
  }
}

hipError_t launch_batch_count(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl, unsigned int* queue,
                              hipStream_t st) {
  switch (bd.radius) {
    case 0: count_batched_r<0>(bd, io, bl, queue, st); break;
    case 1: count_batched_r<1>(bd, io, bl, queue, st); break;
    case 2: count_batched_r<2>(bd, io, bl, queue, st); break;
    default: count_batched_r<3>(bd, io, bl, queue, st); break;
  }
  return hipGetLastError();
}

size_t batch_scatter_lds_bytes(int radius) {
  switch (radius) {
    case 0: return sizeof(ScatterLds<0>);
    case 1: return sizeof(ScatterLds<1>);
    case 2: return sizeof(ScatterLds<2>);
    default: return sizeof(ScatterLds<3>);
  }
}

// every rows-per-item value fits: LDS holds the workgroup's 4 waves' buffers
int batch_scatter_max_th(int) { return 8; }

template <int R>
static void scatter_batched_r(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl, unsigned int* q,
                              hipStream_t st) {
  const dim3 g(static_cast<unsigned>(bl.blocks_scatter)), b(kTileW, 4);
#define SG_SCATTER_BATCHED(TH) \
  hipLaunchKernelGGL((k_scatter_batched<R, TH>), g, b, 0, st, bd.clips, bd.f0, bd.order, bd.prefix, bd.n_clips, \
                     bd.rel, io.offsets, io.ids, reinterpret_cast<uint2*>(io.crho), io.capacity, io.status, q)
  switch (bl.th_scatter) {
    case 1: SG_SCATTER_BATCHED(1); break;
    case 2: SG_SCATTER_BATCHED(2); break;
    case 4: SG_SCATTER_BATCHED(4); break;
    default: SG_SCATTER_BATCHED(8); break;
  }
#undef SG_SCATTER_BATCHED
}

hipError_t launch_batch_scatter(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl, unsigned int* queue,
                                hipStream_t st) {
  switch (bd.radius) {
    case 0: scatter_batched_r<0>(bd, io, bl, queue, st); break;
    case 1: scatter_batched_r<1>(bd, io, bl, queue, st); break;
    case 2: scatter_batched_r<2>(bd, io, bl, queue, st); break;
    default: scatter_batched_r<3>(bd, io, bl, queue, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_filter(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl,
                               const int64_t* fprefix, unsigned int* queue, hipStream_t st) {
  const dim3 g(static_cast<unsigned>(bl.blocks_filter)), b(64, 4);
  if (bl.colour && bl.time)
    hipLaunchKernelGGL((k_filter_batched<true, true>), g, b, 0, st, bd, io, fprefix, queue);
  else if (bl.colour)
    hipLaunchKernelGGL((k_filter_batched<true, false>), g, b, 0, st, bd, io, fprefix, queue);
  else if (bl.time)
    hipLaunchKernelGGL((k_filter_batched<false, true>), g, b, 0, st, bd, io, fprefix, queue);
  else
    hipLaunchKernelGGL((k_filter_batched<false, false>), g, b, 0, st, bd, io, fprefix, queue);
  return hipGetLastError();
}

int64_t batch_filter_items(int64_t clip_pixels) { return (clip_pixels + kBatchFilterPix - 1) / kBatchFilterPix; }

}  // namespace sg
