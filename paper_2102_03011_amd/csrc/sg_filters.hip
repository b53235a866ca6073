// The paper's other filters over stored sample sets (Sec. 5): the per-frame
// factor of deblurring (Eq. 5) and computational shutters (Eq. 10), the frame
// sharpness B(J) that deblurring weights by, inpainting by masked mean-shift
// (Eq. 8-9) and its masks from a scene-space box. Same record layout and lane organisation as the denoising filter:
// 16 lanes per output pixel stride through its CSR segment, each in a fixed
// order, then a fixed butterfly combines them.
//
// Every table lookup made from a record's id (frame factor, source mask) is
// bounds-checked: an id whose source frame or pixel lies outside the clip (sets
// gathered with another window, or not produced by the gather) makes its output
// pixel NaN, never a read outside the table.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "scene_filters.h"
#include "sg_device.h"
#include "sg_internal.h"
#include "sg_validate.h"

namespace sg {
namespace {

constexpr int kLanes = 16;           // lanes per output pixel
constexpr int kFilterThreads = 256;  // 16 pixels per workgroup
constexpr uint32_t kQMask = (1u << SG_ID_SHIFT) - 1u;

// ---------------------------------------------------------------------------
// B(J) of Eq. 5: one workgroup per frame. Each thread walks columns x, x + 1024,
// ... top to bottom, carrying the current row's pixel and its right neighbour and
// loading kSharpRows rows below at a time (all in flight together); magnitudes in
// float32, per-thread sums in float64, then a fixed tree over the workgroup.

constexpr int kSharpThreads = 1024;
constexpr int kSharpRows = 8;

__device__ __forceinline__ float grad_magnitude(uint2 c, uint2 right, uint2 down) {
  const float c0 = h2f(c.x), c1 = h2f(c.x >> 16), c2 = h2f(c.y);
  const float x0 = h2f(right.x) - c0, x1 = h2f(right.x >> 16) - c1, x2 = h2f(right.y) - c2;
  const float y0 = h2f(down.x) - c0, y1 = h2f(down.x >> 16) - c1, y2 = h2f(down.y) - c2;
  return sqrtf(x0 * x0 + x1 * x1 + x2 * x2 + y0 * y0 + y1 * y1 + y2 * y2);
}

__global__ __launch_bounds__(kSharpThreads) void k_frame_sharpness(const uint2* __restrict__ rgbd_, int width,
                                                                   int height, float* __restrict__ out) {
  const int j = blockIdx.x;
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  gp<const uint2> plane = to_global(rgbd_) + static_cast<size_t>(j) * pplane;
  double acc = 0.0;
  for (int x = threadIdx.x; x + 1 < width; x += kSharpThreads) {
    gp<const uint2> col = plane + padded_index(x, 0, pw);  // (x, 0); x + 1 is in the image
    uint2 c = ld2(col), right = ld2(col + 1);
    for (int y = 0; y + 1 < height; y += kSharpRows) {
      uint2 d[kSharpRows], dr[kSharpRows];
#pragma unroll
      for (int k = 0; k < kSharpRows; ++k) {
        // rows past the image's last are replaced by the last (read, not counted)
        const int yy = min(y + 1 + k, height - 1);
        d[k] = ld2(col + static_cast<size_t>(yy) * pw);
        dr[k] = ld2(col + static_cast<size_t>(yy) * pw + 1);
      }
#pragma unroll
      for (int k = 0; k < kSharpRows; ++k) {
        if (y + k + 1 < height) acc += static_cast<double>(grad_magnitude(c, right, d[k]));
        c = d[k];
        right = dr[k];
      }
    }
  }
  __shared__ double part[kSharpThreads];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kSharpThreads / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = static_cast<float>(part[0]);
}

// ---------------------------------------------------------------------------
// Output pixel of a 16-lane group and its set.

struct PixelSet {
  bool live;     // the group has an output pixel
  bool bad;      // its set lies outside the arena (or malformed offsets)
  int f;         // output frame
  int64_t self;  // y * W + x within the frame
  int64_t s, e;  // record range
  float cr, cg, cb;
};

__device__ __forceinline__ PixelSet pixel_set(gp<const uint2> rgbd, int width, int height, int f0, int64_t n_pix,
                                              gp<const int64_t> offsets, int64_t capacity, int64_t pix) {
  PixelSet p{};
  p.live = pix < n_pix;
  if (!p.live) return p;
  const int64_t frame_px = static_cast<int64_t>(width) * height;
  const int64_t fo = pix / frame_px;
  p.f = f0 + static_cast<int>(fo);
  p.self = pix - fo * frame_px;
  const int y = static_cast<int>(p.self / width), x = static_cast<int>(p.self - static_cast<int64_t>(y) * width);
  const int pw = stored_pitch(width);
  const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
  const uint2 ref = ld2(rgbd + static_cast<size_t>(p.f) * pplane + padded_index(x, y, pw));
  p.cr = h2f(ref.x);
  p.cg = h2f(ref.x >> 16);
  p.cb = h2f(ref.y);
  p.s = offsets[pix];
  p.e = offsets[pix + 1];
  p.bad = p.s < 0 || p.e < p.s || p.e > capacity;
  if (p.bad) p.s = p.e = 0;
  return p;
}

// sum over the 16 lanes of a group, the same value in every lane
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int off = kLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanes);
  return v;
}
__device__ __forceinline__ int group_or(int v) {
#pragma unroll
  for (int off = kLanes / 2; off > 0; off >>= 1) v |= __shfl_xor(v, off, kLanes);
  return v;
}

__device__ __forceinline__ void store_rgb(gp<float> out, int64_t pix, float r, float g, float b) {
  gp<float> o = out + static_cast<size_t>(pix) * 3;
  o[0] = r;
  o[1] = g;
  o[2] = b;
}

// ---------------------------------------------------------------------------
// Eq. 3 with the Eq. 4 weight times frame_w[J].

template <bool kColour, bool kTime>
__global__ __launch_bounds__(kFilterThreads) void k_filter_frames(
    const uint2* __restrict__ rgbd_, int width, int height, int n_frames, int f0, int w, int64_t n_pix,
    const int64_t* __restrict__ offsets_, const uint32_t* __restrict__ ids_, const uint2* __restrict__ crho_,
    int64_t capacity, float a_d, float a_c, float a_t, const float* __restrict__ frame_w_, float* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kFilterThreads + threadIdx.x;
  const int64_t pix = t / kLanes;
  const int lane = static_cast<int>(t % kLanes);
  gp<const uint32_t> ids = to_global(ids_);
  gp<const uint2> crho = to_global(crho_);
  gp<const float> frame_w = to_global(frame_w_);
  const PixelSet p = pixel_set(to_global(rgbd_), width, height, f0, n_pix, to_global(offsets_), capacity, pix);
  const int jbase = p.f - w;  // J = jbase + (id >> SG_ID_SHIFT)
  float wsum = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
  int bad_id = 0;
  auto accumulate = [&](uint2 rec, uint32_t id, float fw) {
    const float r = h2f(rec.x), g = h2f(rec.x >> 16), b = h2f(rec.y), rho = h2f(rec.y >> 16);
    float arg = a_d * rho * rho;
    if (kColour) {
      const float er = r - p.cr, eg = g - p.cg, eb = b - p.cb;
      arg = fmaf(a_c, fmaf(er, er, fmaf(eg, eg, eb * eb)), arg);
    }
    if (kTime) {
      const float fdj = static_cast<float>(static_cast<int>(id >> SG_ID_SHIFT) - w);
      arg = fmaf(a_t, fdj * fdj, arg);
    }
    const float wt = __builtin_amdgcn_exp2f(arg) * fw;
    wsum += wt;
    ar = fmaf(wt, r, ar);
    ag = fmaf(wt, g, ag);
    ab = fmaf(wt, b, ab);
  };
  // factor of a record's frame, 0 (and bad_id set) when the id's frame is outside the clip
  auto factor = [&](uint32_t id) {
    const int j = jbase + static_cast<int>(id >> SG_ID_SHIFT);
    if (j < 0 || j >= n_frames) {
      bad_id = 1;
      return 0.0f;
    }
    return frame_w[j];
  };
  // four records per lane in flight (records, then their frames' factors); each
  // lane still adds its records in order
  int64_t i = p.s + lane;
  for (; i + 3 * kLanes < p.e; i += 4 * kLanes) {
    uint2 rec[4];
    uint32_t id[4];
    float fw[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rec[k] = ld2(crho + i + k * kLanes);
      id[k] = ids[i + k * kLanes];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) fw[k] = factor(id[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) accumulate(rec[k], id[k], fw[k]);
  }
  for (; i < p.e; i += kLanes) {
    const uint32_t id = ids[i];
    accumulate(ld2(crho + i), id, factor(id));
  }
  wsum = group_sum(wsum);
  ar = group_sum(ar);
  ag = group_sum(ag);
  ab = group_sum(ab);
  bad_id = group_or(bad_id);
  if (p.live && lane == 0) {
    if (p.bad || bad_id) {
      const float nan = __builtin_nanf("");
      store_rgb(to_global(out), pix, nan, nan, nan);
    } else if (wsum > 0.f) {
      const float inv = 1.0f / wsum;
      store_rgb(to_global(out), pix, ar * inv, ag * inv, ab * inv);
    } else {
      store_rgb(to_global(out), pix, p.cr, p.cg, p.cb);
    }
  }
}

// ---------------------------------------------------------------------------
// Eq. 3 with the full Eq. 4 weight: colour, scene-space position and frame time
// around the reference sample, the depth-residual term, and an optional per-frame
// factor (Eq. 5). The scene-space distance between a sample (J, q, stored depth
// D) and the reference point X of output pixel p is measured in the camera frame
// of J (rigid maps keep distances): with the folded map of (f, J), Y = d_p M (x, y, 1)
// + k = K (camera-J coordinates of X), and K (camera-J coordinates of the sample)
// = D (q_x, q_y, 1), so their difference e = D (q_x, q_y, 1) - Y gives the distance
// vector K^-1 e = ((e_x - cx e_z) / fx, (e_y - cy e_z) / fy, e_z).

struct XyzArgs {
  const float* rel;       // relative maps of the output frames [n_out][2w + 1][kRelStride]
  const uint16_t* depth;  // stored depth planes
  float a_x;              // -log2(e) / (2 sigma_xyz^2), 0 when the term is off
  float fx_inv, fy_inv, cx, cy;
};

__global__ __launch_bounds__(kFilterThreads) void k_filter_xyz(
    const uint2* __restrict__ rgbd_, int width, int height, int n_frames, int f0, int w, int64_t n_pix,
    const int64_t* __restrict__ offsets_, const uint32_t* __restrict__ ids_, const uint2* __restrict__ crho_,
    int64_t capacity, float a_d, float a_c, float a_t, const float* __restrict__ frame_w_, XyzArgs xa,
    float* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kFilterThreads + threadIdx.x;
  const int64_t pix = t / kLanes;
  const int lane = static_cast<int>(t % kLanes);
  gp<const uint32_t> ids = to_global(ids_);
  gp<const uint2> crho = to_global(crho_);
  gp<const float> frame_w = to_global(frame_w_);
  gp<const uint16_t> depth = to_global(xa.depth);
  gp<const uint2> rgbd = to_global(rgbd_);
  const PixelSet p = pixel_set(rgbd, width, height, f0, n_pix, to_global(offsets_), capacity, pix);
  const bool use_xyz = xa.a_x != 0.0f;
  const int pw = stored_pitch(width);
  const size_t dplane = depth_plane_elems(width, height);
  const int64_t frame_px = static_cast<int64_t>(width) * height;
  // the reference point: p's own stored depth
  float dp = 0.0f, px = 0.0f, py = 0.0f;
  bool no_ref = false;
  gp<const float> relf = to_global(xa.rel);
  if (p.live) {
    const int y = static_cast<int>(p.self / width), x = static_cast<int>(p.self - static_cast<int64_t>(y) * width);
    px = static_cast<float>(x);
    py = static_cast<float>(y);
    dp = h2f(depth[static_cast<size_t>(p.f) * dplane + depth_index(x, y, pw)]);
    no_ref = use_xyz && !(dp > 0.0f && dp < INFINITY);
    relf = relf + static_cast<size_t>(p.f - f0) * (2 * w + 1) * kRelStride;
  }
  const int jbase = p.f - w;
  float wsum = 0.f, ar = 0.f, ag = 0.f, ab = 0.f;
  int bad_id = 0;
  const float inv_w = 1.0f / static_cast<float>(width);
  auto accumulate = [&](uint2 rec, uint32_t id) {
    const float r = h2f(rec.x), g = h2f(rec.x >> 16), b = h2f(rec.y), rho = h2f(rec.y >> 16);
    const int dj = static_cast<int>(id >> SG_ID_SHIFT);
    const int j = jbase + dj;
    const int64_t q = static_cast<int64_t>(id & kQMask);
    if (j < 0 || j >= n_frames || q >= frame_px) {  // not an id of this clip and window
      bad_id = 1;
      return;
    }
    float arg = a_d * rho * rho;
    const float er = r - p.cr, eg = g - p.cg, eb = b - p.cb;
    arg = fmaf(a_c, fmaf(er, er, fmaf(eg, eg, eb * eb)), arg);
    const float fdj = static_cast<float>(dj - w);
    arg = fmaf(a_t, fdj * fdj, arg);
    if (use_xyz) {
      // q -> (q_x, q_y): float quotient, corrected to the exact one (q < 2^22)
      const int qi = static_cast<int>(q);
      int qy = static_cast<int>(static_cast<float>(qi) * inv_w);
      int qx = qi - qy * width;
      if (qx < 0) { --qy; qx += width; }
      if (qx >= width) { ++qy; qx -= width; }
      const float d = h2f(depth[static_cast<size_t>(j) * dplane + depth_index(qx, qy, pw)]);
      gp<const float> m = relf + dj * kRelStride;
      const float y0 = fmaf(dp, fmaf(m[0], px, fmaf(m[1], py, m[2])), m[9]);
      const float y1 = fmaf(dp, fmaf(m[3], px, fmaf(m[4], py, m[5])), m[10]);
      const float z = fmaf(dp, fmaf(m[6], px, fmaf(m[7], py, m[8])), m[11]);
      const float ex = fmaf(d, static_cast<float>(qx), -y0);
      const float ey = fmaf(d, static_cast<float>(qy), -y1);
      const float ez = d - z;
      const float vx = fmaf(-xa.cx, ez, ex) * xa.fx_inv;
      const float vy = fmaf(-xa.cy, ez, ey) * xa.fy_inv;
      arg = fmaf(xa.a_x, fmaf(vx, vx, fmaf(vy, vy, ez * ez)), arg);
    }
    float wt = __builtin_amdgcn_exp2f(arg);
    if (frame_w_ != nullptr) wt *= frame_w[j];
    wsum += wt;
    ar = fmaf(wt, r, ar);
    ag = fmaf(wt, g, ag);
    ab = fmaf(wt, b, ab);
  };
  if (!no_ref) {
    // four records per lane in flight; each lane adds its records in order
    int64_t i = p.s + lane;
    for (; i + 3 * kLanes < p.e; i += 4 * kLanes) {
      uint2 rec[4];
      uint32_t id[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rec[k] = ld2(crho + i + k * kLanes);
        id[k] = ids[i + k * kLanes];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) accumulate(rec[k], id[k]);
    }
    for (; i < p.e; i += kLanes) accumulate(ld2(crho + i), ids[i]);
  }
  wsum = group_sum(wsum);
  ar = group_sum(ar);
  ag = group_sum(ag);
  ab = group_sum(ab);
  bad_id = group_or(bad_id);
  if (p.live && lane == 0) {
    if (p.bad || bad_id) {
      const float nan = __builtin_nanf("");
      store_rgb(to_global(out), pix, nan, nan, nan);
    } else if (wsum > 0.f) {
      const float inv = 1.0f / wsum;
      store_rgb(to_global(out), pix, ar * inv, ag * inv, ab * inv);
    } else {
      store_rgb(to_global(out), pix, p.cr, p.cg, p.cb);
    }
  }
}

// ---------------------------------------------------------------------------
// Inpainting: mean of the set, then `steps` weighted means around the current
// estimate with masked source pixels left out.

__global__ __launch_bounds__(kFilterThreads) void k_inpaint(
    const uint2* __restrict__ rgbd_, int width, int height, int n_frames, int f0, int w, int64_t n_pix,
    const int64_t* __restrict__ offsets_, const uint32_t* __restrict__ ids_, const uint2* __restrict__ crho_,
    int64_t capacity, const uint8_t* __restrict__ mask_, float a_c, float a_r, int steps, float* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kFilterThreads + threadIdx.x;
  const int64_t pix = t / kLanes;
  const int lane = static_cast<int>(t % kLanes);
  gp<const uint32_t> ids = to_global(ids_);
  gp<const uint2> crho = to_global(crho_);
  gp<const uint8_t> mask = to_global(mask_);
  const PixelSet p = pixel_set(to_global(rgbd_), width, height, f0, n_pix, to_global(offsets_), capacity, pix);
  const int64_t frame_px = static_cast<int64_t>(width) * height;
  // the same decision in all 16 lanes of the group
  const bool run = p.live && !p.bad && p.e > p.s && mask[static_cast<size_t>(p.f) * frame_px + p.self] != 0;
  float sr = p.cr, sg = p.cg, sb = p.cb;
  bool ok = false;
  int bad_id = 0;
  if (run) {
    float ar = 0.f, ag = 0.f, ab = 0.f;
    int64_t i = p.s + lane;
    for (; i + 3 * kLanes < p.e; i += 4 * kLanes) {
      uint2 rec[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) rec[k] = ld2(crho + i + k * kLanes);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ar += h2f(rec[k].x);
        ag += h2f(rec[k].x >> 16);
        ab += h2f(rec[k].y);
      }
    }
    for (; i < p.e; i += kLanes) {
      const uint2 rec = ld2(crho + i);
      ar += h2f(rec.x);
      ag += h2f(rec.x >> 16);
      ab += h2f(rec.y);
    }
    const float inv_n = 1.0f / static_cast<float>(p.e - p.s);
    sr = group_sum(ar) * inv_n;
    sg = group_sum(ag) * inv_n;
    sb = group_sum(ab) * inv_n;
    ok = true;
    const int jbase = p.f - w;
    // 1 when the record's source pixel may contribute (unmasked); 0 when masked, or
    // when the id lies outside the clip (bad_id set, the table not read)
    auto usable = [&](uint32_t id) {
      const int j = jbase + static_cast<int>(id >> SG_ID_SHIFT);
      const int64_t q = static_cast<int64_t>(id & kQMask);
      if (j < 0 || j >= n_frames || q >= frame_px) {
        bad_id = 1;
        return false;
      }
      return mask[static_cast<size_t>(j) * frame_px + q] == 0;
    };
    for (int step = 0; step < steps && ok; ++step) {
      float wsum = 0.f;
      ar = ag = ab = 0.f;
      auto accumulate = [&](uint2 rec, bool use) {
        if (!use) return;
        const float r = h2f(rec.x), g = h2f(rec.x >> 16), b = h2f(rec.y);
        const float er = r - sr, eg = g - sg, eb = b - sb;
        // semi-transparency: the Gaussian around the input pixel (a_r = 0: inpainting alone)
        const float ir = r - p.cr, ig = g - p.cg, ib = b - p.cb;
        const float wt = __builtin_amdgcn_exp2f(
            fmaf(a_r, fmaf(ir, ir, fmaf(ig, ig, ib * ib)), a_c * fmaf(er, er, fmaf(eg, eg, eb * eb))));
        wsum += wt;
        ar = fmaf(wt, r, ar);
        ag = fmaf(wt, g, ag);
        ab = fmaf(wt, b, ab);
      };
      // four records per lane in flight: records and ids, then the source mask bytes
      int64_t i = p.s + lane;
      for (; i + 3 * kLanes < p.e; i += 4 * kLanes) {
        uint2 rec[4];
        uint32_t id[4];
        bool use[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          rec[k] = ld2(crho + i + k * kLanes);
          id[k] = ids[i + k * kLanes];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) use[k] = usable(id[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k) accumulate(rec[k], use[k]);
      }
      for (; i < p.e; i += kLanes) {
        const uint2 rec = ld2(crho + i);
        accumulate(rec, usable(ids[i]));
      }
      wsum = group_sum(wsum);
      ar = group_sum(ar);
      ag = group_sum(ag);
      ab = group_sum(ab);
      if (wsum > 0.f) {
        const float inv = 1.0f / wsum;
        sr = ar * inv;
        sg = ag * inv;
        sb = ab * inv;
      } else {
        ok = false;
      }
    }
    bad_id = group_or(bad_id);
  }
  if (p.live && lane == 0) {
    if (p.bad || bad_id) {
      const float nan = __builtin_nanf("");
      store_rgb(to_global(out), pix, nan, nan, nan);
    } else if (ok) {
      store_rgb(to_global(out), pix, sr, sg, sb);
    } else {
      store_rgb(to_global(out), pix, p.cr, p.cg, p.cb);
    }
  }
}

// ---------------------------------------------------------------------------
// Masks from a scene-space box: one thread per pixel of the clip, float64.

struct WorldBox {
  double lo[3], hi[3];
};

__global__ __launch_bounds__(256) void k_box_mask(const uint16_t* __restrict__ depth_, const double* __restrict__ c2w_,
                                                  int width, int height, int64_t total, double fx, double fy,
                                                  double cx, double cy, WorldBox box, uint8_t* __restrict__ mask) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= total) return;
  const int64_t frame_px = static_cast<int64_t>(width) * height;
  const int j = static_cast<int>(i / frame_px);
  const int64_t self = i - static_cast<int64_t>(j) * frame_px;
  const int y = static_cast<int>(self / width), x = static_cast<int>(self - static_cast<int64_t>(y) * width);
  const int pw = stored_pitch(width);
  const double d = static_cast<double>(
      h2f(to_global(depth_)[static_cast<size_t>(j) * depth_plane_elems(width, height) + depth_index(x, y, pw)]));
  uint8_t m = 0;
  if (d > 0.0 && d < INFINITY) {  // NaN fails both
    const double xc = d * ((static_cast<double>(x) - cx) / fx);
    const double yc = d * ((static_cast<double>(y) - cy) / fy);
    const double zc = d;
    gp<const double> c = to_global(c2w_) + static_cast<size_t>(j) * 16;
    bool in = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double v = ((c[4 * k] * xc + c[4 * k + 1] * yc) + c[4 * k + 2] * zc) + c[4 * k + 3];
      in = in && v >= box.lo[k] && v <= box.hi[k];
    }
    m = in ? 1 : 0;
  }
  to_global(mask)[i] = m;
}

// Workgroups of a 16-lanes-per-pixel launch over n_pix pixels (0 when it would not
// fit a 32-bit grid).
int64_t filter_blocks(int64_t n_pix) {
  const int64_t b = (n_pix * kLanes + kFilterThreads - 1) / kFilterThreads;
  return b > 0x7FFFFFFF ? 0 : b;
}

// The checks shared by the two set filters.
sg_status check_sets_call(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window, const sg_sample_sets* sets,
                          const void* table, const float* out_rgb) {
  sg_status s = check_clip(clip, false);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if (window < 0) return SG_E_INVALID;
  if (window > SG_MAX_WINDOW) return SG_E_UNSUPPORTED;
  if (sets == nullptr || sets->offsets == nullptr || table == nullptr || out_rgb == nullptr) return SG_E_INVALID;
  if (sets->capacity < 0 || (sets->capacity > 0 && (sets->crho == nullptr || sets->ids == nullptr)))
    return SG_E_INVALID;
  if (filter_blocks(static_cast<int64_t>(f1 - f0) * clip->width * clip->height) == 0) return SG_E_UNSUPPORTED;
  return SG_OK;
}

}  // namespace
}  // namespace sg

using sg::check_clip;
using sg::hip_status;

extern "C" {

sg_status scene_frame_sharpness(const sg_clip* clip, float* out_b, void* stream) {
  const sg_status s = check_clip(clip, false);
  if (s != SG_OK) return s;
  if (out_b == nullptr) return SG_E_INVALID;
  hipLaunchKernelGGL(sg::k_frame_sharpness, dim3(static_cast<unsigned>(clip->num_frames)), dim3(sg::kSharpThreads),
                     0, static_cast<hipStream_t>(stream), reinterpret_cast<const uint2*>(clip->rgbd), clip->width,
                     clip->height, out_b);
  return hip_status(hipGetLastError());
}

sg_status scene_filter_frames(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                              const sg_sample_sets* sets, const sg_filter_params* params, const float* frame_w,
                              float* out_rgb, void* stream) {
  sg_status s = sg::check_sets_call(clip, f0, f1, window, sets, frame_w, out_rgb);
  if (s != SG_OK) return s;
  if (params == nullptr) return SG_E_INVALID;
  sg::FilterJob fj{};
  if ((s = sg::filter_scales(params, &fj)) != SG_OK) return s;
  const int64_t n_pix = static_cast<int64_t>(f1 - f0) * clip->width * clip->height;
  const dim3 g(static_cast<unsigned>(sg::filter_blocks(n_pix)));
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const uint2* rgbd = reinterpret_cast<const uint2*>(clip->rgbd);
  const uint2* crho = reinterpret_cast<const uint2*>(sets->crho);
#define SG_FRAMES(C, T)                                                                                          \
  hipLaunchKernelGGL((sg::k_filter_frames<C, T>), g, dim3(sg::kFilterThreads), 0, st, rgbd, clip->width,         \
                     clip->height, clip->num_frames, f0, window, n_pix, sets->offsets, sets->ids, crho,           \
                     sets->capacity, fj.a_d, fj.a_c, fj.a_t, frame_w, out_rgb)
  if (fj.use_colour && fj.use_time)
    SG_FRAMES(true, true);
  else if (fj.use_colour)
    SG_FRAMES(true, false);
  else if (fj.use_time)
    SG_FRAMES(false, true);
  else
    SG_FRAMES(false, false);
#undef SG_FRAMES
  return hip_status(hipGetLastError());
}

static sg_status inpaint_call(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window, const sg_sample_sets* sets,
                              const uint8_t* mask, float sigma_rgb, float sigma_ref, int32_t steps, float* out_rgb,
                              void* stream) {
  const sg_status s = sg::check_sets_call(clip, f0, f1, window, sets, mask, out_rgb);
  if (s != SG_OK) return s;
  if (!(sigma_rgb > 0.0f) || !isfinite(sigma_rgb)) return SG_E_INVALID;
  if (!(sigma_ref > 0.0f)) return SG_E_INVALID;  // +INFINITY: no factor around the input pixel
  if (steps < 1) return SG_E_INVALID;
  if (steps > SG_MAX_INPAINT_STEPS) return SG_E_UNSUPPORTED;
  const double log2e = 1.4426950408889634;
  const float a_c = static_cast<float>(-log2e / (2.0 * sigma_rgb * static_cast<double>(sigma_rgb)));
  const float a_r =
      isfinite(sigma_ref) ? static_cast<float>(-log2e / (2.0 * sigma_ref * static_cast<double>(sigma_ref))) : 0.0f;
  const int64_t n_pix = static_cast<int64_t>(f1 - f0) * clip->width * clip->height;
  hipLaunchKernelGGL(sg::k_inpaint, dim3(static_cast<unsigned>(sg::filter_blocks(n_pix))), dim3(sg::kFilterThreads),
                     0, static_cast<hipStream_t>(stream), reinterpret_cast<const uint2*>(clip->rgbd), clip->width,
                     clip->height, clip->num_frames, f0, window, n_pix, sets->offsets, sets->ids,
                     reinterpret_cast<const uint2*>(sets->crho), sets->capacity, mask, a_c, a_r, steps, out_rgb);
  return hip_status(hipGetLastError());
}

sg_status scene_inpaint(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window, const sg_sample_sets* sets,
                        const uint8_t* mask, float sigma_rgb, int32_t steps, float* out_rgb, void* stream) {
  return inpaint_call(clip, f0, f1, window, sets, mask, sigma_rgb, INFINITY, steps, out_rgb, stream);
}

sg_status scene_semi_transparent(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                                 const sg_sample_sets* sets, const uint8_t* mask, float sigma_rgb, float sigma_ref,
                                 int32_t steps, float* out_rgb, void* stream) {
  return inpaint_call(clip, f0, f1, window, sets, mask, sigma_rgb, sigma_ref, steps, out_rgb, stream);
}

sg_status scene_filter_xyz(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* gparams,
                           const sg_sample_sets* sets, const sg_filter_params* params, float sigma_xyz,
                           const float* frame_w, void* workspace, size_t workspace_bytes, float* out_rgb,
                           void* stream) {
  sg_status s = sg::check_clip(clip, true);
  if (s != SG_OK) return s;
  if ((s = sg::check_range(clip, f0, f1)) != SG_OK) return s;
  if ((s = sg::check_params(gparams)) != SG_OK) return s;
  if (sets == nullptr || sets->offsets == nullptr || params == nullptr || out_rgb == nullptr || workspace == nullptr)
    return SG_E_INVALID;
  if (sets->capacity < 0 || (sets->capacity > 0 && (sets->crho == nullptr || sets->ids == nullptr)))
    return SG_E_INVALID;
  if (!(sigma_xyz > 0.0f)) return SG_E_INVALID;  // +INFINITY disables the term
  sg::FilterJob fj{};
  if ((s = sg::filter_scales(params, &fj)) != SG_OK) return s;
  size_t need = 0;
  if ((s = scene_gather_workspace_size(clip, f0, f1, gparams, &need)) != SG_OK) return s;
  if (workspace_bytes < need) return SG_E_INVALID;
  const int64_t n_pix = static_cast<int64_t>(f1 - f0) * clip->width * clip->height;
  if (sg::filter_blocks(n_pix) == 0) return SG_E_UNSUPPORTED;
  // relative maps of every (f, J) pair in the workspace (the gather's pose prep)
  sg::GatherJob jb{};
  jb.width = clip->width;
  jb.height = clip->height;
  jb.n_frames = clip->num_frames;
  jb.f0 = f0;
  jb.n_out = f1 - f0;
  jb.w = gparams->window;
  jb.fx = clip->fx;
  jb.fy = clip->fy;
  jb.cx = clip->cx;
  jb.cy = clip->cy;
  jb.c2w = clip->cam_to_world;
  jb.rel = static_cast<float*>(workspace);
  jb.status = nullptr;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = hip_status(sg::launch_pose_prep(jb, st))) != SG_OK) return s;
  sg::XyzArgs xa{};
  xa.rel = jb.rel;
  xa.depth = clip->depth;
  const double log2e = 1.4426950408889634;
  xa.a_x = isfinite(sigma_xyz) ? static_cast<float>(-log2e / (2.0 * sigma_xyz * static_cast<double>(sigma_xyz))) : 0.0f;
  xa.fx_inv = static_cast<float>(1.0 / clip->fx);
  xa.fy_inv = static_cast<float>(1.0 / clip->fy);
  xa.cx = static_cast<float>(clip->cx);
  xa.cy = static_cast<float>(clip->cy);
  hipLaunchKernelGGL(sg::k_filter_xyz, dim3(static_cast<unsigned>(sg::filter_blocks(n_pix))),
                     dim3(sg::kFilterThreads), 0, st, reinterpret_cast<const uint2*>(clip->rgbd), clip->width,
                     clip->height, clip->num_frames, f0, gparams->window, n_pix, sets->offsets, sets->ids,
                     reinterpret_cast<const uint2*>(sets->crho), sets->capacity, fj.a_d, fj.a_c, fj.a_t, frame_w, xa,
                     out_rgb);
  return hip_status(hipGetLastError());
}

sg_status scene_box_mask(const sg_clip* clip, const double* box, uint8_t* mask, void* stream) {
  const sg_status s = check_clip(clip, true);
  if (s != SG_OK) return s;
  if (box == nullptr || mask == nullptr) return SG_E_INVALID;
  sg::WorldBox b{};
  for (int k = 0; k < 3; ++k) {
    if (!isfinite(box[k]) || !isfinite(box[k + 3])) return SG_E_INVALID;
    b.lo[k] = box[k];
    b.hi[k] = box[k + 3];
  }
  const int64_t total = static_cast<int64_t>(clip->num_frames) * clip->width * clip->height;
  hipLaunchKernelGGL(sg::k_box_mask, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), clip->depth, clip->cam_to_world, clip->width, clip->height,
                     total, clip->fx, clip->fy, clip->cx, clip->cy, b, mask);
  return hip_status(hipGetLastError());
}

}  // extern "C"
