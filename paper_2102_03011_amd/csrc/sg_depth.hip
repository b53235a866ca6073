// Data-term-only multi-view depth (Sec. 3, preprocessing): per pixel, the depth
// hypothesis of least mean 3x3 RGB patch SSD over the window frames.
// One lane per pixel of frame f: its own patch stays in registers; per hypothesis
// and window frame, one projection through the frame's folded relative pose, a
// nearest-pixel round and nine 8-byte patch reads; a running minimum with a
// strict comparison keeps the lowest index on ties.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "scene_depth.h"
#include "sg_device.h"
#include "sg_validate.h"

namespace sg {
namespace {

constexpr int kMapFloats = 16;  // per window frame: M (3x3, row-major), k (3), padding
constexpr int kThreads = 256;

size_t depth_workspace(const sg_clip* c, int32_t f, int32_t window, int* jlo, int* n_j) {
  const int lo = f - window > 0 ? f - window : 0;
  const int hi = f + window < c->num_frames - 1 ? f + window : c->num_frames - 1;
  if (jlo != nullptr) *jlo = lo;
  if (n_j != nullptr) *n_j = hi - lo + 1;
  return static_cast<size_t>(hi - lo + 1) * kMapFloats * sizeof(float);
}

// T_{J<-f} = (C^J)^-1 C^f in float64 (rigid), folded with K: a point of camera f at
// d K^-1 (x, y, 1) goes to Y = d M (x, y, 1) + k in J's pixel frame. The entry of
// J = f is not used.
__global__ __launch_bounds__(64) void k_depth_pose(const double* __restrict__ c2w, int f, int jlo, int n_j,
                                                   double fx, double fy, double cx, double cy,
                                                   float* __restrict__ maps) {
  for (int jn = threadIdx.x; jn < n_j; jn += 64) {
    const int j = jlo + jn;
    float* m = maps + jn * kMapFloats;
    for (int i = 0; i < kMapFloats; ++i) m[i] = 0.0f;
    const double* a = c2w + static_cast<size_t>(j) * 16;
    const double* b = c2w + static_cast<size_t>(f) * 16;
    double r[3][3], t[3], am[3][3];
    for (int i = 0; i < 3; ++i) {
      for (int k = 0; k < 3; ++k) r[i][k] = a[i] * b[k] + a[4 + i] * b[4 + k] + a[8 + i] * b[8 + k];
      t[i] = a[i] * (b[3] - a[3]) + a[4 + i] * (b[7] - a[7]) + a[8 + i] * (b[11] - a[11]);
    }
    for (int i = 0; i < 3; ++i) {
      am[i][0] = r[i][0] / fx;
      am[i][1] = r[i][1] / fy;
      am[i][2] = r[i][2] - r[i][0] * cx / fx - r[i][1] * cy / fy;
    }
    for (int k = 0; k < 3; ++k) {
      m[k] = static_cast<float>(fx * am[0][k] + cx * am[2][k]);
      m[3 + k] = static_cast<float>(fy * am[1][k] + cy * am[2][k]);
      m[6 + k] = static_cast<float>(am[2][k]);
    }
    m[9] = static_cast<float>(fx * t[0] + cx * t[2]);
    m[10] = static_cast<float>(fy * t[1] + cy * t[2]);
    m[11] = static_cast<float>(t[2]);
  }
}

__global__ __launch_bounds__(kThreads) void k_estimate_depth(const uint2* __restrict__ rgbd_,
                                                             const float* __restrict__ maps,
                                                             const float* __restrict__ hyp_, int n_hyp, int width,
                                                             int height, int f, int jlo, int n_j,
                                                             float* __restrict__ out_depth,
                                                             float* __restrict__ out_cost) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (p >= static_cast<int64_t>(width) * height) return;
  const int y = static_cast<int>(p / width), x = static_cast<int>(p - static_cast<int64_t>(y) * width);
  float best = INFINITY, best_d = __builtin_nanf("");
  if (x >= 1 && x <= width - 2 && y >= 1 && y <= height - 2) {
    const int pw = stored_pitch(width);
    const size_t pplane = static_cast<size_t>(pw) * stored_rows(height);
    gp<const uint2> rgbd = to_global(rgbd_);
    gp<const float> hyp = to_global(hyp_);
    float own[9][3];
    uint2 blk[3][3];
    load_block_pixels<1>(rgbd + static_cast<size_t>(f) * pplane, padded_index(x, y, pw), pw, blk);
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const uint2 v = blk[o / 3][o % 3];
      own[o][0] = h2f(v.x);
      own[o][1] = h2f(v.x >> 16);
      own[o][2] = h2f(v.y);
    }
    const float fx = static_cast<float>(x), fy = static_cast<float>(y);
    for (int k = 0; k < n_hyp; ++k) {
      const float d = hyp[k];
      if (!(d > 0.0f && d < INFINITY)) continue;
      float sum = 0.0f;
      int cnt = 0;
      for (int jn = 0; jn < n_j; ++jn) {
        if (jlo + jn == f) continue;
        const float* m = maps + jn * kMapFloats;
        const float y2 = fmaf(d, fmaf(m[6], fx, fmaf(m[7], fy, m[8])), m[11]);
        if (!(y2 > 0.0f)) continue;
        const float u = fmaf(d, fmaf(m[0], fx, fmaf(m[1], fy, m[2])), m[9]) / y2;
        const float v = fmaf(d, fmaf(m[3], fx, fmaf(m[4], fy, m[5])), m[10]) / y2;
        const float eu = u + 0.5f, ev = v + 0.5f;
        // q = floor(u + 1/2) in [1, W - 2] x [1, H - 2]; NaN fails
        if (!(eu >= 1.0f && eu < static_cast<float>(width - 1) && ev >= 1.0f &&
              ev < static_cast<float>(height - 1)))
          continue;
        const int qx = static_cast<int>(floorf(eu)), qy = static_cast<int>(floorf(ev));
        uint2 src[3][3];
        load_block_pixels<1>(rgbd + static_cast<size_t>(jlo + jn) * pplane, padded_index(qx, qy, pw), pw, src);
        float ssd = 0.0f;
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const uint2 w2 = src[o / 3][o % 3];
          const float e0 = own[o][0] - h2f(w2.x), e1 = own[o][1] - h2f(w2.x >> 16), e2 = own[o][2] - h2f(w2.y);
          ssd = fmaf(e0, e0, fmaf(e1, e1, fmaf(e2, e2, ssd)));
        }
        sum += ssd;
        ++cnt;
      }
      if (cnt > 0) {
        const float c = sum / static_cast<float>(cnt);
        if (c < best) {
          best = c;
          best_d = d;
        }
      }
    }
  }
  to_global(out_depth)[p] = best_d;
  if (out_cost != nullptr) to_global(out_cost)[p] = best;
}

sg_status check_depth(const sg_clip* clip, int32_t f, int32_t window) {
  const sg_status s = check_clip(clip, false);
  if (s != SG_OK) return s;
  if (f < 0 || f >= clip->num_frames || window < 0) return SG_E_INVALID;
  if (window > SG_MAX_WINDOW) return SG_E_UNSUPPORTED;
  return SG_OK;
}

}  // namespace
}  // namespace sg

extern "C" {

sg_status scene_depth_workspace_size(const sg_clip* clip, int32_t f, int32_t window, size_t* bytes) {
  const sg_status s = sg::check_depth(clip, f, window);
  if (s != SG_OK) return s;
  if (bytes == nullptr) return SG_E_INVALID;
  *bytes = sg::depth_workspace(clip, f, window, nullptr, nullptr);
  return SG_OK;
}

sg_status scene_estimate_depth(const sg_clip* clip, int32_t f, int32_t window, const float* hypotheses,
                               int32_t n_hyp, float* out_depth, float* out_cost, void* workspace,
                               size_t workspace_bytes, void* stream) {
  const sg_status s = sg::check_depth(clip, f, window);
  if (s != SG_OK) return s;
  if (hypotheses == nullptr || out_depth == nullptr || workspace == nullptr || n_hyp < 1) return SG_E_INVALID;
  if (n_hyp > SG_MAX_DEPTH_HYPOTHESES) return SG_E_UNSUPPORTED;
  int jlo = 0, n_j = 0;
  if (workspace_bytes < sg::depth_workspace(clip, f, window, &jlo, &n_j)) return SG_E_INVALID;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float* maps = static_cast<float*>(workspace);
  hipLaunchKernelGGL(sg::k_depth_pose, dim3(1), dim3(64), 0, st, clip->cam_to_world, f, jlo, n_j, clip->fx, clip->fy,
                     clip->cx, clip->cy, maps);
  const int64_t n_pix = static_cast<int64_t>(clip->width) * clip->height;
  hipLaunchKernelGGL(sg::k_estimate_depth, dim3(static_cast<unsigned>((n_pix + sg::kThreads - 1) / sg::kThreads)),
                     dim3(sg::kThreads), 0, st, reinterpret_cast<const uint2*>(clip->rgbd), maps, hypotheses, n_hyp,
                     clip->width, clip->height, f, jlo, n_j, out_depth, out_cost);
  return sg::hip_status(hipGetLastError());
}

}  // extern "C"
