// Host-side argument checks shared by the C entry points (no GPU work).
#ifndef SG_VALIDATE_H
#define SG_VALIDATE_H

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "scene_gather.h"
#include "sg_internal.h"

namespace sg {

inline bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

inline sg_status check_clip(const sg_clip* c, bool need_depth) {
  if (c == nullptr) return SG_E_INVALID;
  if (c->width <= 0 || c->height <= 0 || c->num_frames <= 0) return SG_E_INVALID;
  if (c->rgbd == nullptr || c->cam_to_world == nullptr) return SG_E_INVALID;
  if (need_depth && c->depth == nullptr) return SG_E_INVALID;
  // the gather reads rgbd as 8-byte pixels and the depth plane as 32-bit row pairs
  if ((reinterpret_cast<uintptr_t>(c->rgbd) & 7u) != 0 || (reinterpret_cast<uintptr_t>(c->depth) & 3u) != 0)
    return SG_E_INVALID;
  if (!isfinite(c->fx) || !isfinite(c->fy) || c->fx == 0.0 || c->fy == 0.0) return SG_E_INVALID;
  if (!isfinite(c->cx) || !isfinite(c->cy)) return SG_E_INVALID;
  if (static_cast<int64_t>(c->width) * c->height > SG_MAX_PIXELS_PER_FRAME) return SG_E_UNSUPPORTED;
  if (c->num_frames > 65535) return SG_E_UNSUPPORTED;
  return SG_OK;
}

// Workgroups of one gather launch over n_out output frames with tw x th tiles.
inline int64_t gather_tiles(const sg_clip* c, int64_t n_out, int tw, int th) {
  return n_out * ((c->width + tw - 1) / tw) * ((c->height + th - 1) / th);
}

inline sg_status check_range(const sg_clip* c, int32_t f0, int32_t f1) {
  if (f0 < 0 || f1 <= f0 || f1 > c->num_frames) return SG_E_INVALID;
  // the kernels index their 1-D grid with int
  if (gather_tiles(c, f1 - f0, kTileW, kTileH) > INT32_MAX || gather_tiles(c, f1 - f0, kFuseW, kFuseH) > INT32_MAX)
    return SG_E_UNSUPPORTED;
  return SG_OK;
}

inline sg_status check_params(const sg_gather_params* p) {
  if (p == nullptr) return SG_E_INVALID;
  if (p->window < 0 || p->radius < 0) return SG_E_INVALID;
  if (!finite_pos(p->tol) || !finite_pos(p->z_near)) return SG_E_INVALID;
  if (p->window > SG_MAX_WINDOW || p->radius > SG_MAX_RADIUS) return SG_E_UNSUPPORTED;
  return SG_OK;
}

// Filter weights as exp2 arguments: a = -log2(e) / (2 sigma^2); each sigma must be
// > 0 (+inf allowed, disabling its term).
inline sg_status filter_scales(const sg_filter_params* params, sg::FilterJob* fj) {
  const float sd = params->sigma_d, sc = params->sigma_c, stt = params->sigma_t;
  if (!(sd > 0.0f) || !(sc > 0.0f) || !(stt > 0.0f)) return SG_E_INVALID;
  const bool use_c = isfinite(sc), use_t = isfinite(stt);
  const double log2e = 1.4426950408889634;
  fj->a_d = isfinite(sd) ? static_cast<float>(-log2e / (2.0 * sd * static_cast<double>(sd))) : 0.0f;
  fj->a_c = use_c ? static_cast<float>(-log2e / (2.0 * sc * static_cast<double>(sc))) : 0.0f;
  fj->a_t = use_t ? static_cast<float>(-log2e / (2.0 * stt * static_cast<double>(stt))) : 0.0f;
  fj->use_colour = use_c;
  fj->use_time = use_t;
  return SG_OK;
}

inline sg_status hip_status(hipError_t e) { return e == hipSuccess ? SG_OK : SG_E_HIP; }

}  // namespace sg

#endif  // SG_VALIDATE_H
