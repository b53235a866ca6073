// C entry points: host-side argument checks (before any GPU work), workspace
// layout, and the enqueue order of the gather/filter kernels.
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "scene_gather.h"
#include "sg_internal.h"
#include "sg_validate.h"

namespace {

using sg::check_clip;
using sg::check_params;
using sg::check_range;
using sg::filter_scales;
using sg::hip_status;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t rel_off, rel_bytes, part_off, part_bytes, total;
};

Layout layout(const sg_clip* c, int32_t f0, int32_t f1, const sg_gather_params* p) {
  Layout l{};
  const size_t n_out = static_cast<size_t>(f1 - f0);
  const size_t n_pix = n_out * static_cast<size_t>(c->width) * static_cast<size_t>(c->height);
  l.rel_off = 0;
  l.rel_bytes = align_up(n_out * (2 * static_cast<size_t>(p->window) + 1) * sg::kRelStride * sizeof(float));
  l.part_off = l.rel_off + l.rel_bytes;
  const size_t nb = (n_pix + sg::kScanTile - 1) / sg::kScanTile;
  l.part_bytes = align_up((nb + 1) * sizeof(int64_t));
  l.total = l.part_off + l.part_bytes;
  return l;
}

sg_status validate(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                   const sg_sample_sets* sets, bool need_arena) {
  sg_status s = check_clip(clip, true);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if ((s = check_params(params)) != SG_OK) return s;
  if (sets == nullptr || sets->offsets == nullptr || sets->status == nullptr) return SG_E_INVALID;
  if (need_arena && (sets->capacity < 0 || (sets->capacity > 0 && (sets->ids == nullptr || sets->crho == nullptr))))
    return SG_E_INVALID;
  return SG_OK;
}

sg_status prepare(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                  sg_sample_sets* sets, void* ws, size_t ws_bytes, bool need_arena,
                  sg::GatherJob* jb) {
  sg_status s = validate(clip, f0, f1, params, sets, need_arena);
  if (s != SG_OK) return s;
  if (ws == nullptr) return SG_E_INVALID;
  const Layout l = layout(clip, f0, f1, params);
  if (ws_bytes < l.total) return SG_E_INVALID;
  char* base = static_cast<char*>(ws);
  jb->width = clip->width;
  jb->height = clip->height;
  jb->n_frames = clip->num_frames;
  jb->f0 = f0;
  jb->n_out = f1 - f0;
  jb->w = params->window;
  jb->radius = params->radius;
  jb->tol = params->tol;
  jb->z_near = params->z_near;
  jb->fx = clip->fx;
  jb->fy = clip->fy;
  jb->cx = clip->cx;
  jb->cy = clip->cy;
  jb->c2w = clip->cam_to_world;
  jb->rgbd = clip->rgbd;
  jb->depth = clip->depth;
  jb->rel = reinterpret_cast<float*>(base + l.rel_off);
  jb->partial = reinterpret_cast<int64_t*>(base + l.part_off);
  jb->offsets = sets->offsets;
  jb->ids = sets->ids;
  jb->crho = sets->crho;
  jb->capacity = sets->capacity;
  jb->status = sets->status;
  return SG_OK;
}

sg_status run_count(const sg::GatherJob& jb, hipStream_t st) {
  sg_status s = hip_status(sg::launch_pose_prep(jb, st));
  if (s != SG_OK) return s;
  if ((s = hip_status(sg::launch_count(jb, st))) != SG_OK) return s;
  const int64_t n = static_cast<int64_t>(jb.n_out) * jb.width * jb.height;
  return hip_status(sg::launch_scan(jb.offsets, n, jb.partial, st));
}

}  // namespace

namespace sg {

sg_status gather_host_checks(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                             const sg_sample_sets* sets, size_t* ws_bytes) {
  const sg_status s = validate(clip, f0, f1, params, sets, true);
  if (s != SG_OK) return s;
  *ws_bytes = layout(clip, f0, f1, params).total;
  return SG_OK;
}

}  // namespace sg

extern "C" {

int32_t sg_version(void) { return SG_VERSION; }

const char* sg_status_string(int32_t status) {
  switch (status) {
    case SG_OK: return "ok";
    case SG_E_INVALID: return "invalid argument";
    case SG_E_CAPACITY: return "sample arena capacity exceeded";
    case SG_E_HIP: return "HIP runtime error";
    case SG_E_UNSUPPORTED: return "outside supported limits";
    default: return "unknown status";
  }
}

sg_status scene_stage(const uint8_t* rgb_u8, const float* depth, int32_t n_frames, int32_t width,
                      int32_t height, uint16_t* rgbd, uint16_t* depth16, void* stream) {
  if (n_frames < 0 || width <= 0 || height <= 0) return SG_E_INVALID;
  if (n_frames > 0 && (rgb_u8 == nullptr || depth == nullptr || rgbd == nullptr || depth16 == nullptr))
    return SG_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(rgbd) & 7u) != 0 || (reinterpret_cast<uintptr_t>(depth16) & 3u) != 0)
    return SG_E_INVALID;
  if (static_cast<int64_t>(width) * height > SG_MAX_PIXELS_PER_FRAME) return SG_E_UNSUPPORTED;
  if (n_frames > 65535) return SG_E_UNSUPPORTED;
  return hip_status(sg::launch_stage(rgb_u8, depth, n_frames, width, height, rgbd, depth16,
                                     static_cast<hipStream_t>(stream)));
}

sg_status scene_gather_workspace_size(const sg_clip* clip, int32_t f0, int32_t f1,
                                      const sg_gather_params* params, size_t* bytes) {
  if (bytes == nullptr) return SG_E_INVALID;
  sg_status s = check_clip(clip, false);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if ((s = check_params(params)) != SG_OK) return s;
  *bytes = layout(clip, f0, f1, params).total;
  return SG_OK;
}

sg_status scene_gather_count(const sg_clip* clip, int32_t f0, int32_t f1,
                             const sg_gather_params* params, sg_sample_sets* sets, void* workspace,
                             size_t workspace_bytes, void* stream) {
  sg::GatherJob jb{};
  sg_status s = prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, false, &jb);
  if (s != SG_OK) return s;
  return run_count(jb, static_cast<hipStream_t>(stream));
}

sg_status scene_gather_scatter(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, sg_sample_sets* sets,
                               void* workspace, size_t workspace_bytes, void* stream) {
  sg::GatherJob jb{};
  sg_status s = prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, true, &jb);
  if (s != SG_OK) return s;
  return hip_status(sg::launch_scatter(jb, static_cast<hipStream_t>(stream)));
}

sg_status scene_gather(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                       sg_sample_sets* sets, void* workspace, size_t workspace_bytes,
                       void* stream) {
  sg::GatherJob jb{};
  sg_status s = prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, true, &jb);
  if (s != SG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = run_count(jb, st)) != SG_OK) return s;
  return hip_status(sg::launch_scatter(jb, st));
}

sg_status scene_filter(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                       const sg_sample_sets* sets, const sg_filter_params* params, float* out_rgb,
                       void* stream) {
  sg_status s = check_clip(clip, false);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if (window < 0) return SG_E_INVALID;
  if (window > SG_MAX_WINDOW) return SG_E_UNSUPPORTED;
  if (sets == nullptr || sets->offsets == nullptr || params == nullptr || out_rgb == nullptr)
    return SG_E_INVALID;
  sg::FilterJob fj{};
  if ((s = filter_scales(params, &fj)) != SG_OK) return s;
  if (sets->capacity < 0 || (sets->capacity > 0 && sets->crho == nullptr)) return SG_E_INVALID;
  if (fj.use_time && sets->capacity > 0 && sets->ids == nullptr) return SG_E_INVALID;
  fj.width = clip->width;
  fj.height = clip->height;
  fj.f0 = f0;
  fj.w = window;
  fj.n_pix = static_cast<int64_t>(f1 - f0) * clip->width * clip->height;
  fj.rgbd = clip->rgbd;
  fj.offsets = sets->offsets;
  fj.ids = sets->ids;
  fj.crho = sets->crho;
  fj.capacity = sets->capacity;
  fj.out = out_rgb;
  return hip_status(sg::launch_filter(fj, static_cast<hipStream_t>(stream)));
}

sg_status scene_gather_filter(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                              const sg_filter_params* fparams, float* out_rgb, void* workspace,
                              size_t workspace_bytes, void* stream) {
  sg_status s = check_clip(clip, true);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if ((s = check_params(params)) != SG_OK) return s;
  if (fparams == nullptr || out_rgb == nullptr || workspace == nullptr) return SG_E_INVALID;
  sg::FilterJob fj{};
  if ((s = filter_scales(fparams, &fj)) != SG_OK) return s;
  const Layout l = layout(clip, f0, f1, params);
  if (workspace_bytes < l.total) return SG_E_INVALID;
  sg::GatherJob jb{};
  jb.width = clip->width;
  jb.height = clip->height;
  jb.n_frames = clip->num_frames;
  jb.f0 = f0;
  jb.n_out = f1 - f0;
  jb.w = params->window;
  jb.radius = params->radius;
  jb.tol = params->tol;
  jb.z_near = params->z_near;
  jb.fx = clip->fx;
  jb.fy = clip->fy;
  jb.cx = clip->cx;
  jb.cy = clip->cy;
  jb.c2w = clip->cam_to_world;
  jb.rgbd = clip->rgbd;
  jb.depth = clip->depth;
  jb.rel = reinterpret_cast<float*>(static_cast<char*>(workspace) + l.rel_off);
  fj.out = out_rgb;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = hip_status(sg::launch_pose_prep(jb, st))) != SG_OK) return s;
  return hip_status(sg::launch_gather_filter(jb, fj, st));
}

static sg_status learned_prepare(const sg_clip* clip, int32_t f0, int32_t f1,
                                 const sg_gather_params* params, const sg_sample_sets* sets,
                                 void* ws, size_t ws_bytes, sg::GatherJob* jb, sg::LearnedJob* lj) {
  sg_status s = check_clip(clip, true);
  if (s != SG_OK) return s;
  if ((s = check_range(clip, f0, f1)) != SG_OK) return s;
  if ((s = check_params(params)) != SG_OK) return s;
  if (sets == nullptr || sets->offsets == nullptr || sets->capacity < 0) return SG_E_INVALID;
  if (sets->capacity > 0 && (sets->ids == nullptr || sets->crho == nullptr)) return SG_E_INVALID;
  if (ws == nullptr) return SG_E_INVALID;
  const Layout l = layout(clip, f0, f1, params);
  if (ws_bytes < l.total) return SG_E_INVALID;
  char* base = static_cast<char*>(ws);
  *jb = sg::GatherJob{};
  jb->width = clip->width;
  jb->height = clip->height;
  jb->n_frames = clip->num_frames;
  jb->f0 = f0;
  jb->n_out = f1 - f0;
  jb->w = params->window;
  jb->fx = clip->fx;
  jb->fy = clip->fy;
  jb->cx = clip->cx;
  jb->cy = clip->cy;
  jb->c2w = clip->cam_to_world;
  jb->rel = reinterpret_cast<float*>(base + l.rel_off);
  jb->status = nullptr;
  *lj = sg::LearnedJob{};
  lj->width = clip->width;
  lj->height = clip->height;
  lj->n_frames = clip->num_frames;
  lj->f0 = f0;
  lj->w = params->window;
  lj->n_pix = static_cast<int64_t>(f1 - f0) * clip->width * clip->height;
  const double side = 2.0 * params->radius + 1.0;
  lj->log_norm = static_cast<float>(log1p(side * side * (2.0 * params->window + 1.0)));
  lj->fx = clip->fx;
  lj->fy = clip->fy;
  lj->cx = clip->cx;
  lj->cy = clip->cy;
  lj->rgbd = clip->rgbd;
  lj->depth = clip->depth;
  lj->rel = jb->rel;
  lj->offsets = sets->offsets;
  lj->ids = sets->ids;
  lj->crho = sets->crho;
  lj->capacity = sets->capacity;
  return SG_OK;
}

sg_status scene_filter_learned(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, const sg_sample_sets* sets,
                               const sg_mlp* mlp, void* workspace, size_t workspace_bytes,
                               float* out_rgb, void* stream) {
  sg::GatherJob jb;
  sg::LearnedJob lj;
  sg_status s = learned_prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, &jb, &lj);
  if (s != SG_OK) return s;
  if (mlp == nullptr || mlp->w == nullptr || mlp->b == nullptr || out_rgb == nullptr) return SG_E_INVALID;
  lj.mw = mlp->w;
  lj.mb = mlp->b;
  lj.out = out_rgb;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = hip_status(sg::launch_pose_prep(jb, st))) != SG_OK) return s;
  return hip_status(sg::launch_filter_learned(lj, st));
}

sg_status scene_mlp_train_step(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, const sg_sample_sets* sets,
                               const int32_t* pixel_idx, int32_t n_pix, const float* clean_rgb,
                               sg_mlp_train* state, float lr, int32_t t, void* workspace,
                               size_t workspace_bytes, void* stream) {
  sg::GatherJob jb;
  sg::LearnedJob lj;
  sg_status s = learned_prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, &jb, &lj);
  if (s != SG_OK) return s;
  if (state == nullptr || state->master == nullptr || state->adam_m == nullptr ||
      state->adam_v == nullptr || state->grad == nullptr || state->w_bf16 == nullptr ||
      state->b_f32 == nullptr || state->loss == nullptr)
    return SG_E_INVALID;
  if (n_pix < 0 || (n_pix > 0 && (pixel_idx == nullptr || clean_rgb == nullptr))) return SG_E_INVALID;
  if (t < 1 || !(lr > 0.0f) || !isfinite(lr)) return SG_E_INVALID;
  sg::TrainJob tj{};
  tj.pixel_idx = pixel_idx;
  tj.n_pix = n_pix;
  tj.clean = clean_rgb;
  tj.master = state->master;
  tj.adam_m = state->adam_m;
  tj.adam_v = state->adam_v;
  tj.grad = state->grad;
  tj.w_bf16 = state->w_bf16;
  tj.b_f32 = state->b_f32;
  tj.loss = state->loss;
  tj.lr = lr;
  tj.t = t;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = hip_status(sg::launch_pose_prep(jb, st))) != SG_OK) return s;
  return hip_status(sg::launch_mlp_train(lj, tj, st));
}

sg_status scene_feature_moments(const sg_clip* clip, int32_t f0, int32_t f1,
                                const sg_gather_params* params, const sg_sample_sets* sets,
                                const int32_t* pixel_idx, int32_t n_pix, double* moments,
                                void* workspace, size_t workspace_bytes, void* stream) {
  sg::GatherJob jb;
  sg::LearnedJob lj;
  sg_status s = learned_prepare(clip, f0, f1, params, sets, workspace, workspace_bytes, &jb, &lj);
  if (s != SG_OK) return s;
  if (n_pix < 0 || moments == nullptr || (n_pix > 0 && pixel_idx == nullptr)) return SG_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = hip_status(sg::launch_pose_prep(jb, st))) != SG_OK) return s;
  return hip_status(sg::launch_feature_moments(lj, pixel_idx, n_pix, moments, st));
}

sg_status scene_mlp_standardise(const double* moments, float* mlp_b, void* stream) {
  if (moments == nullptr || mlp_b == nullptr) return SG_E_INVALID;
  return hip_status(sg::launch_standardise(moments, mlp_b, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
