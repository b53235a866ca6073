/* scene_depth.h -- data-term-only multi-view depth (HIP, gfx950).
 *
 * Klose et al., Sampling Based Scene-Space Video Processing, Sec. 3
 * (preprocessing): for each pixel p of frame f, search along the epipolar lines of
 * the frames of a temporal window and keep the depth of lowest mean cost, the cost
 * being the sum of squared RGB differences over 3x3 patches; no smoothness term.
 * Here the search runs over a caller-given list of depth hypotheses: for each
 * hypothesis d, p's scene point d K^-1 (p_x, p_y, 1) in camera f is projected into
 * every window frame J != f and rounded to the nearest pixel q_J; J counts when the
 * point is in front of it and both patches (around p and q_J) lie inside the image;
 * cost(d) = the mean over the counted frames of the patch SSD of the stored
 * binary16 colours; D(p) = the hypothesis of least cost, the lowest index on ties.
 * A pixel on the image border (no full patch) or with no counted frame for any
 * hypothesis gets NaN depth and +INFINITY cost; hypotheses that are not finite and
 * positive are skipped. Relative poses in float64 folded to float32, projection
 * and costs in float32.
 *
 * Conventions as in scene_gather.h: device buffers caller-owned, borrowed on
 * `stream`; host checks before any GPU work.
 */
#ifndef SCENE_DEPTH_H
#define SCENE_DEPTH_H

#include "scene_gather.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SG_MAX_DEPTH_HYPOTHESES 4096

/* Bytes of device workspace (the relative pose maps of the window). */
sg_status scene_depth_workspace_size(const sg_clip* clip, int32_t f, int32_t window, size_t* bytes);

/* hypotheses: device [n_hyp] float32, 1 <= n_hyp <= SG_MAX_DEPTH_HYPOTHESES (their
 * values are the caller's: not read on the host). out_depth: device [H][W]
 * float32; out_cost: device [H][W] float32 or NULL. 0 <= window <= SG_MAX_WINDOW. */
sg_status scene_estimate_depth(const sg_clip* clip, int32_t f, int32_t window, const float* hypotheses,
                               int32_t n_hyp, float* out_depth, float* out_cost, void* workspace,
                               size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SCENE_DEPTH_H */
