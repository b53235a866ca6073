/* scene_frustum.h -- the depth-agnostic frustum gather (HIP, gfx950).
 *
 * Klose et al., Sampling Based Scene-Space Video Processing, Sec. 4, Eq. 1-2:
 * output pixel p of frame f defines the frustum V of a pixel-sized square of side
 * l (the paper uses l = 3) between the depths near and far (0.01 and 1000); a pixel
 * q of a window frame J with stored depth D^J(q) is a member of S(p) when its
 * scene point, carried into the output view (p', z'), satisfies
 *   near <= z' <= far   and   |p_x - p'_x| + |p_y - p'_y| < l / 2   (Eq. 2).
 * The depth of p plays no part in membership: a set holds every observation along
 * p's ray (occluders and occluded points included), a few hundred per pixel.
 *
 * The sets use the sg_sample_sets layout of scene_gather.h for ONE output frame
 * (P = W * H pixels, offsets [P + 1]), so the filters of scene_gather.h and
 * scene_filters.h reduce them unchanged: id = ((J - f + w) << 22) | q, records in
 * ascending id, crho = (r, g, b, rho) with rho = (z' - d_p) / d_p (the member's
 * offset along p's ray from p's own scene point; NaN when p has no valid depth).
 *
 * Conventions as in scene_gather.h: device buffers are caller-owned and borrowed
 * on `stream`; host checks return SG_E_INVALID / SG_E_UNSUPPORTED before any GPU
 * work; kernel-side conditions set sets->status bits. Arithmetic: the relative
 * pose (C^f)^-1 C^J in float64, folded with the intrinsics and rounded to float32;
 * carrying and the membership test in float32.
 */
#ifndef SCENE_FRUSTUM_H
#define SCENE_FRUSTUM_H

#include "scene_gather.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SG_MAX_FRUSTUM_L 7.0f

/* window: w >= 0, J in [max(0, f - w), min(N - 1, f + w)] (<= SG_MAX_WINDOW);
 * l: frustum side in pixels, 0 < l <= SG_MAX_FRUSTUM_L; 0 < near_z < far_z, finite. */
typedef struct sg_frustum_params {
  int32_t window;
  float l;
  float near_z;
  float far_z;
} sg_frustum_params;

/* Bytes of device workspace for output frame f: per window frame, every pixel's
 * bucket and slot (8 B), bucket counter (4 B), filed record (32 B: carried
 * position and depth, pixel index, stored colour) and its position again (8 B,
 * the count pass's copy), and the bucket grid's offsets. */
sg_status scene_frustum_workspace_size(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                                       size_t* bytes);

/* Pass 1: carry every pixel of every window frame into the output view, bucket
 * them by nearest output pixel (each filed with its stored colour), count each
 * output pixel's members and scan the counts into sets->offsets (total at
 * offsets[P]). Clears *sets->status (as scene_gather_count does). Needs
 * clip->depth and clip->rgbd. */
sg_status scene_frustum_count(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                              sg_sample_sets* sets, void* workspace, size_t workspace_bytes, void* stream);

/* Pass 2: write each member's record at its CSR slot (ascending id). Needs the
 * offsets and the workspace left by scene_frustum_count with identical arguments
 * (the colours come from the workspace) and clip->depth.
 * A pixel whose records would pass `capacity` writes none and sets
 * SG_FLAG_CAPACITY; a count that differs from pass 1 sets SG_FLAG_INCONSISTENT. */
sg_status scene_frustum_scatter(const sg_clip* clip, int32_t f, const sg_frustum_params* params,
                                sg_sample_sets* sets, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SCENE_FRUSTUM_H */
