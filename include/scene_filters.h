/* scene_filters.h -- the paper's other filters over stored sample sets (HIP, gfx950).
 *
 * Klose et al., Sampling Based Scene-Space Video Processing, Sec. 5: deblurring
 * (Eq. 5), computational scene-space shutters (Eq. 10) and inpainting (Eq. 8-9)
 * reduce the same sample sets S(p) as the denoising filter of scene_gather.h with
 * other weights; scene_filter_xyz adds Eq. 4's scene-space term, and
 * scene_semi_transparent the semi-transparency of the inpainting paragraph. The sets, clip and status conventions are those of
 * scene_gather.h: every pointer named "device" is device memory owned by the
 * caller and borrowed for the call on `stream` (a hipStream_t, NULL = the null
 * stream); arguments are checked on the host before any GPU work, and a failed
 * check returns SG_E_INVALID or SG_E_UNSUPPORTED without enqueuing anything; a
 * failing HIP call returns SG_E_HIP. No call allocates device memory.
 */
#ifndef SCENE_FILTERS_H
#define SCENE_FILTERS_H

#include "scene_gather.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SG_MAX_INPAINT_STEPS 16

/* Blurriness measure of Eq. 5 for every frame J of the clip:
 *   B(J) = sum over pixels q of |grad I^J(q)|,
 * from the stored binary16 colours, with forward differences
 * gx = I(x + 1, y) - I(x, y), gy = I(x, y + 1) - I(x, y) per channel and
 * |grad I(q)| = sqrt(sum over r, g, b of gx^2 + gy^2), over the pixels whose right
 * and lower neighbours lie in the image (the paper names the operator only).
 * Magnitudes in float32, sums in float64 in a fixed order (bit-reproducible).
 * out_b: device [num_frames] float32, every entry written.
 * Needs clip->rgbd only (depth, poses and intrinsics are not read but must pass
 * the usual clip checks). */
sg_status scene_frame_sharpness(const sg_clip* clip, float* out_b, void* stream);

/* Filter with a per-source-frame factor (Eq. 3 with the weight of Eq. 4 times
 * frame_w[J], J = the frame the sample came from):
 *   deblurring, Eq. 5: frame_w = B from scene_frame_sharpness, sigmas of Eq. 4;
 *   computational shutter, Eq. 10: frame_w[J] = xi(J), every sigma +INFINITY
 *   (a box, impulse train or decaying tail over absolute frame times).
 * frame_w: device [num_frames] float32, each finite and >= 0 (not checked on the
 * host: the caller's table). Sets, window and out_rgb as for scene_filter, and
 * sets->ids must be non-NULL when capacity > 0. An
 * output pixel whose weights sum to zero (empty set, or every sample on a frame of
 * factor 0) gets I^f(p); a set that did not fit the arena (SG_FLAG_CAPACITY) gets
 * NaN. */
sg_status scene_filter_frames(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                              const sg_sample_sets* sets, const sg_filter_params* params,
                              const float* frame_w, float* out_rgb, void* stream);

/* The full weight of Eq. 4 (Sec. 5, denoising): Eq. 3 with
 *   w(s) = exp(-rho^2 / 2 sigma_d^2) exp(-|c_s - c_ref|^2 / 2 sigma_c^2)
 *          exp(-|X_s - X_ref|^2 / 2 sigma_xyz^2) exp(-(J - f)^2 / 2 sigma_t^2) * frame_w[J]
 * (params->sigma_d, sigma_c, sigma_t as for scene_filter; +INFINITY disables a term).
 * X_s is the sample's scene point (its source pixel q with its stored depth D^J(q) and
 * camera C^J) and X_ref the scene point of the output pixel p (stored depth d_p,
 * camera C^f): the distance is measured in the camera frame of J through the gather's
 * folded relative map, in float32. sigma_xyz > 0 in world units (the paper states
 * its sigma_xyz for a scene scaled so that 90 % of its points lie in a 10^3 cube:
 * the caller converts), +INFINITY disables the term. frame_w: device [num_frames]
 * float32 factors (deblurring, Eq. 5: B(J) from scene_frame_sharpness) or NULL for
 * none. gparams: the gather parameters the sets were gathered with (window decodes
 * J; the relative maps of every (f, J) pair are written into `workspace`, of at
 * least scene_gather_workspace_size(clip, f0, f1, gparams) bytes). Needs clip->depth
 * and the poses. An output pixel without a valid stored depth (not finite, or <= 0)
 * has no reference point: with a finite sigma_xyz it gets I^f(p), as does a set
 * whose weights sum to zero; a set that did not fit the arena, or an id outside the
 * clip, gives NaN. sets->ids must be non-NULL when capacity > 0. */
sg_status scene_filter_xyz(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* gparams,
                           const sg_sample_sets* sets, const sg_filter_params* params, float sigma_xyz,
                           const float* frame_w, void* workspace, size_t workspace_bytes, float* out_rgb,
                           void* stream);

/* Inpainting, Eq. 8-9. mask: device [num_frames][H][W] uint8, nonzero where the
 * pixel shows content to remove (M = 1). For an output pixel with M^f(p) = 1:
 * s_ref starts as the mean colour of all samples of its set (Eq. 8), and each of
 * `steps` steps (the paper uses 2) replaces it with the mean of the samples
 * weighted by exp(-|s_ref - c_s|^2 / (2 sigma_rgb^2)) for samples from unmasked
 * source pixels and 0 for masked ones (Eq. 9; colour dimensions only). The output
 * is the last s_ref. Unmasked output pixels, empty sets and pixels where a step's
 * weights sum to zero get I^f(p); a set that did not fit the arena gets NaN.
 * sigma_rgb > 0 and finite, on the stored colours' scale (full scale 1: the
 * paper's 55 of 255 is 55 / 255 here); 1 <= steps <= SG_MAX_INPAINT_STEPS (more:
 * SG_E_UNSUPPORTED). sets->ids must be non-NULL when capacity > 0. */
sg_status scene_inpaint(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                        const sg_sample_sets* sets, const uint8_t* mask, float sigma_rgb, int32_t steps,
                        float* out_rgb, void* stream);

/* Semi-transparency (Sec. 5, inpainting paragraph: the standard multivariate
 * weighting around the input pixel added to the inpainting weight, sigma_rgb = 80
 * of 255 there): scene_inpaint with every weight of Eq. 9 also multiplied by
 * exp(-|c_s - I^f(p)|^2 / (2 sigma_ref^2)), which favours samples coloured like the
 * object being made transparent. sigma_ref > 0 on the stored colours' scale
 * (+INFINITY gives scene_inpaint exactly); other arguments and results as for
 * scene_inpaint. */
sg_status scene_semi_transparent(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                                 const sg_sample_sets* sets, const uint8_t* mask, float sigma_rgb, float sigma_ref,
                                 int32_t steps, float* out_rgb, void* stream);

/* Inpainting masks from a scene-space region (Sec. 5, inpainting: the samples that
 * fall into the region, projected back into the images, form M). M^J(q) = 1 when
 * the scene point of pixel q = (x, y) of frame J lies in the world-space box
 * [lo, hi] (bounds included), 0 otherwise and for pixels without a valid stored
 * depth d (not finite, or <= 0). Float64, each sum left to right:
 * X_cam = d ((x - cx) / fx, (y - cy) / fy, 1), X = R^J X_cam + t^J with
 * C^J = cam_to_world[J] = [R^J | t^J].
 * box: HOST [6] float64 = (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi), each finite
 * (lo > hi gives an empty mask), read before the call returns.
 * mask: device [num_frames][H][W] uint8, every entry written (0 or 1). */
sg_status scene_box_mask(const sg_clip* clip, const double* box, uint8_t* mask, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SCENE_FILTERS_H */
