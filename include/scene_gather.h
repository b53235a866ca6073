/*
 * scene_gather.h -- C ABI of the MI355X (gfx950) scene-space gather + filter library.
 *
 * Method: Klose, Wang, Bazin, Magnor, Sorkine-Hornung, "Sampling Based
 * Scene-Space Video Processing" (ACM TOG). For every output pixel p of frame f
 * the library gathers a sample set S^f(p) of source pixels from the frames of a
 * temporal window that observe the same scene point (Sec. 4), then reduces each
 * set to an output colour with a weighted mean (Sec. 5, Eq. 3 / Eq. 4).
 *
 * Conventions used by every entry point:
 *   - pixel (x, y): x = column, y = row, pixel centres at integer coordinates;
 *     flat pixel index y * W + x; planes are row-major [frame][row][column];
 *   - intrinsics K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]];
 *   - camera frame x right, y down, z forward; depth is z-depth;
 *   - cam_to_world[f] is the rigid 4x4 camera-to-world matrix C^f (row-major,
 *     float64, last row 0 0 0 1);
 *   - colour is on the 0-1 scale (the paper's 0-255 divided by 255);
 *   - binary16 values are passed as their 16-bit patterns (uint16_t).
 *
 * Memory ownership: every data buffer (planes, poses, sample sets, outputs,
 * workspaces) is allocated by the caller and only borrowed for the duration of the
 * work enqueued on `stream`. The single-clip entry points allocate no device
 * memory. Two exceptions own device memory of their own: a batch
 * (sg_batch_create allocates its plan, relative maps, scan partials, queue
 * counters and a pinned host copy of the step's frames; sg_batch_destroy frees
 * them), and scene_gather_noalloc's static scratch array (SG_NOALLOC_SCRATCH_BYTES
 * per GPU, held until the process ends). `stream` is a hipStream_t (NULL = the
 * default stream); all GPU work is enqueued asynchronously on it.
 *
 * Errors: argument checks run on the host before any GPU work and return
 * synchronously (SG_E_INVALID, SG_E_UNSUPPORTED). A failing HIP call returns
 * SG_E_HIP. Conditions found by kernels (sample arena too small, count/scatter
 * disagreement) are OR-ed into the caller's device status word as SG_FLAG_*
 * bits; read it after synchronising the stream. No C++ exception crosses this
 * interface.
 */
#ifndef SCENE_GATHER_H
#define SCENE_GATHER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_VERSION 1

/* Limits. Sample ids pack (J - f + w) into 10 bits and the source pixel index
 * into 22 bits, so W * H <= 2^22 and 2w + 1 <= 1024. */
#define SG_MAX_PIXELS_PER_FRAME (1 << 22)
/* Stored planes carry an apron: SG_APRON rows above and below the image and
 * SG_APRON columns on its left, SG_APRON_RIGHT columns on its right. A projection
 * is kept when its block centre lies at most r pixels outside the image, so the
 * block reaches 2r beyond it: SG_APRON >= 2 SG_MAX_RADIUS, and so is the right
 * apron (one column wider than it needs to be). */
#define SG_APRON 6
#define SG_APRON_RIGHT 7
#define SG_MAX_WINDOW 511
#define SG_MAX_RADIUS 3
/* One call's output frames f0 .. f1 - 1 are gathered as one launch of workgroups
 * of 256 pixels (64 x 4 tiles, 16 x 16 in scene_gather_filter): the number of
 * tiles, (f1 - f0) ceil(W / 64) ceil(H / 4) and (f1 - f0) ceil(W / 16) ceil(H / 16),
 * must stay below 2^31, else SG_E_UNSUPPORTED (split the range into calls). */
#define SG_ID_SHIFT 22

/* Device status bits (OR-ed into sg_sample_sets.status). */
#define SG_FLAG_CAPACITY 1u      /* a pixel's records would pass `capacity`; its records were not written */
#define SG_FLAG_INCONSISTENT 2u  /* scatter found a different count than the count pass (planes changed?) */

typedef enum sg_status {
  SG_OK = 0,
  SG_E_INVALID = 1,     /* null pointer, size out of range, non-finite parameter, workspace too small */
  SG_E_CAPACITY = 2,    /* reserved for callers mapping SG_FLAG_CAPACITY to a status */
  SG_E_HIP = 3,         /* a HIP runtime call or kernel launch failed */
  SG_E_UNSUPPORTED = 4  /* outside the limits above */
} sg_status;

/* A staged clip: the stored input planes of N frames of W x H pixels, written by
 * scene_stage. Each plane is padded by the apron: stored rows SH = H + 2A, stored
 * row pitch SW = W + A + AR (A = SG_APRON, AR = SG_APRON_RIGHT); image pixel (x, y)
 * sits at stored row y + A, column x + A. Apron pixels hold an invalid depth
 * (binary16 NaN) and zero colour.
 * rgbd : device [N][SH][SW][4] binary16 (r, g, b, z-depth); the 4th channel is the
 *        same binary16 depth as `depth`.
 * depth: device [N][SP][SW][2] binary16 z-depth with stored rows paired, SP =
 *        ceil(SH / 2): entry [n][P][X][s] is stored row 2P + s, column X, so one
 *        32-bit word holds two vertically adjacent depths (the count pass reads a
 *        block of 2r + 1 rows as r + 1 rows of words). With SH odd the last pair's
 *        second row is apron. The pointer must be 4-byte aligned (rgbd: 8-byte).
 * cam_to_world: device [N][4][4] float64.                                    */
typedef struct sg_clip {
  int32_t width;
  int32_t height;
  int32_t num_frames;
  int32_t reserved;
  const uint16_t* rgbd;
  const uint16_t* depth;
  const double* cam_to_world;
  double fx, fy, cx, cy;
} sg_clip;

/* Gather parameters (Sec. 4).
 * window: w >= 0; source frames J in [max(0, f - w), min(N - 1, f + w)], f included.
 * radius: r in [0, SG_MAX_RADIUS]; the l x l block with l = 2r + 1 (the paper uses l = 3).
 * tol   : tau > 0; q is kept when |D^J(q) - z| <= tau * z, z the predicted depth in J.
 * z_near: > 0; output pixels with depth <= z_near (or non-finite) get an empty set,
 *         and frames where the point lies at z <= z_near are skipped (near plane, Sec. 4 Eq. 1). */
typedef struct sg_gather_params {
  int32_t window;
  int32_t radius;
  float tol;
  float z_near;
} sg_gather_params;

/* Sample sets of the P = (f1 - f0) * H * W output pixels of frames [f0, f1), in CSR form.
 * offsets : device [P + 1] int64; the set of output pixel i (i = (f - f0) * H * W + y * W + x)
 *           is records [offsets[i], offsets[i + 1]); offsets[0] = 0, offsets[P] = total.
 * ids     : device [capacity] uint32; id = ((J - f + w) << 22) | (q_y * W + q_x).
 * crho    : device [capacity][4] binary16 (r, g, b, rho), rho = (D^J(q) - z) / z.
 * Within a set, records are in ascending id (J ascending, block row-major).
 * status  : device uint32 word; scene_gather_count clears it, kernels OR SG_FLAG_* bits. */
typedef struct sg_sample_sets {
  int64_t* offsets;
  uint32_t* ids;
  uint16_t* crho;
  int64_t capacity;
  uint32_t* status;
} sg_sample_sets;

/* Filter weights (Sec. 5 Eq. 4, diagonal Gaussian around the reference sample):
 * w(s) = exp(-rho^2 / 2 sigma_d^2) * exp(-|c_s - c_ref|^2 / 2 sigma_c^2) * exp(-(J - f)^2 / 2 sigma_t^2),
 * c_ref = I^f(p). A sigma of +INFINITY disables its term. */
typedef struct sg_filter_params {
  float sigma_d;
  float sigma_c;
  float sigma_t;
  float reserved;
} sg_filter_params;

/* Library version (SG_VERSION). */
int32_t sg_version(void);

/* Human-readable name of a status code (static string). */
const char* sg_status_string(int32_t status);

/* Stage the stored input planes of n_frames frames (Sec. 3: the colour of each
 * pixel and its depth D^f(p) are the inputs of sampling).
 * rgb_u8  : device [n_frames][H][W][3] uint8 colour on the 0-255 scale.
 * depth   : device [n_frames][H][W] float32 z-depth.
 * rgbd    : device [n_frames][SH][SW][4] binary16 out: (c/255, c/255, c/255, depth),
 *           each rounded to nearest even; stored geometry and apron as at sg_clip.
 * depth16 : device [n_frames][SP][SW][2] binary16 out: depth (inf above 65504), stored
 *           rows paired as at sg_clip (4-byte aligned; rgbd 8-byte aligned).
 * n_frames >= 0 (0 enqueues nothing); W, H > 0 with W * H <= SG_MAX_PIXELS_PER_FRAME. */
sg_status scene_stage(const uint8_t* rgb_u8, const float* depth, int32_t n_frames,
                      int32_t width, int32_t height, uint16_t* rgbd, uint16_t* depth16,
                      void* stream);

/* Workspace bytes needed by scene_gather_count / scene_gather_scatter / scene_gather
 * for output frames [f0, f1): relative camera maps for every (f, J) pair plus scan
 * partials. Pure host computation. */
sg_status scene_gather_workspace_size(const sg_clip* clip, int32_t f0, int32_t f1,
                                      const sg_gather_params* params, size_t* bytes);

/* Gather pass 1 (Sec. 4, parallel over output pixels): computes, in float64 on the
 * device, T_{J<-f} = (C^J)^{-1} C^f for every (f, J) pair (exact identity for J = f),
 * folds it with K into float32 maps M = K R K^{-1}, k = K t kept in `workspace`,
 * counts each output pixel's members, and scans the counts into sets->offsets.
 * Clears *sets->status. The total is sets->offsets[P] on the device; a caller may
 * synchronise and read it to size the arena. ids/crho/capacity are not used. */
sg_status scene_gather_count(const sg_clip* clip, int32_t f0, int32_t f1,
                             const sg_gather_params* params, sg_sample_sets* sets,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Gather pass 2: same traversal as pass 1 (same arithmetic, bit for bit), writing
 * each member's record at its CSR slot. Needs the offsets and the workspace left by
 * scene_gather_count with identical arguments. A pixel whose records would pass
 * `capacity` writes none and sets SG_FLAG_CAPACITY. */
sg_status scene_gather_scatter(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, sg_sample_sets* sets,
                               void* workspace, size_t workspace_bytes, void* stream);

/* scene_gather_count followed by scene_gather_scatter, enqueued without any host
 * synchronisation (the caller sizes `capacity` in advance). */
sg_status scene_gather(const sg_clip* clip, int32_t f0, int32_t f1,
                       const sg_gather_params* params, sg_sample_sets* sets,
                       void* workspace, size_t workspace_bytes, void* stream);

/* scene_gather without a caller workspace and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc). The workspace is a library-owned static device
 * array of SG_NOALLOC_SCRATCH_BYTES bytes; each GPU the library runs on holds its
 * own copy until the process ends (its address is looked up on the first call on
 * that GPU: the GPU of `stream`). Results are identical to scene_gather's with the
 * same arguments. Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams, or different host threads) race and give wrong
 * sets; serialise them. Nothing in the array needs clearing between calls.
 * SG_E_UNSUPPORTED when the call's workspace (scene_gather_workspace_size) exceeds
 * SG_NOALLOC_SCRATCH_BYTES (split [f0, f1) into calls); other errors as scene_gather. */
#define SG_NOALLOC_SCRATCH_BYTES (4u << 20)
sg_status scene_gather_noalloc(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, sg_sample_sets* sets, void* stream);

/* Filter (Sec. 5 Eq. 3 with the weight above): out_rgb device [P][3] float32 with
 * O(p) = sum w(s) c_s / sum w(s) over the set of p, or I^f(p) (the stored colour of
 * the output pixel) when the set is empty. `window` must be the w used to gather
 * (it decodes J - f from the ids). Records are read only below sets->capacity: a
 * pixel whose set did not fit the arena (SG_FLAG_CAPACITY) gets NaN. */
sg_status scene_filter(const sg_clip* clip, int32_t f0, int32_t f1, int32_t window,
                       const sg_sample_sets* sets, const sg_filter_params* params,
                       float* out_rgb, void* stream);

/* Gather + filter in one pass, without storing the sets (the paper's own flow,
 * Sec. 4-5: samples are weighted as they are found). For output frames [f0, f1):
 * the same projection, block and membership test as scene_gather, each member
 * weighted as scene_filter weights its record (rho rounded to binary16 as a
 * record stores it), so out_rgb (device [P][3] float32) equals scene_gather +
 * scene_filter up to the order of the float32 additions; an empty set gives I^f(p).
 * workspace: as for scene_gather (only the relative maps are written). */
sg_status scene_gather_filter(const sg_clip* clip, int32_t f0, int32_t f1,
                              const sg_gather_params* params, const sg_filter_params* fparams,
                              float* out_rgb, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learned per-sample weights (replacing the hand-set weight of Sec. 5 Eq. 4 in
 * the weighted mean of Sec. 5 Eq. 3): O(p) = sum_s softmax(m)_s c_s over the set of
 * p, m_s = MLP(standardised features of s), MLP 8 -> 64 -> 64 -> 1 with GELU.
 * Features of a sample (source frame J, source pixel q) of output pixel p, frame f:
 *   1 rho; 2 |c - lower median of the set|_2 (per channel); 3 |J - f| / w;
 *   4 |q - (u, v)|_2 with (u, v) the unrounded projection in J; 5 1 - cosine of the
 *   angle at the scene point between the rays from the camera centres of f and J;
 *   6 |grad D^J|(q) / D^J(q) (central differences, one-sided where a neighbour has
 *   no valid depth); 7 log(1 + n) / log(1 + (2r + 1)^2 (2w + 1)); 8 (J - f) / w.
 * GELU is the exact form GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (Phi the
 * standard normal CDF; not the tanh approximation); the learned filter evaluates
 * it from a table of chords over z in [-8, 8) (cells of width 1/64, continued as
 * z above the range and 0 below; |error| <= 2.5e-5; built in each workgroup from
 * erff), the training step
 * with Abramowitz-Stegun 7.1.28 for erf (|error| <= 3e-7). Matrix operands (standardised
 * features, hidden activations) are bfloat16 hi/lo pairs, products accumulate in
 * float32 on the matrix cores.
 *
 * Parameter layout (device):
 *   w : bfloat16 [SG_MLP_NW] = W1 [8][64] (feature, hidden), W2 [64][64] (in, out), W3 [64]
 *   b : float32  [SG_MLP_NB] = b1 [64], b2 [64], b3, 3 unused, feature mean [8],
 *       feature 1/std [8].                                                      */
#define SG_MLP_NW (8 * 64 + 64 * 64 + 64)
#define SG_MLP_NB (64 + 64 + 4 + 8 + 8)
/* trainable parameters in float32 master order: W1, W2, W3, b1, b2, b3 */
#define SG_MLP_NPARAM (SG_MLP_NW + 64 + 64 + 1)

typedef struct sg_mlp {
  const uint16_t* w;
  const float* b;
} sg_mlp;

/* Learned filter. Same sets, geometry and workspace contract as the gather of
 * [f0, f1) with `params` (the workspace's relative maps are recomputed here).
 * out_rgb device [P][3] float32; an empty set gives I^f(p); a set that did not fit
 * the arena gives NaN. */
sg_status scene_filter_learned(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, const sg_sample_sets* sets,
                               const sg_mlp* mlp, void* workspace, size_t workspace_bytes,
                               float* out_rgb, void* stream);

/* Training state (device, caller-owned).
 *   master : float32 [SG_MLP_NPARAM] parameters; adam_m, adam_v : same size;
 *   grad   : float32 [SG_MLP_NPARAM] accumulator (cleared by the step);
 *   w_bf16 : the step writes the bfloat16 forward copy of W1, W2, W3 here;
 *   b_f32  : [SG_MLP_NB]; the step writes b1, b2, b3, reads the feature mean / 1/std;
 *   loss   : float32 [1], the step's loss L = sum_p |O(p) - G(p)|^2 / (3 n_pix).    */
typedef struct sg_mlp_train {
  float* master;
  float* adam_m;
  float* adam_v;
  float* grad;
  uint16_t* w_bf16;
  float* b_f32;
  float* loss;
} sg_mlp_train;

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr, step number
 * t >= 1) on the loss over the sets of the n_pix output pixels pixel_idx (device
 * int32, indices into [0, P)); clean_rgb device [n_pix][3] float32 is the ground
 * truth G of those pixels, row i for pixel_idx[i]. An index outside [0, P) is
 * skipped. Forward uses the bfloat16 copy in state->w_bf16 / b_f32 (the previous step's
 * result, or the caller's initial copy); forward and backward run on the matrix cores
 * with bfloat16 hi/lo operands and float32 accumulation (the W1, W3 and bias
 * gradients on the vector units in float32). Requires the workspace of a gather of
 * [f0, f1) with `params` (relative maps recomputed here). */
sg_status scene_mlp_train_step(const sg_clip* clip, int32_t f0, int32_t f1,
                               const sg_gather_params* params, const sg_sample_sets* sets,
                               const int32_t* pixel_idx, int32_t n_pix, const float* clean_rgb,
                               sg_mlp_train* state, float lr, int32_t t, void* workspace,
                               size_t workspace_bytes, void* stream);

/* Feature statistics for the standardisation of the MLP input: over the records
 * of the sets of pixel_idx[0 .. n_pix) (device int32 indices into [0, P); an index
 * outside is skipped), ADDS the record count to moments[0], the sum of raw feature
 * k to moments[1 + k] and the sum of its square to moments[9 + k] (device float64
 * [17]; the caller clears it, and can accumulate over several calls and clips).
 * Same workspace contract as scene_filter_learned. */
sg_status scene_feature_moments(const sg_clip* clip, int32_t f0, int32_t f1,
                                const sg_gather_params* params, const sg_sample_sets* sets,
                                const int32_t* pixel_idx, int32_t n_pix, double* moments,
                                void* workspace, size_t workspace_bytes, void* stream);

/* The MLP's input standardisation from moments accumulated by
 * scene_feature_moments (device float64 [17]: count, sums, sums of squares): in
 * float64 on the device, mean_k = sum_k / n and std_k = sqrt(max(sumsq_k / n -
 * mean_k^2, 0)) (n = max(count, 1)); a feature with std_k <= 1e-12 max(|mean_k|, 1)
 * (no spread) gets std_k = 1. Writes float32 mean_k and 1 / std_k into the feature
 * mean and 1/std entries of mlp_b (device float32 [SG_MLP_NB]); the other entries
 * are left as they are. SG_E_INVALID on a null pointer. */
sg_status scene_mlp_standardise(const double* moments, float* mlp_b, void* stream);

/* ---------------------------------------------------------------------------
 * Batched gather + filter (the per-clip computation of Sec. 4 and Sec. 5 Eq. 3,
 * run for many clips of different size, length and window in one step).
 *
 * A batch holds n_clips clips and, per clip, n_out consecutive output frames per
 * step; their output pixels form ONE CSR over the batch: clip c's pixels start at
 * sg_batch_pixel_base(b, c), frame-major then row-major within the clip. A step
 * (scene_gather_batched) runs pose prep, count, scan, scatter and filter for every
 * clip, each pass as one persistent launch whose workgroups draw work items from
 * an atomic queue (gather items: 64 x TH pixel tiles, clips in decreasing order of
 * estimated work; filter items: runs of 64 pixels of one clip; each wave of a
 * workgroup draws its own items). Each clip's records and
 * filtered colours are bit-identical to those of scene_gather / scene_filter on
 * that clip alone. All clips of a batch share one radius (else SG_E_UNSUPPORTED).
 * The batch object owns only small device buffers (plan, relative maps, scan
 * partials, queues) and a pinned copy of the step's frames; it is not thread-safe.
 */
#define SG_MAX_BATCH_CLIPS 4096

typedef struct sg_batch sg_batch;

/* Caller-owned device buffers of a step; P = sg_batch_pixel_base(b, n_clips).
 *   offsets : [P + 1] int64 CSR offsets (written by the step)
 *   ids, crho, capacity : record arena as in sg_sample_sets (scatter writes at most
 *             capacity records, else sets SG_FLAG_CAPACITY)
 *   status  : device uint32 flags of the step (cleared by the step)
 *   out_rgb : [P][3] float32 filtered colours, or NULL to gather only. */
typedef struct sg_batch_io {
  int64_t* offsets;
  uint32_t* ids;
  uint16_t* crho;
  int64_t capacity;
  uint32_t* status;
  float* out_rgb;
} sg_batch_io;

/* Plan a batch: clips[c] (stored planes, device poses, intrinsics), params[c],
 * fparams[c] (sigmas, as scene_filter) and n_out[c] >= 1 output frames per step.
 * The descriptors' device pointers must stay valid for the batch's lifetime.
 * SG_E_UNSUPPORTED: more than SG_MAX_BATCH_CLIPS clips, clips with different radii,
 * or more than 2^31 - 1 relative-map floats in total (sum over clips of
 * n_out[c] * (2 window + 1) * 16). */
sg_status sg_batch_create(sg_batch** out, const sg_clip* clips, int32_t n_clips,
                          const sg_gather_params* params, const sg_filter_params* fparams,
                          const int32_t* n_out);
void sg_batch_destroy(sg_batch* b);

/* CSR index of clip c's first output pixel (c = n_clips: total pixels P); -1 on a
 * bad argument. */
int64_t sg_batch_pixel_base(const sg_batch* b, int32_t clip);

/* First output frame of every clip for the next step (host [n_clips]; f0 + n_out
 * <= num_frames). Waits until the previous step has consumed the last frames. */
sg_status sg_batch_set_frames(sg_batch* b, const int32_t* f0);

/* Count pass only (pose prep, count, scan): offsets[P] = records of the step.
 * For sizing the arena; the caller synchronises and reads it. */
sg_status sg_batch_count(sg_batch* b, const sg_batch_io* io, void* stream);

/* One step. Replays the captured graph when io equals the captured one. */
sg_status scene_gather_batched(sg_batch* b, const sg_batch_io* io, void* stream);

/* Capture one step for io into a HIP graph (stream: not the null stream); later
 * scene_gather_batched calls with the same io replay it (frames still come from
 * sg_batch_set_frames through a copy node). Any configuration change drops it. */
sg_status sg_batch_capture(sg_batch* b, const sg_batch_io* io, void* stream);

/* Autotuner: times every count configuration (rows of 64 pixels per work item 1,
 * 2, 4, 8 x source-frame unroll 1, 2, 4) and every scatter rows-per-item value on
 * this batch and step, keeps the fastest and writes it to cfg_out[3] (may be
 * NULL). Needs frames set and an arena that holds the step (else SG_E_CAPACITY).
 * Synchronises the stream. */
sg_status sg_batch_autotune(sg_batch* b, const sg_batch_io* io, void* stream, int32_t* cfg_out);

/* One eager step with events between the passes; ms_out[5] = pose prep, count,
 * scan, scatter, filter (ms). Synchronises the stream. */
sg_status sg_batch_time_passes(sg_batch* b, const sg_batch_io* io, void* stream, float* ms_out);

/* Set / read the configuration (count rows per item, count unroll, scatter rows
 * per item); results do not depend on it. */
sg_status sg_batch_set_config(sg_batch* b, int32_t th_count, int32_t k_count, int32_t th_scatter);
sg_status sg_batch_get_config(const sg_batch* b, int32_t* cfg);

#ifdef __cplusplus
}
#endif

#endif /* SCENE_GATHER_H */
