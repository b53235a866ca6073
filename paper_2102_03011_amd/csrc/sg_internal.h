// Internal declarations shared by the C entry points and the kernel launchers.
#ifndef SG_INTERNAL_H
#define SG_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scene_gather.h"

namespace sg {

constexpr int kRelStride = 16;    // floats per (output frame, source frame) map record
constexpr int kTileW = 64;        // gather tile: one wave per 64-pixel row segment
constexpr int kTileH = 4;         // four waves per workgroup
constexpr int kFuseW = 16;        // fused gather + filter tile: 16 x 16 pixels,
constexpr int kFuseH = 16;        //   four waves of 16 x 4
constexpr int kScanThreads = 256;
constexpr int kScanTile = 4096;   // elements per scan block (16 per thread)
constexpr int kGroup = 16;        // filter lanes per output pixel

struct GatherJob {
  int width, height, n_frames, f0, n_out, w, radius;
  float tol, z_near;
  double fx, fy, cx, cy;
  const double* c2w;
  const uint16_t* rgbd;
  const uint16_t* depth;
  float* rel;          // workspace: n_out * (2w+1) * kRelStride floats
  int64_t* partial;    // workspace: scan partials
  int64_t* offsets;
  uint32_t* ids;
  uint16_t* crho;
  int64_t capacity;
  uint32_t* status;
};

struct FilterJob {
  int width, height, f0, w;
  int64_t n_pix;
  const uint16_t* rgbd;
  const int64_t* offsets;
  const uint32_t* ids;
  const uint16_t* crho;
  int64_t capacity;
  float a_d, a_c, a_t;
  bool use_colour, use_time;
  float* out;
};

struct LearnedJob {
  int width, height, n_frames, f0, w;
  int64_t n_pix;
  float log_norm;
  double fx, fy, cx, cy;
  const uint16_t* rgbd;
  const uint16_t* depth;
  const float* rel;
  const int64_t* offsets;
  const uint32_t* ids;
  const uint16_t* crho;
  int64_t capacity;
  const uint16_t* mw;
  const float* mb;
  float* out;
};

struct TrainJob {
  const int32_t* pixel_idx;
  int n_pix;
  const float* clean;
  float* master;
  float* adam_m;
  float* adam_v;
  float* grad;
  uint16_t* w_bf16;
  float* b_f32;
  float* loss;
  float lr;
  int t;
};

// ---------------------------------------------------------------------------
// batched persistent gather + filter over uneven clips

// One clip of a batch as the batched kernels read it (device memory).
struct BatchClip {
  const uint16_t* rgbd;
  const uint16_t* depth;
  const double* c2w;
  float* rel;            // n_out x (2w+1) x kRelStride floats, owned by the batch
  int width, height, n_frames, n_out, w;
  int rel_at;            // rel - BatchDev::rel, in floats
  float tol, z_near;
  double fx, fy, cx, cy;
  int64_t pix_base;      // CSR index of the clip's first output pixel
  float a_d, a_c, a_t, pad1;
};

// Device-side plan of a batch: clips, per-step first output frames, and the work
// order of the gather passes (clip slots sorted by estimated cost).
struct BatchDev {
  const BatchClip* clips;
  const int* f0;             // [n_clips], updated per step
  const int* order;          // [n_clips]: clip of each slot
  const int64_t* prefix;     // [n_clips + 1] first work item of each slot (tile height th)
  const int64_t* pix_prefix; // [n_clips + 1] CSR base of each clip (clip order)
  const float* rel;          // all clips' relative maps; each BatchClip::rel points into it
  int n_clips;
  int radius;
};

struct BatchIo {
  int64_t* offsets;
  uint32_t* ids;
  uint16_t* crho;
  int64_t capacity;
  uint32_t* status;
  float* out;
};

struct BatchLaunch {
  int th_count, k_count, th_scatter;  // rows per wave work item, source-frame unroll
  int blocks_count, blocks_scatter, blocks_filter;
  bool colour, time;
  int max_slots;                     // max over clips of n_out (2w + 1)
};

int batch_scatter_max_th(int radius);         // largest scatter rows-per-item
size_t batch_scatter_lds_bytes(int radius);   // LDS of one scatter wave
hipError_t launch_batch_prep(const BatchDev& bd, unsigned int* queues, uint32_t* status, int max_slots,
                             hipStream_t st);
hipError_t launch_batch_count(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl,
                              unsigned int* queue, hipStream_t st);
hipError_t launch_batch_scatter(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl,
                                unsigned int* queue, hipStream_t st);
hipError_t launch_batch_filter(const BatchDev& bd, const BatchIo& io, const BatchLaunch& bl,
                               const int64_t* fprefix, unsigned int* queue, hipStream_t st);
int64_t batch_filter_items(int64_t clip_pixels);  // filter work items of a clip

hipError_t launch_filter_learned(const LearnedJob& lj, hipStream_t st);
hipError_t launch_mlp_train(const LearnedJob& lj, const TrainJob& tj, hipStream_t st);
hipError_t launch_standardise(const double* moments, float* mlp_b, hipStream_t st);
hipError_t launch_feature_moments(const LearnedJob& lj, const int32_t* pixel_idx, int n_pix, double* moments,
                                  hipStream_t st);

// Every host-side check of scene_gather (no HIP call) and its workspace bytes.
sg_status gather_host_checks(const sg_clip* clip, int32_t f0, int32_t f1, const sg_gather_params* params,
                             const sg_sample_sets* sets, size_t* ws_bytes);

hipError_t launch_stage(const uint8_t* rgb, const float* depth, int n_frames, int width, int height,
                        uint16_t* rgbd, uint16_t* depth16, hipStream_t st);
hipError_t launch_pose_prep(const GatherJob& jb, hipStream_t st);
hipError_t launch_count(const GatherJob& jb, hipStream_t st);
hipError_t launch_scan(int64_t* offsets, int64_t n, int64_t* partial, hipStream_t st);
hipError_t launch_scatter(const GatherJob& jb, hipStream_t st);
hipError_t launch_filter(const FilterJob& fj, hipStream_t st);
hipError_t launch_gather_filter(const GatherJob& jb, const FilterJob& fj, hipStream_t st);

}  // namespace sg

#endif
