// Batched gather + filter over clips of uneven size, length and window: the host
// plan (work order, per-step frames), the enqueue of one step (persistent passes),
// its capture as a HIP graph, and the autotuner of tile shape and source-frame
// unroll.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "scene_gather.h"
#include "sg_internal.h"
#include "sg_validate.h"

using sg::hip_status;

struct sg_batch {
  int device = 0;
  int n_clips = 0;
  int radius = 0;
  int cus = 256;
  std::vector<sg_clip> clips;
  std::vector<sg_gather_params> params;
  std::vector<int> n_out;
  std::vector<int64_t> pix_prefix;  // CSR base per clip (clip order), n + 1
  std::vector<int> order;           // slots: clips by decreasing estimated work
  int64_t total_pix = 0;
  int max_slots = 1;
  bool colour = false, time = false;
  // one device allocation holds every small buffer of the plan
  void* dmem = nullptr;
  sg::BatchClip* d_clips = nullptr;
  int* d_f0 = nullptr;
  int* d_order = nullptr;
  int64_t* d_prefix[4] = {nullptr, nullptr, nullptr, nullptr};  // tile heights 1, 2, 4, 8
  int64_t* d_pix_prefix = nullptr;
  int64_t* d_fprefix = nullptr;     // first filter work item of each clip (clip order), n + 1
  int64_t* d_partial = nullptr;
  unsigned int* d_queues = nullptr;
  float* d_rel = nullptr;
  int* h_f0 = nullptr;          // pinned: the frames of the next step
  hipEvent_t step_done = nullptr;
  bool step_recorded = false;
  bool frames_set = false;
  // launch configuration (autotuned)
  int th_count = 4, k_count = 1, th_scatter = 4;
  // captured step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  sg::BatchIo graph_io{};
};

namespace {

// cleanup calls whose failure changes nothing the caller can act on
void ignore(hipError_t) {}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int th_index(int th) { return th == 1 ? 0 : (th == 2 ? 1 : (th == 4 ? 2 : 3)); }

int64_t items_of(const sg_batch& b, int clip, int th) {
  const sg_clip& c = b.clips[clip];
  const int64_t tx = (c.width + sg::kTileW - 1) / sg::kTileW, ty = (c.height + th - 1) / th;
  return tx * ty * b.n_out[clip];
}

void drop_graph(sg_batch* b) {
  if (b->exec != nullptr) ignore(hipGraphExecDestroy(b->exec));
  if (b->graph != nullptr) ignore(hipGraphDestroy(b->graph));
  b->exec = nullptr;
  b->graph = nullptr;
}

sg::BatchDev dev_view(const sg_batch& b, int th) {
  sg::BatchDev d{};
  d.clips = b.d_clips;
  d.f0 = b.d_f0;
  d.order = b.d_order;
  d.prefix = b.d_prefix[th_index(th)];
  d.pix_prefix = b.d_pix_prefix;
  d.rel = b.d_rel;
  d.n_clips = b.n_clips;
  d.radius = b.radius;
  return d;
}

sg::BatchLaunch launch_cfg(const sg_batch& b) {
  sg::BatchLaunch l{};
  l.th_count = b.th_count;
  l.k_count = b.k_count;
  l.th_scatter = b.th_scatter;
  // persistent grids of 4-wave workgroups: enough to fill every CU (8 waves per SIMD,
  // or as many scatter workgroups as LDS holds), never more than there are items
  const int64_t items_c = b.total_pix > 0 ? (b.total_pix + 255) / 256 : 1;
  l.blocks_count = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(b.cus) * 8, items_c));
  const size_t lds = sg::batch_scatter_lds_bytes(b.radius) * 4;
  const int per_cu = std::max<int>(1, static_cast<int>(163840 / std::max<size_t>(lds, 1)));
  l.blocks_scatter = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(b.cus) * std::min(per_cu, 8), items_c));
  l.blocks_filter = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(b.cus) * 8, items_c));
  if (l.blocks_count < 1) l.blocks_count = 1;
  if (l.blocks_scatter < 1) l.blocks_scatter = 1;
  if (l.blocks_filter < 1) l.blocks_filter = 1;
  l.colour = b.colour;
  l.time = b.time;
  l.max_slots = b.max_slots;
  return l;
}

sg::BatchIo io_of(const sg_batch_io* io) {
  sg::BatchIo r{};
  r.offsets = io->offsets;
  r.ids = io->ids;
  r.crho = io->crho;
  r.capacity = io->capacity;
  r.status = io->status;
  r.out = io->out_rgb;
  return r;
}

bool same_io(const sg::BatchIo& a, const sg::BatchIo& b) {
  return a.offsets == b.offsets && a.ids == b.ids && a.crho == b.crho && a.capacity == b.capacity &&
         a.status == b.status && a.out == b.out;
}

sg_status check_io(const sg_batch* b, const sg_batch_io* io, bool need_arena) {
  if (b == nullptr || io == nullptr || io->offsets == nullptr || io->status == nullptr) return SG_E_INVALID;
  if (need_arena && (io->capacity < 0 || (io->capacity > 0 && (io->ids == nullptr || io->crho == nullptr))))
    return SG_E_INVALID;
  if (!b->frames_set) return SG_E_INVALID;
  return SG_OK;
}

// Frames copy, pose prep (also clears queues and status), count, scan.
sg_status enqueue_count(sg_batch* b, const sg::BatchIo& io, const sg::BatchLaunch& l, hipStream_t st) {
  sg_status s = hip_status(hipMemcpyAsync(b->d_f0, b->h_f0, sizeof(int) * b->n_clips, hipMemcpyHostToDevice, st));
  if (s != SG_OK) return s;
  if ((s = hip_status(sg::launch_batch_prep(dev_view(*b, 1), b->d_queues, io.status, l.max_slots, st))) != SG_OK)
    return s;
  if ((s = hip_status(sg::launch_batch_count(dev_view(*b, l.th_count), io, l, b->d_queues + 0, st))) != SG_OK)
    return s;
  return hip_status(sg::launch_scan(io.offsets, b->total_pix, b->d_partial, st));
}

sg_status enqueue_step(sg_batch* b, const sg::BatchIo& io, hipStream_t st) {
  const sg::BatchLaunch l = launch_cfg(*b);
  sg_status s = enqueue_count(b, io, l, st);
  if (s != SG_OK) return s;
  if ((s = hip_status(sg::launch_batch_scatter(dev_view(*b, l.th_scatter), io, l, b->d_queues + 1, st))) != SG_OK)
    return s;
  if (io.out == nullptr) return SG_OK;
  return hip_status(sg::launch_batch_filter(dev_view(*b, 1), io, l, b->d_fprefix, b->d_queues + 2, st));
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) return INFINITY;
  return ms;
}

}  // namespace

extern "C" {

sg_status sg_batch_create(sg_batch** out, const sg_clip* clips, int32_t n_clips, const sg_gather_params* params,
                          const sg_filter_params* fparams, const int32_t* n_out) {
  if (out == nullptr) return SG_E_INVALID;
  *out = nullptr;
  if (clips == nullptr || params == nullptr || fparams == nullptr || n_out == nullptr) return SG_E_INVALID;
  if (n_clips <= 0) return SG_E_INVALID;
  if (n_clips > SG_MAX_BATCH_CLIPS) return SG_E_UNSUPPORTED;
  size_t maps = 0;  // relative-map floats of all clips: the kernels index them with int offsets
  for (int c = 0; c < n_clips; ++c) {
    sg_status s = sg::check_clip(&clips[c], true);
    if (s != SG_OK) return s;
    if ((s = sg::check_params(&params[c])) != SG_OK) return s;
    if (params[c].radius != params[0].radius) return SG_E_UNSUPPORTED;
    if (n_out[c] < 1 || n_out[c] > clips[c].num_frames) return SG_E_INVALID;
    const float sd = fparams[c].sigma_d, sc = fparams[c].sigma_c, stt = fparams[c].sigma_t;
    if (!(sd > 0.0f) || !(sc > 0.0f) || !(stt > 0.0f)) return SG_E_INVALID;
    maps += static_cast<size_t>(n_out[c]) * (2 * static_cast<size_t>(params[c].window) + 1) * sg::kRelStride;
  }
  if (maps > static_cast<size_t>(INT32_MAX)) return SG_E_UNSUPPORTED;
  sg_batch* b = new (std::nothrow) sg_batch();
  if (b == nullptr) return SG_E_HIP;
  b->n_clips = n_clips;
  b->radius = params[0].radius;
  b->clips.assign(clips, clips + n_clips);
  b->params.assign(params, params + n_clips);
  b->n_out.assign(n_out, n_out + n_clips);
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    delete b;
    return SG_E_HIP;
  }
  // CSR layout (clip order) and work order (decreasing candidates per step)
  b->pix_prefix.assign(n_clips + 1, 0);
  std::vector<double> cost(n_clips);
  size_t rel_floats = 0;
  for (int c = 0; c < n_clips; ++c) {
    const int64_t pix = static_cast<int64_t>(clips[c].width) * clips[c].height * n_out[c];
    b->pix_prefix[c + 1] = b->pix_prefix[c] + pix;
    const int slots = 2 * params[c].window + 1;
    cost[c] = static_cast<double>(pix) * std::min(slots, clips[c].num_frames);
    b->max_slots = std::max(b->max_slots, n_out[c] * slots);
    rel_floats += static_cast<size_t>(n_out[c]) * slots * sg::kRelStride;
    if (isfinite(fparams[c].sigma_c)) b->colour = true;
    if (isfinite(fparams[c].sigma_t)) b->time = true;
  }
  b->total_pix = b->pix_prefix[n_clips];
  b->order.resize(n_clips);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  // device buffers
  const size_t n = static_cast<size_t>(n_clips);
  const size_t nb = static_cast<size_t>((b->total_pix + sg::kScanTile - 1) / sg::kScanTile) + 1;
  size_t off = 0;
  const size_t o_clips = off; off = align_up(off + n * sizeof(sg::BatchClip));
  const size_t o_f0 = off; off = align_up(off + n * sizeof(int));
  const size_t o_order = off; off = align_up(off + n * sizeof(int));
  size_t o_prefix[4];
  for (int t = 0; t < 4; ++t) { o_prefix[t] = off; off = align_up(off + (n + 1) * sizeof(int64_t)); }
  const size_t o_pix = off; off = align_up(off + (n + 1) * sizeof(int64_t));
  const size_t o_fpre = off; off = align_up(off + (n + 1) * sizeof(int64_t));
  const size_t o_part = off; off = align_up(off + nb * sizeof(int64_t));
  const size_t o_q = off; off = align_up(off + 4 * sizeof(unsigned int));
  const size_t o_rel = off; off = align_up(off + rel_floats * sizeof(float));
  if (hipMalloc(&b->dmem, off) != hipSuccess) {
    b->dmem = nullptr;
    sg_batch_destroy(b);
    return SG_E_HIP;
  }
  char* base = static_cast<char*>(b->dmem);
  b->d_clips = reinterpret_cast<sg::BatchClip*>(base + o_clips);
  b->d_f0 = reinterpret_cast<int*>(base + o_f0);
  b->d_order = reinterpret_cast<int*>(base + o_order);
  for (int t = 0; t < 4; ++t) b->d_prefix[t] = reinterpret_cast<int64_t*>(base + o_prefix[t]);
  b->d_pix_prefix = reinterpret_cast<int64_t*>(base + o_pix);
  b->d_fprefix = reinterpret_cast<int64_t*>(base + o_fpre);
  b->d_partial = reinterpret_cast<int64_t*>(base + o_part);
  b->d_queues = reinterpret_cast<unsigned int*>(base + o_q);
  float* rel = reinterpret_cast<float*>(base + o_rel);
  b->d_rel = rel;
  const double log2e = 1.4426950408889634;
  std::vector<sg::BatchClip> hc(n);
  size_t rel_at = 0;
  for (int c = 0; c < n_clips; ++c) {
    sg::BatchClip& d = hc[c];
    memset(&d, 0, sizeof(d));
    d.rgbd = clips[c].rgbd;
    d.depth = clips[c].depth;
    d.c2w = clips[c].cam_to_world;
    d.rel = rel + rel_at;
    d.rel_at = static_cast<int>(rel_at);
    rel_at += static_cast<size_t>(n_out[c]) * (2 * params[c].window + 1) * sg::kRelStride;
    d.width = clips[c].width;
    d.height = clips[c].height;
    d.n_frames = clips[c].num_frames;
    d.n_out = n_out[c];
    d.w = params[c].window;
    d.tol = params[c].tol;
    d.z_near = params[c].z_near;
    d.fx = clips[c].fx;
    d.fy = clips[c].fy;
    d.cx = clips[c].cx;
    d.cy = clips[c].cy;
    d.pix_base = b->pix_prefix[c];
    // the same constants as the single-clip filter entry point
    const float sd = fparams[c].sigma_d, sc = fparams[c].sigma_c, stt = fparams[c].sigma_t;
    d.a_d = isfinite(sd) ? static_cast<float>(-log2e / (2.0 * sd * static_cast<double>(sd))) : 0.0f;
    d.a_c = isfinite(sc) ? static_cast<float>(-log2e / (2.0 * sc * static_cast<double>(sc))) : 0.0f;
    d.a_t = isfinite(stt) ? static_cast<float>(-log2e / (2.0 * stt * static_cast<double>(stt))) : 0.0f;
  }
  std::vector<int64_t> prefix(n + 1), fprefix(n + 1, 0);
  for (int c = 0; c < n_clips; ++c)
    fprefix[c + 1] = fprefix[c] + sg::batch_filter_items(b->pix_prefix[c + 1] - b->pix_prefix[c]);
  bool ok = hipMemcpy(b->d_clips, hc.data(), n * sizeof(sg::BatchClip), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(b->d_order, b->order.data(), n * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(b->d_pix_prefix, b->pix_prefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(b->d_fprefix, fprefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
  for (int t = 0; t < 4 && ok; ++t) {
    const int th = 1 << t;
    prefix[0] = 0;
    for (int k = 0; k < n_clips; ++k) prefix[k + 1] = prefix[k] + items_of(*b, b->order[k], th);
    ok = hipMemcpy(b->d_prefix[t], prefix.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
  }
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_f0), n * sizeof(int), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->step_done, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    sg_batch_destroy(b);
    return SG_E_HIP;
  }
  b->th_scatter = std::min(b->th_scatter, sg::batch_scatter_max_th(b->radius));
  *out = b;
  return SG_OK;
}

void sg_batch_destroy(sg_batch* b) {
  if (b == nullptr) return;
  if (b->step_recorded) ignore(hipEventSynchronize(b->step_done));
  drop_graph(b);
  if (b->step_done != nullptr) ignore(hipEventDestroy(b->step_done));
  if (b->h_f0 != nullptr) ignore(hipHostFree(b->h_f0));
  if (b->dmem != nullptr) ignore(hipFree(b->dmem));
  delete b;
}

int64_t sg_batch_pixel_base(const sg_batch* b, int32_t clip) {
  if (b == nullptr || clip < 0 || clip > b->n_clips) return -1;
  return b->pix_prefix[clip];
}

sg_status sg_batch_set_frames(sg_batch* b, const int32_t* f0) {
  if (b == nullptr || f0 == nullptr) return SG_E_INVALID;
  for (int c = 0; c < b->n_clips; ++c)
    if (f0[c] < 0 || f0[c] + b->n_out[c] > b->clips[c].num_frames) return SG_E_INVALID;
  // the previous step's copy of the frames must have been consumed
  if (b->step_recorded && hipEventSynchronize(b->step_done) != hipSuccess) return SG_E_HIP;
  for (int c = 0; c < b->n_clips; ++c) b->h_f0[c] = f0[c];
  b->frames_set = true;
  return SG_OK;
}

sg_status sg_batch_set_config(sg_batch* b, int32_t th_count, int32_t k_count, int32_t th_scatter) {
  if (b == nullptr) return SG_E_INVALID;
  auto pow2 = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
  if (!pow2(th_count) || !pow2(th_scatter) || !(k_count == 1 || k_count == 2 || k_count == 4)) return SG_E_INVALID;
  if (th_scatter > sg::batch_scatter_max_th(b->radius)) return SG_E_UNSUPPORTED;
  b->th_count = th_count;
  b->k_count = k_count;
  b->th_scatter = th_scatter;
  drop_graph(b);
  return SG_OK;
}

sg_status sg_batch_get_config(const sg_batch* b, int32_t* cfg) {
  if (b == nullptr || cfg == nullptr) return SG_E_INVALID;
  cfg[0] = b->th_count;
  cfg[1] = b->k_count;
  cfg[2] = b->th_scatter;
  return SG_OK;
}

sg_status sg_batch_count(sg_batch* b, const sg_batch_io* io, void* stream) {
  sg_status s = check_io(b, io, false);
  if (s != SG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = enqueue_count(b, io_of(io), launch_cfg(*b), st)) != SG_OK) return s;
  if ((s = hip_status(hipEventRecord(b->step_done, st))) != SG_OK) return s;
  b->step_recorded = true;
  return SG_OK;
}

sg_status scene_gather_batched(sg_batch* b, const sg_batch_io* io, void* stream) {
  sg_status s = check_io(b, io, true);
  if (s != SG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const sg::BatchIo bio = io_of(io);
  if (b->exec != nullptr && same_io(bio, b->graph_io))
    s = hip_status(hipGraphLaunch(b->exec, st));
  else
    s = enqueue_step(b, bio, st);
  if (s != SG_OK) return s;
  if ((s = hip_status(hipEventRecord(b->step_done, st))) != SG_OK) return s;
  b->step_recorded = true;
  return SG_OK;
}

sg_status sg_batch_capture(sg_batch* b, const sg_batch_io* io, void* stream) {
  sg_status s = check_io(b, io, true);
  if (s != SG_OK) return s;
  if (stream == nullptr) return SG_E_INVALID;  // the null stream cannot be captured
  hipStream_t st = static_cast<hipStream_t>(stream);
  drop_graph(b);
  const sg::BatchIo bio = io_of(io);
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SG_E_HIP;
  const sg_status se = enqueue_step(b, bio, st);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(st, &g);
  if (se != SG_OK || ee != hipSuccess || g == nullptr) {
    if (g != nullptr) ignore(hipGraphDestroy(g));
    return se != SG_OK ? se : SG_E_HIP;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    ignore(hipGraphDestroy(g));
    return SG_E_HIP;
  }
  b->graph = g;
  b->exec = ex;
  b->graph_io = bio;
  return SG_OK;
}

sg_status sg_batch_time_passes(sg_batch* b, const sg_batch_io* io, void* stream, float* ms_out) {
  sg_status s = check_io(b, io, true);
  if (s != SG_OK) return s;
  if (ms_out == nullptr) return SG_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const sg::BatchIo bio = io_of(io);
  const sg::BatchLaunch l = launch_cfg(*b);
  hipEvent_t ev[6] = {};
  for (int i = 0; i < 6; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) {
      for (int k = 0; k < i; ++k) ignore(hipEventDestroy(ev[k]));
      return SG_E_HIP;
    }
  s = hip_status(hipMemcpyAsync(b->d_f0, b->h_f0, sizeof(int) * b->n_clips, hipMemcpyHostToDevice, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[0], st));
  if (s == SG_OK) s = hip_status(sg::launch_batch_prep(dev_view(*b, 1), b->d_queues, bio.status, l.max_slots, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[1], st));
  if (s == SG_OK) s = hip_status(sg::launch_batch_count(dev_view(*b, l.th_count), bio, l, b->d_queues, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[2], st));
  if (s == SG_OK) s = hip_status(sg::launch_scan(bio.offsets, b->total_pix, b->d_partial, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[3], st));
  if (s == SG_OK)
    s = hip_status(sg::launch_batch_scatter(dev_view(*b, l.th_scatter), bio, l, b->d_queues + 1, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[4], st));
  if (s == SG_OK && bio.out != nullptr)
    s = hip_status(sg::launch_batch_filter(dev_view(*b, 1), bio, l, b->d_fprefix, b->d_queues + 2, st));
  if (s == SG_OK) s = hip_status(hipEventRecord(ev[5], st));
  for (int i = 0; i < 5 && s == SG_OK; ++i) ms_out[i] = elapsed(ev[i], ev[i + 1]);
  for (int i = 0; i < 6; ++i) ignore(hipEventDestroy(ev[i]));
  if (s == SG_OK) s = hip_status(hipEventRecord(b->step_done, st));
  if (s == SG_OK) b->step_recorded = true;
  return s;
}

sg_status sg_batch_autotune(sg_batch* b, const sg_batch_io* io, void* stream, int32_t* cfg_out) {
  sg_status s = check_io(b, io, true);
  if (s != SG_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const sg::BatchIo bio = io_of(io);
  drop_graph(b);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0 != nullptr) ignore(hipEventDestroy(e0));
    return SG_E_HIP;
  }
  // the arena must hold the step, or the scatter timings mean nothing
  s = enqueue_count(b, bio, launch_cfg(*b), st);
  int64_t total = -1;
  if (s == SG_OK)
    s = hip_status(hipMemcpyAsync(&total, bio.offsets + b->total_pix, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (s == SG_OK) s = hip_status(hipStreamSynchronize(st));
  if (s == SG_OK && total > bio.capacity) s = SG_E_CAPACITY;
  const int reps = 2;
  // count: tile height x source-frame unroll
  float best = INFINITY;
  int best_th = b->th_count, best_k = b->k_count;
  for (int th = 1; th <= 8 && s == SG_OK; th <<= 1)
    for (int k = 1; k <= 4 && s == SG_OK; k <<= 1) {
      b->th_count = th;
      b->k_count = k;
      const sg::BatchLaunch l = launch_cfg(*b);
      float t = INFINITY;
      for (int r = 0; r < reps && s == SG_OK; ++r) {
        s = hip_status(sg::launch_batch_prep(dev_view(*b, 1), b->d_queues, bio.status, l.max_slots, st));
        if (s == SG_OK) s = hip_status(hipEventRecord(e0, st));
        if (s == SG_OK) s = hip_status(sg::launch_batch_count(dev_view(*b, th), bio, l, b->d_queues, st));
        if (s == SG_OK) s = hip_status(hipEventRecord(e1, st));
        if (s == SG_OK) t = std::min(t, elapsed(e0, e1));
      }
      if (t < best) {
        best = t;
        best_th = th;
        best_k = k;
      }
    }
  b->th_count = best_th;
  b->k_count = best_k;
  // scatter: tile height (offsets from a scan of the last count)
  if (s == SG_OK) s = enqueue_count(b, bio, launch_cfg(*b), st);
  best = INFINITY;
  int best_ts = b->th_scatter;
  for (int th = 1; th <= sg::batch_scatter_max_th(b->radius) && s == SG_OK; th <<= 1) {
    b->th_scatter = th;
    const sg::BatchLaunch l = launch_cfg(*b);
    float t = INFINITY;
    for (int r = 0; r < reps && s == SG_OK; ++r) {
      s = hip_status(sg::launch_batch_prep(dev_view(*b, 1), b->d_queues, bio.status, l.max_slots, st));
      if (s == SG_OK) s = hip_status(hipEventRecord(e0, st));
      if (s == SG_OK) s = hip_status(sg::launch_batch_scatter(dev_view(*b, th), bio, l, b->d_queues + 1, st));
      if (s == SG_OK) s = hip_status(hipEventRecord(e1, st));
      if (s == SG_OK) t = std::min(t, elapsed(e0, e1));
    }
    if (t < best) {
      best = t;
      best_ts = th;
    }
  }
  b->th_scatter = best_ts;
  ignore(hipStreamSynchronize(st));
  ignore(hipEventDestroy(e0));
  ignore(hipEventDestroy(e1));
  if (s == SG_OK && cfg_out != nullptr) {
    cfg_out[0] = b->th_count;
    cfg_out[1] = b->k_count;
    cfg_out[2] = b->th_scatter;
  }
  return s;
}

}  // extern "C"
