// Allocation-free gather: scene_gather with its workspace (relative camera maps and
// scan partials) in a fixed-size array of device memory owned by the library, for
// callers that cannot allocate.
//
// The array is a file-scope __device__ variable, so every GPU the library runs on
// holds its own copy until the process ends. In host code the variable's name is
// not a device address: the address of each GPU's copy is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept, and only that
// address is handed to the kernels.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "scene_gather.h"
#include "sg_internal.h"

namespace {

static_assert(SG_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of its alignment");

__device__ __align__(256) unsigned char scratch[SG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, looked up on the first call for that device.
sg_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return SG_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return SG_E_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return SG_E_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return SG_E_HIP;
    if (e != hipSuccess || p == nullptr) return SG_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SG_OK;
}

}  // namespace

extern "C" sg_status scene_gather_noalloc(const sg_clip* clip, int32_t f0, int32_t f1,
                                          const sg_gather_params* params, sg_sample_sets* sets,
                                          void* stream) {
  // every host check of scene_gather first, before any HIP call
  size_t need = 0;
  sg_status s = sg::gather_host_checks(clip, f0, f1, params, sets, &need);
  if (s != SG_OK) return s;
  if (need > SG_NOALLOC_SCRATCH_BYTES) return SG_E_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = -1;
  if (hipStreamGetDevice(st, &dev) != hipSuccess) return SG_E_HIP;
  void* ws = nullptr;
  if ((s = scratch_on(dev, &ws)) != SG_OK) return s;
  // every byte the gather reads from its workspace is written earlier in the same
  // call (pose prep writes all maps, the scan's first phase all partials), so the
  // previous call's contents never need clearing
  return scene_gather(clip, f0, f1, params, sets, ws, SG_NOALLOC_SCRATCH_BYTES, stream);
}
