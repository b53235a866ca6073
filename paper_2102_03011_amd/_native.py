"""ctypes declarations of the C ABI in include/scene_gather.h, include/scene_filters.h,
include/scene_frustum.h and include/scene_depth.h.

Loads the in-tree libscenegather.so. There is no fallback: if the library is
missing or fails to load, import of the binding raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscenegather.so")

SG_OK, SG_E_INVALID, SG_E_CAPACITY, SG_E_HIP, SG_E_UNSUPPORTED = 0, 1, 2, 3, 4
SG_FLAG_CAPACITY, SG_FLAG_INCONSISTENT = 1, 2
SG_ID_SHIFT = 22
SG_MAX_WINDOW = 511
SG_MAX_RADIUS = 3
SG_APRON = 6
SG_APRON_RIGHT = 7
SG_MAX_INPAINT_STEPS = 16
SG_MAX_FRUSTUM_L = 7.0
SG_MAX_DEPTH_HYPOTHESES = 4096
SG_NOALLOC_SCRATCH_BYTES = 4 << 20

c_void_p = ctypes.c_void_p


class SgClip(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("num_frames", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("rgbd", c_void_p), ("depth", c_void_p), ("cam_to_world", c_void_p),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
    ]


class SgGatherParams(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("tol", ctypes.c_float), ("z_near", ctypes.c_float)]


class SgSampleSets(ctypes.Structure):
    _fields_ = [("offsets", c_void_p), ("ids", c_void_p), ("crho", c_void_p),
                ("capacity", ctypes.c_int64), ("status", c_void_p)]


class SgFrustumParams(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("l", ctypes.c_float), ("near_z", ctypes.c_float),
                ("far_z", ctypes.c_float)]


class SgFilterParams(ctypes.Structure):
    _fields_ = [("sigma_d", ctypes.c_float), ("sigma_c", ctypes.c_float),
                ("sigma_t", ctypes.c_float), ("reserved", ctypes.c_float)]


SG_MLP_NW = 8 * 64 + 64 * 64 + 64
SG_MLP_NB = 64 + 64 + 4 + 8 + 8
SG_MLP_NPARAM = SG_MLP_NW + 64 + 64 + 1


class SgMlp(ctypes.Structure):
    _fields_ = [("w", c_void_p), ("b", c_void_p)]


class SgMlpTrain(ctypes.Structure):
    _fields_ = [("master", c_void_p), ("adam_m", c_void_p), ("adam_v", c_void_p), ("grad", c_void_p),
                ("w_bf16", c_void_p), ("b_f32", c_void_p), ("loss", c_void_p)]


class SgBatchIo(ctypes.Structure):
    _fields_ = [("offsets", c_void_p), ("ids", c_void_p), ("crho", c_void_p), ("capacity", ctypes.c_int64),
                ("status", c_void_p), ("out_rgb", c_void_p)]


SG_MAX_BATCH_CLIPS = 4096

# name -> (restype, argtypes); every function declared in include/scene_gather.h
SIGNATURES = {
    "sg_version": (ctypes.c_int32, []),
    "sg_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "scene_stage": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    c_void_p, c_void_p, c_void_p]),
    "scene_gather_workspace_size": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.POINTER(SgGatherParams), ctypes.POINTER(ctypes.c_size_t)]),
    "scene_gather_count": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                           c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_gather_scatter": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                             c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_gather": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                     c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_gather_noalloc": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                             c_void_p]),
    "scene_filter": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(SgSampleSets), ctypes.POINTER(SgFilterParams),
                                     c_void_p, c_void_p]),
    "scene_gather_filter": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgFilterParams),
                                            c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_frame_sharpness": (ctypes.c_int, [ctypes.POINTER(SgClip), c_void_p, c_void_p]),
    "scene_filter_frames": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(SgSampleSets), ctypes.POINTER(SgFilterParams),
                                            c_void_p, c_void_p, c_void_p]),
    "scene_inpaint": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(SgSampleSets), c_void_p, ctypes.c_float, ctypes.c_int32,
                                      c_void_p, c_void_p]),
    "scene_filter_xyz": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                         ctypes.POINTER(SgFilterParams), ctypes.c_float, c_void_p, c_void_p,
                                         ctypes.c_size_t, c_void_p, c_void_p]),
    "scene_semi_transparent": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(SgSampleSets), c_void_p, ctypes.c_float, ctypes.c_float,
                                               ctypes.c_int32, c_void_p, c_void_p]),
    "scene_box_mask": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.POINTER(ctypes.c_double), c_void_p, c_void_p]),
    "scene_frustum_workspace_size": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32,
                                                     ctypes.POINTER(SgFrustumParams), ctypes.POINTER(ctypes.c_size_t)]),
    "scene_frustum_count": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.POINTER(SgFrustumParams),
                                            ctypes.POINTER(SgSampleSets), c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_frustum_scatter": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.POINTER(SgFrustumParams),
                                              ctypes.POINTER(SgSampleSets), c_void_p, ctypes.c_size_t, c_void_p]),
    "scene_depth_workspace_size": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "scene_estimate_depth": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32, c_void_p,
                                             ctypes.c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_size_t,
                                             c_void_p]),
    "scene_filter_learned": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                             ctypes.POINTER(SgMlp), c_void_p, ctypes.c_size_t, c_void_p, c_void_p]),
    "scene_feature_moments": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                              c_void_p, ctypes.c_int32, c_void_p, c_void_p, ctypes.c_size_t,
                                              c_void_p]),
    "scene_mlp_standardise": (ctypes.c_int, [c_void_p, c_void_p, c_void_p]),
    "sg_batch_create": (ctypes.c_int, [ctypes.POINTER(c_void_p), ctypes.POINTER(SgClip), ctypes.c_int32,
                                        ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgFilterParams),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "sg_batch_destroy": (None, [c_void_p]),
    "sg_batch_pixel_base": (ctypes.c_int64, [c_void_p, ctypes.c_int32]),
    "sg_batch_set_frames": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "sg_batch_count": (ctypes.c_int, [c_void_p, ctypes.POINTER(SgBatchIo), c_void_p]),
    "scene_gather_batched": (ctypes.c_int, [c_void_p, ctypes.POINTER(SgBatchIo), c_void_p]),
    "sg_batch_capture": (ctypes.c_int, [c_void_p, ctypes.POINTER(SgBatchIo), c_void_p]),
    "sg_batch_autotune": (ctypes.c_int, [c_void_p, ctypes.POINTER(SgBatchIo), c_void_p,
                                          ctypes.POINTER(ctypes.c_int32)]),
    "sg_batch_time_passes": (ctypes.c_int, [c_void_p, ctypes.POINTER(SgBatchIo), c_void_p,
                                             ctypes.POINTER(ctypes.c_float)]),
    "sg_batch_set_config": (ctypes.c_int, [c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "sg_batch_get_config": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "scene_mlp_train_step": (ctypes.c_int, [ctypes.POINTER(SgClip), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(SgGatherParams), ctypes.POINTER(SgSampleSets),
                                             c_void_p, ctypes.c_int32, c_void_p, ctypes.POINTER(SgMlpTrain),
                                             ctypes.c_float, ctypes.c_int32, c_void_p, ctypes.c_size_t, c_void_p]),
}


def load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run `python -m paper_2102_03011_amd.build`)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
