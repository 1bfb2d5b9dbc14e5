"""ctypes mirror of include/dvr.h and the loader of libdvr.so.

Argument marshalling only: every step of the feature pass and of the raymarch runs in the HIP
kernels of libdvr.so.  There is no fallback path; a missing library is an error.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dvr.h")

DVR_OK = 0
STATUS = {0: "DVR_OK", -1: "DVR_E_INVALID_ARG", -2: "DVR_E_NULL", -3: "DVR_E_ALIGN", -4: "DVR_E_UNSUPPORTED",
          -5: "DVR_E_NOMEM", -6: "DVR_E_DEVICE", -8: "DVR_E_TIMEOUT", -9: "DVR_E_WORKSPACE"}
DVR_F32, DVR_F16, DVR_U16 = 0, 1, 2
DVR_PLANAR, DVR_INTERLEAVED, DVR_SPLIT, DVR_QUAD = 0, 1, 2, 3
DVR_MAX_SIGMA = 8
DVR_BRICK = 4
DVR_DENOISE_GAUSS, DVR_DENOISE_MEDIAN3 = 0, 1


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("hx", C.c_float), ("hy", C.c_float), ("hz", C.c_float)]


class FeatureParams(C.Structure):
    _fields_ = [("nsigma", C.c_int32), ("sigma_mm", C.c_float * DVR_MAX_SIGMA), ("alpha", C.c_float),
                ("beta", C.c_float), ("c", C.c_float), ("eig_gap_fp64", C.c_float)]


class FeaturesBuf(C.Structure):
    _fields_ = [("grad", C.c_void_p), ("kappa", C.c_void_p), ("ves", C.c_void_p), ("gmax", C.c_void_p),
                ("dtype", C.c_int32), ("layout", C.c_int32), ("bricks", C.c_void_p), ("iquad", C.c_void_p)]


class Peaks(C.Structure):
    _fields_ = [("bin", C.c_int32 * 3), ("peak", C.c_float * 3), ("in_window", C.c_int32 * 3)]


class TissueTFParams(C.Structure):
    _fields_ = [("rgb", (C.c_float * 3) * 3), ("tau", C.c_float * 3), ("rgb_hi", C.c_float * 3), ("tau_hi", C.c_float)]


class TF(C.Structure):
    _fields_ = [("K", C.c_int32), ("knots", C.c_void_p), ("rgba", C.c_void_p)]


class RenderParams(C.Structure):
    _fields_ = [("lambda_g", C.c_float), ("lambda_k", C.c_float), ("kappa0", C.c_float), ("lambda_v", C.c_float),
                ("step_vox", C.c_float), ("et_alpha", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("persp", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("o", C.c_float * 3),
                ("d0", C.c_float * 3), ("du", C.c_float * 3), ("dv", C.c_float * 3)]


class RayState(C.Structure):
    _fields_ = [("T_last", C.c_void_p), ("k_last", C.c_void_p), ("counters", C.c_void_p)]


class FeatureGrads(C.Structure):
    _fields_ = [("dfeat", C.c_void_p), ("dgmax", C.c_void_p)]


class BatchVolume(C.Structure):
    _fields_ = [("vol", C.c_void_p), ("vol_dtype", C.c_int32), ("grid", Grid), ("feat", FeaturesBuf)]


class BatchView(C.Structure):
    _fields_ = [("volume", C.c_int32), ("cam", Camera), ("rgba", C.c_void_p), ("T_last", C.c_void_p),
                ("k_last", C.c_void_p)]


class Tune(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("xy_tile", C.c_int32), ("xy_zrun", C.c_int32), ("z_chunk", C.c_int32),
                ("ray_tile", C.c_int32)]


class BatchDesc(C.Structure):
    _fields_ = [("nvol", C.c_int32), ("vols", C.POINTER(BatchVolume)), ("nview", C.c_int32),
                ("views", C.POINTER(BatchView)), ("fp", FeatureParams), ("tf", TF), ("rp", RenderParams),
                ("tune", C.POINTER(Tune))]


class DVRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libdvr.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.dvr_version.restype = i32
    L.dvr_last_error.restype = C.c_char_p
    L.dvr_normalize_workspace.argtypes = [i64, P(sz)]
    L.dvr_normalize.argtypes = [vp, i32, vp, i32, i64, vp, sz, vp]
    L.dvr_normalize_noalloc.argtypes = [vp, i32, vp, i32, i64, vp]
    L.dvr_features_workspace.argtypes = [P(Grid), P(FeatureParams), P(sz)]
    L.dvr_bricks_count.argtypes = [P(Grid), P(i64)]
    L.dvr_histogram.argtypes = [vp, i32, i64, C.c_float, vp, vp, vp]
    L.dvr_denoise_workspace.argtypes = [P(Grid), i32, P(sz)]
    L.dvr_denoise.argtypes = [vp, i32, P(Grid), i32, C.c_float, vp, vp, sz, vp]
    L.dvr_tissue_peaks.argtypes = [vp, i32, vp, vp]
    L.dvr_tissue_tf.argtypes = [vp, P(TissueTFParams), vp, vp, vp]
    L.dvr_bricks_bytes.argtypes = [P(Grid), P(sz)]
    L.dvr_features.argtypes = [vp, i32, P(Grid), P(FeatureParams), P(FeaturesBuf), vp, sz, vp]
    L.dvr_render.argtypes = [vp, i32, P(Grid), P(FeaturesBuf), P(TF), P(RenderParams), P(Camera), i32, vp,
                             P(RayState), vp]
    L.dvr_render_gather.argtypes = [vp, i32, P(Grid), P(FeaturesBuf), P(TF), P(RenderParams), P(Camera), i32, vp,
                                    vp, vp, vp]
    L.dvr_render_backward.argtypes = [vp, i32, P(Grid), P(FeaturesBuf), P(TF), P(RenderParams), P(Camera), i32,
                                      P(RayState), vp, vp, vp, vp]
    L.dvr_render_backward_features.argtypes = [vp, i32, P(Grid), P(FeaturesBuf), P(TF), P(RenderParams), P(Camera),
                                               i32, P(RayState), vp, vp, vp, P(FeatureGrads), vp]
    L.dvr_features_backward_workspace.argtypes = [P(Grid), P(FeatureParams), P(sz)]
    L.dvr_features_backward.argtypes = [vp, i32, P(Grid), P(FeatureParams), P(FeatureGrads), vp, vp, sz, vp]
    L.dvr_batch_create.argtypes = [P(BatchDesc), P(vp)]
    L.dvr_batch_launch.argtypes = [vp, vp]
    L.dvr_batch_check.argtypes = [vp, vp]
    L.dvr_batch_destroy.argtypes = [vp]
    L.dvr_batch_autotune.argtypes = [P(BatchDesc), C.c_char_p, P(Tune)]
    for name in ("dvr_normalize_workspace", "dvr_normalize", "dvr_normalize_noalloc", "dvr_features_workspace", "dvr_bricks_count", "dvr_bricks_bytes", "dvr_histogram", "dvr_denoise_workspace", "dvr_denoise", "dvr_tissue_peaks", "dvr_tissue_tf", "dvr_features",
                 "dvr_render", "dvr_render_gather", "dvr_render_backward", "dvr_render_backward_features", "dvr_features_backward_workspace",
                 "dvr_features_backward", "dvr_batch_create", "dvr_batch_launch", "dvr_batch_check",
                 "dvr_batch_destroy", "dvr_batch_autotune"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(status):
    if status != DVR_OK:
        raise DVRError(status, load().dvr_last_error().decode())


def declared_functions():
    """Names of the functions include/dvr.h declares (for the export check)."""
    import re
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(dvr_[a-z_0-9]+)\s*\(", text, flags=re.M)))
