"""ctypes declarations of the C-ABI in include/fwi.h.

Loads ``libfwi.so`` from this package directory, or from the path in the
environment variable ``FWI_LIBRARY`` (another build of the same sources, for
instance one made with different tuning macros by ``build.py --out``).  There
is no fallback: if the library is missing, loading raises ``FwiLibraryMissing``.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int8, c_int32, c_int64, c_uint8, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FWI_LIBRARY") or os.path.join(HERE, "libfwi.so")

FWI_OK = 0
FWI_ERR_INVALID_ARG = 1
FWI_ERR_UNSUPPORTED = 2
FWI_ERR_OOM = 3
FWI_ERR_NO_TAPE = 4
FWI_ERR_HIP = 5
FWI_ERR_UNSTABLE = 6

FWI_SAVE_TAPE = 1
FWI_CHECK_INPUT = 2
FWI_CHECK_FINITE = 4
FWI_TR_FINAL_STATE = 8
FWI_GRAPH = 16
FWI_MEAN = 32
FWI_EXACT = 64

FWI_NOALLOC_MAX_PAIRS = 256   # static scratch of fwi_lbfgs_apply_noalloc

SUPPORTED_LENGTHS = (8, 12, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128, 160, 192, 224, 240, 256, 320, 384, 448,
                     480, 512)

# every symbol declared in include/fwi.h
EXPORTED = (
    "fwi_create", "fwi_destroy", "fwi_workspace_bytes", "fwi_rademacher", "fwi_delays", "fwi_forward",
    "fwi_gradient", "fwi_backward", "fwi_derivative", "fwi_get_tuning", "fwi_set_tuning",
    "fwi_set_absorption", "fwi_set_delays",
    "fwi_timing_enable", "fwi_timing_read", "fwi_gamma_size", "fwi_gamma_gather", "fwi_gamma_scatter",
    "fwi_lbfgs_create", "fwi_lbfgs_destroy", "fwi_lbfgs_push", "fwi_lbfgs_apply", "fwi_lbfgs_apply_noalloc",
    "fwi_lbfgs_count",
    "fwi_vec_axpby", "fwi_vec_clip", "fwi_vec_sqslowness", "fwi_interp_fourier", "fwi_resample_time",
    "fwi_status_string", "fwi_last_error",
)

PASS_NAMES = ("y_fwd", "y_inv", "z_plus", "z_minus", "x_vel", "x_den_fwd", "x_den_pair", "y_vel_q")
PASS_KERNELS = ("k_axis_y<*, false, *>", "k_axis_y<*, true, *>", "k_axis_z_plus", "k_axis_z_minus",
                "k_x_velocity", "k_x_density<*, 0, *>", "k_x_density<*, 1, *>", "k_axis_y_vel")


class FwiLibraryMissing(ImportError):
    pass


class FwiParams(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("dx", c_double), ("dt", c_double), ("c_ref", c_double),
        ("c_min", c_double), ("c_max", c_double), ("rho0", c_double),
        ("pml", c_int32 * 3), ("pml_alpha", c_double),
        ("nt", c_int32), ("precision", c_int32), ("batch", c_int32),
    ]


class FwiGeometry(ctypes.Structure):
    _fields_ = [
        ("n_src", c_int32), ("src_ijk", POINTER(c_int32)),
        ("n_rec", c_int32), ("rec_ijk", POINTER(c_int32)),
        ("gamma_mask", POINTER(c_uint8)), ("boundary_mask", POINTER(c_uint8)),
    ]


class FwiTuning(ctypes.Structure):
    _fields_ = [("y_tile_bytes", c_int32), ("zm_tile_bytes", c_int32), ("zp_tile_bytes", c_int32),
                ("y_plan", c_int32), ("zm_plan", c_int32), ("zp_plan", c_int32), ("x_plan", c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load and declare the library (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FwiLibraryMissing(
            f"{path} not found: build it with `python -m paper_2102_00755_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    h = c_void_p
    lib.fwi_create.argtypes = [POINTER(FwiParams), POINTER(FwiGeometry), c_int, POINTER(c_void_p)]
    lib.fwi_create.restype = c_int
    lib.fwi_destroy.argtypes = [h]
    lib.fwi_destroy.restype = None
    lib.fwi_workspace_bytes.argtypes = [POINTER(FwiParams), POINTER(FwiGeometry)]
    lib.fwi_workspace_bytes.restype = c_int64
    lib.fwi_rademacher.argtypes = [c_uint64, c_int32, POINTER(c_int8)]
    lib.fwi_rademacher.restype = c_int
    lib.fwi_delays.argtypes = [c_uint64, c_int32, c_int32, POINTER(c_int32)]
    lib.fwi_delays.restype = c_int
    lib.fwi_forward.argtypes = [h, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.fwi_forward.restype = c_int
    lib.fwi_gradient.argtypes = [h, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int32, c_void_p]
    lib.fwi_gradient.restype = c_int
    lib.fwi_backward.argtypes = [h, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.fwi_backward.restype = c_int
    lib.fwi_derivative.argtypes = [h, c_void_p, c_void_p, c_int32, c_int32, c_void_p]
    lib.fwi_derivative.restype = c_int
    lib.fwi_get_tuning.argtypes = [h, POINTER(FwiTuning)]
    lib.fwi_get_tuning.restype = c_int
    lib.fwi_set_tuning.argtypes = [h, POINTER(FwiTuning)]
    lib.fwi_set_tuning.restype = c_int
    lib.fwi_set_absorption.argtypes = [h, c_double, c_double, c_void_p, c_int32]
    lib.fwi_set_absorption.restype = c_int
    lib.fwi_set_delays.argtypes = [h, c_int32, POINTER(c_int32)]
    lib.fwi_set_delays.restype = c_int
    lib.fwi_gamma_size.argtypes = [h, POINTER(c_int64)]
    lib.fwi_gamma_size.restype = c_int
    lib.fwi_gamma_gather.argtypes = [h, c_void_p, c_void_p, c_void_p]
    lib.fwi_gamma_gather.restype = c_int
    lib.fwi_gamma_scatter.argtypes = [h, c_void_p, c_void_p, c_void_p]
    lib.fwi_gamma_scatter.restype = c_int
    lib.fwi_lbfgs_create.argtypes = [c_int64, c_int32, c_int32, c_int32, POINTER(c_void_p)]
    lib.fwi_lbfgs_create.restype = c_int
    lib.fwi_lbfgs_destroy.argtypes = [c_void_p]
    lib.fwi_lbfgs_destroy.restype = None
    lib.fwi_lbfgs_push.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.fwi_lbfgs_push.restype = c_int
    lib.fwi_lbfgs_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_void_p]
    lib.fwi_lbfgs_apply.restype = c_int
    lib.fwi_lbfgs_apply_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_void_p]
    lib.fwi_lbfgs_apply_noalloc.restype = c_int
    lib.fwi_lbfgs_count.argtypes = [c_void_p, POINTER(c_int32)]
    lib.fwi_lbfgs_count.restype = c_int
    lib.fwi_vec_axpby.argtypes = [c_int64, c_double, c_void_p, c_double, c_void_p, c_int32, c_void_p]
    lib.fwi_vec_axpby.restype = c_int
    lib.fwi_vec_clip.argtypes = [c_int64, c_void_p, c_double, c_double, c_int32, c_void_p]
    lib.fwi_vec_clip.restype = c_int
    lib.fwi_vec_sqslowness.argtypes = [c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]
    lib.fwi_vec_sqslowness.restype = c_int
    lib.fwi_interp_fourier.argtypes = [h, h, c_void_p, c_void_p, c_int32, c_void_p]
    lib.fwi_interp_fourier.restype = c_int
    lib.fwi_resample_time.argtypes = [c_int32, c_int32, c_void_p, c_double, c_int32, c_double, c_double, c_double,
                                      c_double, c_double, c_void_p, c_int32, c_void_p]
    lib.fwi_resample_time.restype = c_int
    lib.fwi_timing_enable.argtypes = [h, c_int32]
    lib.fwi_timing_enable.restype = c_int
    lib.fwi_timing_read.argtypes = [h, c_int32, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]
    lib.fwi_timing_read.restype = c_int
    lib.fwi_status_string.argtypes = [c_int]
    lib.fwi_status_string.restype = c_char_p
    lib.fwi_last_error.argtypes = []
    lib.fwi_last_error.restype = c_char_p
    _lib = lib
    return lib
