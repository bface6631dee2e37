"""ctypes binding of libcfust.so (include/cfust.h).  Argument marshalling only:
every step of the E-step / M-step runs in the library's HIP kernels.

PyTorch is used for device memory and streams.  The library must be built
(``python -m paper_1606_02054_amd.build``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfust.so")

CFUST_FP64 = 0
CFUST_MIXED = 1
LATTICE_DIM = 8
MAX_P, MAX_Q, MAX_G, MAX_SHIFTS = 16, 8, 64, 64
NOALLOC_WS_BYTES = 64 << 20
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_LAYERS = 16, 256, 16, 5
MLP_K = [MLP_IN, MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN]
MLP_N = [MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN, MLP_OUT]

STATUS = {0: "CFUST_OK", -1: "CFUST_EINVAL", -2: "CFUST_ENOTSPD", -3: "CFUST_ENUMERIC",
          -4: "CFUST_EDEVICE", -5: "CFUST_ENOMEM", -6: "CFUST_EUNSUPPORTED"}

DEV_BITS = {1: "NOTSPD_OMEGA", 2: "NOTSPD_LAMBDA", 4: "BADPARAM", 8: "NOTSPD_E3",
            16: "NOTSPD_SIGMA", 32: "FROZEN", 64: "NU_CLAMPED"}

EXPORTS = ["cfust_create", "cfust_destroy", "cfust_last_error", "cfust_estep", "cfust_mstep",
           "cfust_loglik", "mvt_cdf_batch", "cfust_reserve", "cfust_profile_enable", "cfust_profile_read",
           "cfust_autotune", "cfust_mlp_forward", "cfust_mlp_backward", "cfust_mlp_adam",
           "cfust_mlp_loss", "cfust_mlp_features", "cfust_estep_surrogate", "cfust_batch_create",
           "cfust_batch_destroy", "cfust_batch_estep", "cfust_batch_mstep", "cfust_fit_batch", "cfust_batch_tune",
           "cfust_init", "cfust_estep_noalloc"]
MAX_FITS = 1024


class Dims(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("g", C.c_int32)]


class ParamsC(C.Structure):
    _fields_ = [("pi", C.c_void_p), ("mu", C.c_void_p), ("Sigma", C.c_void_p),
                ("Delta", C.c_void_p), ("nu", C.c_void_p)]


class QmcC(C.Structure):
    _fields_ = [("N", C.c_int32), ("S", C.c_int32), ("z", C.c_void_p), ("shifts", C.c_void_p),
                ("precision", C.c_int32)]


class EstepOutC(C.Structure):
    _fields_ = [("tau", C.c_void_p), ("logf_obs", C.c_void_p), ("loglik", C.c_void_p),
                ("w", C.c_void_p), ("e1", C.c_void_p), ("e2", C.c_void_p), ("e3", C.c_void_p),
                ("logf_comp", C.c_void_p), ("cdf_stderr", C.c_void_p), ("status", C.c_void_p)]


class FitC(C.Structure):
    _fields_ = [("dims", Dims), ("y", C.c_void_p), ("params", ParamsC), ("out", EstepOutC), ("status", C.c_void_p)]


class MlpWeightsC(C.Structure):
    _fields_ = [("W", C.c_void_p * MLP_LAYERS), ("Wt", C.c_void_p * MLP_LAYERS), ("b", C.c_void_p * MLP_LAYERS)]


class MlpActsC(C.Structure):
    _fields_ = [("X", C.c_void_p * MLP_LAYERS), ("XT", C.c_void_p * MLP_LAYERS), ("Z", C.c_void_p * (MLP_LAYERS - 1))]


class MlpGradsC(C.Structure):
    _fields_ = [("dW", C.c_void_p * MLP_LAYERS), ("db", C.c_void_p * MLP_LAYERS)]


class MlpMasterC(C.Structure):
    _fields_ = [(k, C.c_void_p * MLP_LAYERS) for k in ("W", "mW", "vW", "b", "mb", "vb")]


class SurrogateC(C.Structure):
    _fields_ = [("model", C.c_void_p * (MAX_Q + 1)), ("tol", C.c_float), ("n_fallback", C.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcfust.so and declare the C signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcfust.so not found at {path}: build it with "
                           "`python -m paper_1606_02054_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    vp, i32 = C.c_void_p, C.c_int32
    lib.cfust_create.restype = C.c_int; lib.cfust_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.cfust_destroy.restype = C.c_int; lib.cfust_destroy.argtypes = [vp]
    lib.cfust_last_error.restype = C.c_char_p; lib.cfust_last_error.argtypes = [vp]
    lib.cfust_estep.restype = C.c_int
    lib.cfust_estep.argtypes = [vp, vp, Dims, C.POINTER(ParamsC), C.POINTER(QmcC), C.POINTER(EstepOutC), vp]
    lib.cfust_estep_noalloc.restype = C.c_int
    lib.cfust_estep_noalloc.argtypes = [vp, vp, Dims, C.POINTER(ParamsC), C.POINTER(QmcC), C.POINTER(EstepOutC), vp]
    lib.cfust_mstep.restype = C.c_int
    lib.cfust_mstep.argtypes = [vp, vp, Dims, C.POINTER(EstepOutC), i32, C.POINTER(ParamsC),
                                C.POINTER(ParamsC), vp, vp]
    lib.cfust_loglik.restype = C.c_int
    lib.cfust_loglik.argtypes = [vp, vp, Dims, C.POINTER(ParamsC), C.POINTER(QmcC), vp, vp, vp, vp]
    lib.mvt_cdf_batch.restype = C.c_int
    lib.mvt_cdf_batch.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp, C.POINTER(QmcC), vp, vp, vp, vp]
    lib.cfust_reserve.restype = C.c_int
    lib.cfust_reserve.argtypes = [vp, Dims, C.POINTER(QmcC)]
    f = C.c_float
    lib.cfust_mlp_forward.restype = C.c_int
    lib.cfust_mlp_forward.argtypes = [vp, C.POINTER(MlpWeightsC), vp, i32, vp, C.POINTER(MlpActsC), vp]
    lib.cfust_mlp_backward.restype = C.c_int
    lib.cfust_mlp_backward.argtypes = [vp, C.POINTER(MlpWeightsC), C.POINTER(MlpActsC), vp, i32,
                                       C.POINTER(MlpGradsC), vp]
    lib.cfust_mlp_adam.restype = C.c_int
    lib.cfust_mlp_adam.argtypes = [vp, C.POINTER(MlpMasterC), C.POINTER(MlpGradsC), C.POINTER(MlpWeightsC),
                                   f, f, f, f, i32, vp]
    lib.cfust_mlp_loss.restype = C.c_int
    lib.cfust_mlp_loss.argtypes = [vp, vp, vp, i32, i32, f, vp, vp, vp]
    lib.cfust_mlp_features.restype = C.c_int
    lib.cfust_mlp_features.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.cfust_estep_surrogate.restype = C.c_int
    lib.cfust_estep_surrogate.argtypes = [vp, vp, Dims, C.POINTER(ParamsC), C.POINTER(QmcC), C.POINTER(SurrogateC),
                                          C.POINTER(EstepOutC), vp]
    lib.cfust_autotune.restype = C.c_int
    lib.cfust_autotune.argtypes = [vp, vp, Dims, C.POINTER(ParamsC), C.POINTER(QmcC), C.POINTER(C.c_int32), vp]
    lib.cfust_batch_create.restype = C.c_int
    lib.cfust_batch_create.argtypes = [vp, i32, C.POINTER(FitC), C.POINTER(QmcC), C.POINTER(vp)]
    lib.cfust_batch_destroy.restype = C.c_int; lib.cfust_batch_destroy.argtypes = [vp]
    lib.cfust_batch_estep.restype = C.c_int; lib.cfust_batch_estep.argtypes = [vp, vp]
    lib.cfust_batch_mstep.restype = C.c_int; lib.cfust_batch_mstep.argtypes = [vp, vp]
    lib.cfust_fit_batch.restype = C.c_int
    lib.cfust_fit_batch.argtypes = [vp, i32, C.c_double, i32, vp, vp, vp]
    lib.cfust_batch_tune.restype = C.c_int
    lib.cfust_batch_tune.argtypes = [vp, C.POINTER(C.c_int32), vp]
    lib.cfust_init.restype = C.c_int
    lib.cfust_init.argtypes = [vp, vp, Dims, i32, vp, i32, C.POINTER(C.c_double), C.c_double, C.POINTER(QmcC),
                               C.POINTER(ParamsC), vp, vp, vp]
    lib.cfust_profile_enable.restype = C.c_int
    lib.cfust_profile_enable.argtypes = [vp, C.c_int]
    lib.cfust_profile_read.restype = C.c_int
    lib.cfust_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    _lib = lib
    return lib


def exported_symbols(path: str = LIB_PATH):
    """Names of the C-ABI entry points that resolve in the library (no GPU needed)."""
    lib = C.CDLL(path)
    found = []
    for name in EXPORTS:
        try:
            getattr(lib, name)
            found.append(name)
        except AttributeError:
            pass
    return found


def check(status: int, handle=None, what: str = "") -> None:
    if status != 0:
        msg = ""
        if handle is not None and _lib is not None:
            m = _lib.cfust_last_error(handle)
            msg = m.decode() if m else ""
        raise RuntimeError(f"{what}: {STATUS.get(status, status)} {msg}")
