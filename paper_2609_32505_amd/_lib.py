"""ctypes declarations of the C ABI in ``include/svdp.h`` (argument
marshalling only; every step of the method runs in ``libsvdp.so``)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsvdp.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_flt = ctypes.c_float
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t

SVDP_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "bad shape", 3: "workspace too small",
          4: "HIP error", 5: "no model loaded"}

PREC_FP32, PREC_BF16 = 0, 1
BOUND_CONSERVATIVE, BOUND_LEARNED, BOUND_USER = 0, 1, 2
POLY_CANS3, POLY_NS, POLY_CANS5, POLY_PE = 0, 1, 2, 3
FLAG_NOT_CONVERGED = 1
FLAG_FALLBACK_USED = 2
FLAG_NEG_EIGENVALUE = 4
FLAG_RANK_DEFICIENT = 8
FLAG_NONFINITE = 16
FLAG_EIGH_NOT_CONVERGED = 32
OP_SVD_FWD, OP_SVD_BWD, OP_POLAR_FWD, OP_POLAR_BWD, OP_EIGH, OP_FEATURES, OP_EIGH_BWD, OP_EIGH_DC = range(8)
MLP_PARAMS = 4866
MODEL_FLOATS = MLP_PARAMS + 16


class Params(ctypes.Structure):
    _fields_ = [
        ("batch", c_i64), ("m", c_i64), ("n", c_i64),
        ("precision", c_i32), ("bound", c_i32),
        ("max_iters", c_i32), ("pre_iters", c_i32), ("refine_steps", c_i32),
        ("max_sweeps", c_i32), ("inner_sweeps", c_i32), ("fp64_sweeps", c_i32),
        ("delta", c_dbl), ("tol", c_dbl), ("eps_qr", c_dbl), ("bf16_handoff", c_dbl),
        ("refine_tol", c_dbl), ("jacobi_tol", c_dbl), ("jacobi_abs", c_dbl), ("bf16_from", c_dbl),
        ("eps_K", c_dbl), ("eps_R", c_dbl), ("eps_T", c_dbl),
        ("margin_max", c_dbl), ("margin_min", c_dbl),
        ("user_bounds", c_vp), ("probe", c_vp),
        ("eigh_off_tol", c_dbl), ("eigh_restarts", c_i32), ("jacobi_fro_tol", c_dbl), ("poly", c_i32),
        ("bf16_correct", c_i32), ("pe_lo", c_dbl), ("tall_qr", c_i32),
    ]


class Info(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("sweeps", c_i32), ("flags", c_i32), ("residual", c_flt)]


# (name, restype, argtypes) of every exported function of svdp.h
SIGNATURES = {
    "svdp_default_params": (None, [ctypes.POINTER(Params), c_i64, c_i64, c_i64]),
    "svdp_create": (c_i32, [ctypes.POINTER(c_vp)]),
    "svdp_destroy": (c_i32, [c_vp]),
    "svdp_set_model": (c_i32, [c_vp, c_vp]),
    "svdp_workspace_size": (c_i32, [ctypes.POINTER(Params), c_i32, ctypes.POINTER(c_sz)]),
    "svdp_status_string": (ctypes.c_char_p, [c_i32]),
    "svdp_last_error": (ctypes.c_char_p, []),
    "svdp_host_syncs": (c_i64, []),
    "svd_polar_fwd": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64, c_i64,
                              c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "svd_polar_bwd": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64,
                              c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64,
                              c_i64, c_vp, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "svd_polar_bwd_noalloc": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64,
                                      c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64,
                                      c_i64, c_vp, c_i64, c_i64, c_vp]),
    "polar_fwd": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64, c_i64,
                          c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp, c_sz,
                          c_vp]),
    "polar_bwd": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64, c_i64,
                          c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64,
                          c_vp, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "svdp_eigh": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64, c_vp,
                          c_i64, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "svdp_eigh_dc": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_i64, c_vp,
                             c_i64, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "svdp_eigh_bwd": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64,
                              c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "svdp_bound_features": (c_i32, [c_vp, ctypes.POINTER(Params), c_vp, c_i64, c_i64, c_vp, c_vp,
                                    c_vp, c_vp, c_sz, c_vp]),
    "svdp_spectral_features": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "svdp_training_targets": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "svdp_feature_stats": (c_i32, [c_vp, c_i64, c_vp, c_vp, c_vp]),
    "svdp_mlp_fwd": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "svdp_mlp_bwd_ws_bytes": (c_sz, [c_i64]),
    "svdp_mlp_bwd": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "svdp_pinball": (c_i32, [c_vp, c_vp, c_i64, c_flt, c_flt, c_vp, c_vp, c_vp]),
    "svdp_adam_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_flt, c_flt, c_flt, c_flt, c_i64,
                               c_vp]),
    "svdp_cans_table": (c_i32, [c_i32, c_dbl, c_i32, c_dbl, c_i32, ctypes.POINTER(c_dbl),
                                ctypes.POINTER(c_dbl)]),
    "svdp_poly_table": (c_i32, [c_i32, c_dbl, c_i32, c_i32, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]),
    "svdp_pe_table": (c_i32, [c_dbl, c_i32, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i32)]),
    "svdp_profile_enable": (None, [ctypes.c_int]),
    "svdp_profile_reset": (None, []),
    "svdp_profile_read": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64),
                                         ctypes.POINTER(c_dbl)]),
}
PROF_KINDS = {"jac_solve_f32": 0, "jac_solve_f64": 1, "jac_apply": 2, "gemm_f32": 3, "gemm_bf16": 4,
              "jac_vsweep": 14}
PROF_PHASES = {"bound": 5, "cans": 6, "refine": 7, "H": 8, "eigh": 9, "U": 10, "fallback": 11, "backward": 12,
               "qr": 13}

_lib = None


class SvdpError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load ``libsvdp.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise SvdpError(f"{path} is missing: build it with `python -m paper_2609_32505_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, what: str = ""):
    if status != SVDP_OK:
        msg = load().svdp_last_error().decode()
        raise SvdpError(f"{what}: {STATUS.get(status, status)} ({msg})")


def default_params(batch: int, m: int, n: int, **kw) -> Params:
    p = Params()
    load().svdp_default_params(ctypes.byref(p), batch, m, n)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p
