"""ctypes declarations of libfdcgks.so (the C ABI in include/fdcgks.h).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FDCGKS_LIB may point at another build of the same library (A/B timing).
LIB_PATH = os.environ.get("FDCGKS_LIB") or os.path.join(HERE, "libfdcgks.so")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS, ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONPHYS", -5: "ESTATE"}
BC_PERIODIC, BC_ZERO_GRADIENT, BC_REFLECTING, BC_NO_SLIP = 0, 1, 2, 3
FLUX_6_4, FLUX_6_2, FLUX_LINEAR = 0, 1, 2
FP64, FP32_FLUX = 0, 1
GRAD_REEVAL, GRAD_CARRIED = 0, 1
RECON_CONSERVATIVE, RECON_CHARACTERISTIC = 0, 1
OPT_GRAPH, OPT_TILE_EDGE, OPT_TILE_NODE, OPT_TILE_UPDATE, OPT_FUSE_NODES, OPT_FUSE_STAGE, OPT_FUSED_ROWS = \
    0, 1, 2, 3, 4, 5, 6
BATCH_PERSISTENT, BATCH_PHASED, BATCH_GRAPH = 0, 1, 2


class Params(C.Structure):
    """Mirror of fdcgks_params."""
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32),
        ("dual_1d", C.c_int32), ("flux_variant", C.c_int32), ("flux_precision", C.c_int32),
        ("grad_update", C.c_int32), ("geno_r", C.c_int32), ("recon_vars", C.c_int32), ("flux_order", C.c_int32),
        ("side", C.c_int32 * 4),
        ("x0", C.c_double), ("lx", C.c_double), ("y0", C.c_double), ("ly", C.c_double),
        ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
        ("geno_C", C.c_double), ("geno_eps", C.c_double), ("geno_eps_a", C.c_double),
        ("geno_d_central", C.c_double), ("geno_d_side", C.c_double),
        ("tau_c1", C.c_double), ("tau_c2", C.c_double),
    ]


class Params3D(C.Structure):
    """Mirror of fdcgks3d_params."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("flux_variant", C.c_int32),
        ("flux_order", C.c_int32), ("grad_update", C.c_int32), ("geno_r", C.c_int32), ("recon_vars", C.c_int32),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double), ("lx", C.c_double),
        ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
        ("geno_C", C.c_double), ("geno_eps", C.c_double), ("geno_eps_a", C.c_double),
        ("geno_d_central", C.c_double), ("geno_d_side", C.c_double),
        ("tau_c1", C.c_double), ("tau_c2", C.c_double),
    ]


class FdcgksError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fdcgks {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# name -> (restype, argtypes); every symbol include/fdcgks.h declares
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_i32 = C.c_int32
SIGNATURES = {
    "fdcgks_default_params": (None, [C.POINTER(Params)]),
    "fdcgks_create": (C.c_int, [C.POINTER(Params), _vp, C.POINTER(_vp)]),
    "fdcgks_set_state": (C.c_int, [_vp, _i32, _vp, _vp, _vp, C.c_int64, _i32]),
    "fdcgks_get_state": (C.c_int, [_vp, _i32, _vp, _vp, _vp, C.c_int64, _i32]),
    "fdcgks_set_state_from_samples": (C.c_int, [_vp, _vp, _i32]),
    "fdcgks_compute_dt": (C.c_int, [_vp, C.c_double, _dp]),
    "fdcgks_diagnostics": (C.c_int, [_vp, _dp]),
    "fdcgks_step": (C.c_int, [_vp, C.c_double, C.c_double, _i32, C.c_double, _dp, C.POINTER(_i32)]),
    "fdcgks_step_timed": (C.c_int, [_vp, C.c_double, C.c_double, _i32, C.c_double, _dp, C.POINTER(_i32), _dp]),
    "fdcgks_step1d_static": (C.c_int, [C.POINTER(Params), _vp, C.c_double, C.c_double, _i32, C.c_double, _dp,
                                       C.POINTER(_i32), _vp]),
    "fdcgks_destroy": (C.c_int, [_vp]),
    "fdcgks_last_error": (C.c_char_p, [_vp]),
    "fdcgks_debug_stage": (C.c_int, [_vp, _i32, C.c_double, _vp, _vp]),
    "fdcgks_debug_intermediates": (C.c_int, [_vp, C.c_double, _vp, _vp, _vp, _vp]),
    "fdcgks_step_vjp": (C.c_int, [_vp, C.c_double, _vp, _vp, _i32]),
    "fdcgks_set_option": (C.c_int, [_vp, _i32, C.c_int64]),
    "fdcgks_get_option": (C.c_int, [_vp, _i32, C.POINTER(C.c_int64)]),
    "fdcgks_autotune": (C.c_int, [_vp, _i32]),
    "fdcgks_batch_create": (C.c_int, [_i32, C.POINTER(Params), _vp, C.POINTER(_vp)]),
    "fdcgks_batch_set_state": (C.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i32]),
    "fdcgks_batch_get_state": (C.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _i32]),
    "fdcgks_batch_step": (C.c_int, [_vp, C.c_double, _i32, _dp, _dp, C.POINTER(_i32)]),
    "fdcgks_batch_destroy": (C.c_int, [_vp]),
    "fdcgks_batch_last_error": (C.c_char_p, [_vp]),
    "fdcgks_batch_set_mode": (C.c_int, [_vp, _i32]),
    # 3D (include/fdcgks3d.h)
    "fdcgks3d_default_params": (None, [C.POINTER(Params3D)]),
    "fdcgks3d_create": (C.c_int, [C.POINTER(Params3D), _vp, C.POINTER(_vp)]),
    "fdcgks3d_set_state": (C.c_int, [_vp, _i32, _vp, _i32]),
    "fdcgks3d_get_state": (C.c_int, [_vp, _i32, _vp, _i32]),
    "fdcgks3d_compute_dt": (C.c_int, [_vp, C.c_double, _dp]),
    "fdcgks3d_diagnostics": (C.c_int, [_vp, _dp]),
    "fdcgks3d_step": (C.c_int, [_vp, C.c_double, C.c_double, _i32, C.c_double, _dp, C.POINTER(_i32)]),
    "fdcgks3d_step_timed": (C.c_int, [_vp, C.c_double, C.c_double, _i32, C.c_double, _dp, C.POINTER(_i32), _dp]),
    "fdcgks3d_debug_stage": (C.c_int, [_vp, _i32, C.c_double, _vp, _vp]),
    "fdcgks3d_debug_intermediates": (C.c_int, [_vp, C.c_double, _vp, _vp]),
    "fdcgks3d_destroy": (C.c_int, [_vp]),
    "fdcgks3d_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def load():
    """Load libfdcgks.so; raises if it is missing (build it with
    ``python -m paper_2606_17772_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library has not been built "
                          "(python -m paper_2606_17772_amd.build)")
    # One HIP runtime per process: let torch load (and initialise) its HIP
    # runtime first, so that libfdcgks.so binds to the same libamdhip64 and
    # torch's streams and device pointers are valid handles for it.
    try:
        import torch  # noqa: PLC0415
        torch.cuda.is_available()
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status, handle=None, batch=False, dim3=False):
    if status != OK:
        L = load()
        msg = (L.fdcgks_batch_last_error if batch else
               L.fdcgks3d_last_error if dim3 else L.fdcgks_last_error)(handle)
        raise FdcgksError(status, msg.decode() if msg else "")
    return status
