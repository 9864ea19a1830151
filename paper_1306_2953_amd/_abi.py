"""ctypes declarations of librsdft.so (the C ABI in include/rsdft.h).

Argument marshalling only: every computation runs inside the library.  The
library must be built (``python -m paper_1306_2953_amd.build``); importing a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsdft.so")

RS_OK, RS_EINVAL, RS_ENOTPOSDEF, RS_ENONFINITE, RS_EHIP, RS_ENOMEM, RS_ENOTSUP, RS_ENOTCONV = range(8)
RS_CNN_NPARAM = 2162
RS_F64, RS_F32 = 0, 1
RS_C128, RS_C64 = 2, 3          # complex states, (re, im) interleaved
RS_PREC_NATIVE, RS_PREC_BF16X3 = 0, 1
RS_GRID_BOX, RS_GRID_PERIODIC, RS_GRID_SPHERE, RS_GRID_UNION = 0, 1, 2, 3
RS_GRID_HOST_ONLY = 1

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F64 = ctypes.c_double
PI32 = ctypes.POINTER(ctypes.c_int32)
PI64 = ctypes.POINTER(ctypes.c_int64)
PF64 = ctypes.POINTER(ctypes.c_double)


class SolverOpts(ctypes.Structure):
    _fields_ = [("m", I32), ("alpha", F64), ("tol", F64), ("block_stop", I32), ("record", I32),
                ("rr_sweeps", I32)]


class ScfOpts(ctypes.Structure):
    _fields_ = [("nocc", I32), ("eig_steps", I32), ("history", I32), ("mix", F64), ("solver", SolverOpts)]


class SolverStats(ctypes.Structure):
    _fields_ = [("steps", I32), ("rr_sweeps", I32), ("frozen_blocks", I32), ("net_states", I32)]


class GridDesc(ctypes.Structure):
    _fields_ = [("kind", I32), ("h", F64), ("n", I32), ("radius", F64),
                ("brick", I32 * 3), ("flags", I32), ("natoms", I32), ("centres", P)]


# name -> (restype, argtypes); the list of exported entry points
SIGNATURES = {
    "rs_last_error": (ctypes.c_char_p, []),
    "rs_version": (ctypes.c_int, []),
    "rs_grid_create": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(P)]),
    "rs_grid_destroy": (None, [P]),
    "rs_grid_info": (ctypes.c_int, [P, PI64, PI64, PI64, PI32, PI32]),
    "rs_grid_export": (ctypes.c_int, [P, P, P, P, P]),
    "rs_nl_create": (ctypes.c_int, [P, I32, P, P, F64, F64, I32, I32, ctypes.POINTER(P)]),
    "rs_nl_destroy": (None, [P]),
    "rs_nl_info": (ctypes.c_int, [P, PI64, PI32, PI32]),
    "rs_nl_export": (ctypes.c_int, [P, P, P, P, P]),
    "rs_hpsi_block": (ctypes.c_int, [P, P, P, P, P, I32, I32, I32, P]),
    "rs_project_nl": (ctypes.c_int, [P, P, P, P, I32, I32, I32, P]),
    "rs_apply_nl": (ctypes.c_int, [P, P, P, P, I32, I32, I32, P]),
    "rs_ctx_create": (ctypes.c_int, [P, I32, ctypes.POINTER(P)]),
    "rs_ctx_destroy": (None, [P]),
    "rs_overlap": (ctypes.c_int, [P, P, P, P, I32, I32, I32, I32, P]),
    "rs_overlap_noalloc": (ctypes.c_int, [P, P, P, P, I32, I32, I32, I32, P]),
    "rs_rotate": (ctypes.c_int, [P, P, P, I32, I32, I32, I32, P]),
    "rs_cholesky": (ctypes.c_int, [P, P, P, I32, P, P]),
    "rs_eigh": (ctypes.c_int, [P, P, P, P, I32, P]),
    "rs_orthonormalize_block": (ctypes.c_int, [P, P, I32, I32, I32, I32, P, PI32, P]),
    "rs_subspace_diag": (ctypes.c_int, [P, P, P, P, I32, I32, I32, I32, P]),
    "rs_eigensolve_create": (ctypes.c_int, [P, P, P, I32, I32, I32, P, ctypes.POINTER(P)]),
    "rs_eigensolve_destroy": (None, [P]),
    "rs_eigensolve_step": (ctypes.c_int, [P, P, PF64, PF64, PI32, P]),
    "rs_eigensolve_set_precond": (ctypes.c_int, [P, P]),
    "rs_eigensolve_orthonormalize": (ctypes.c_int, [P, P, P]),
    "rs_eigensolve_residuals": (ctypes.c_int, [P, P, P, P]),
    "rs_eigensolve_stats": (ctypes.c_int, [P, P]),
    "rs_cnn_create": (ctypes.c_int, [I32, I64, ctypes.POINTER(P)]),
    "rs_cnn_destroy": (None, [P]),
    "rs_cnn_set_params": (ctypes.c_int, [P, P]),
    "rs_cnn_get_params": (ctypes.c_int, [P, P]),
    "rs_cnn_save": (ctypes.c_int, [P, ctypes.c_char_p]),
    "rs_cnn_load": (ctypes.c_int, [P, ctypes.c_char_p]),
    "rs_cnn_forward": (ctypes.c_int, [P, P, P, I32, PI32, I32, P]),
    "rs_cnn_loss_grad": (ctypes.c_int, [P, P, P, P, I32, PI32, F64, I32, PF64, P, P, P]),
    "rs_cnn_adam_step": (ctypes.c_int, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]),
    "rs_cnn_precondition": (ctypes.c_int, [P, P, P, P, P, I32, I32, I32, P]),
    "rs_cnn_box": (ctypes.c_int, [P, P, PI32]),
    "rs_cnn_crops": (ctypes.c_int, [P, P, P, P, I32, I32, I32, I32, P, PI32, P, P, P]),
    "rs_poisson_create": (ctypes.c_int, [P, ctypes.POINTER(P)]),
    "rs_poisson_destroy": (None, [P]),
    "rs_poisson_info": (ctypes.c_int, [P, PI32, PF64]),
    "rs_poisson_solve": (ctypes.c_int, [P, P, P, P]),
    "rs_scf_create": (ctypes.c_int, [P, P, P, I32, I32, I32, P, ctypes.POINTER(P)]),
    "rs_scf_destroy": (None, [P]),
    "rs_scf_start": (ctypes.c_int, [P, P, P]),
    "rs_scf_iterate": (ctypes.c_int, [P, P, PF64, PF64, PF64, P]),
    "rs_scf_density": (ctypes.c_int, [P, P, P, P]),
    "rs_shifted_solve": (ctypes.c_int, [P, P, P, P, I32, I32, I32, F64, I32, PI32, P]),
}

_lib = None


class RsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rsdft error {code}: {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1306_2953_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != RS_OK:
        raise RsError(code, lib().rs_last_error().decode(errors="replace"))
