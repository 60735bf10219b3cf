"""ctypes declarations of the C ABI in ``include/bttb.h``.

Argument marshalling only.  Loading fails loudly when ``libbttb.so`` is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbttb.so")

BTTB_OK, BTTB_EINVAL, BTTB_ENOMEM, BTTB_EHIP, BTTB_ESIZE, BTTB_ESTATE, BTTB_ENAN = 0, -1, -2, -3, -4, -5, -6
BTTB_F64, BTTB_F32 = 0, 1
BTTB_GRAVITY, BTTB_MAGNETIC = 0, 1
BTTB_OP_FORWARD, BTTB_OP_ADJOINT = 0, 1
BTTB_ANCHOR_APR, BTTB_ANCHOR_PREV = 0, 1
BTTB_PAD_POW2 = 0x10
BTTB_PAD_AUTO = 0x40
BTTB_EIG_FULL = 0x20
MAX_TRANSFORM = 2048
NOALLOC_MAX_SCRATCH = 32 << 20

EXPORTED = [
    "bttb_prism_kernels", "bttb_setup", "bttb_matvec", "bttb_rmatvec", "bttb_apply", "bttb_set_launch",
    "bttb_plan_info", "bttb_plan_eigenvalues", "bttb_destroy", "rrcg_create", "rrcg_step",
    "rrcg_read_scalars", "rrcg_write_scalars", "rrcg_refresh", "rrcg_destroy", "bttb_strerror",
    "bttb_last_error", "bttb_timing_enable", "bttb_timing_read",
    "bttb_group_create", "bttb_group_apply", "bttb_group_set_launch", "bttb_group_info", "bttb_group_destroy",
    "rrcg_group_create", "rrcg_group_step", "rrcg_group_read_scalars", "rrcg_group_write_scalars",
    "rrcg_group_refresh", "rrcg_group_set_launch", "rrcg_group_products", "rrcg_group_destroy",
    "bttb_autotune", "bttb_group_autotune", "rrcg_group_autotune", "bttb_group_timing_enable",
    "bttb_group_timing_read", "rrcg_products", "rrcg_autotune", "rrcg_prepare", "rrcg_group_prepare",
    "bttb_group_timing_list", "bttb_apply_noalloc",
]
NKERNELS = 6
KERNEL_NAMES = ["fwd_row_r2c", "fwd_col_eig_sum", "fwd_row_c2r", "adj_row_r2c", "adj_col_conj_eig", "adj_row_c2r"]


class BTTBError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("sx", C.c_int), ("sy", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("height", C.c_double),
                ("top", C.c_double), ("incl_deg", C.c_double), ("decl_deg", C.c_double),
                ("field_nt", C.c_double), ("ox", C.c_int), ("oy", C.c_int)]


class PlanDesc(C.Structure):
    _fields_ = [("sx", C.c_int), ("sy", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("Px", C.c_int), ("Py", C.c_int), ("precision", C.c_int), ("max_batch", C.c_int),
                ("eig_bytes", C.c_size_t), ("scratch_bytes", C.c_size_t), ("col_fft_per_block", C.c_int),
                ("row_fft_per_block", C.c_int), ("layer_chunks", C.c_int), ("eig_real_even", C.c_int)]


class GroupDesc(C.Structure):
    _fields_ = [("count", C.c_int), ("precision", C.c_int), ("model_row_threads", C.c_int),
                ("data_row_threads", C.c_int), ("col_threads", C.c_int), ("layer_chunks", C.c_int),
                ("blocks", C.c_int * 6)]


class TuneResult(C.Structure):
    _fields_ = [("us_per_pair", C.c_double), ("shape", C.c_int * 4), ("tried", C.c_int)]


class RrcgDesc(C.Structure):
    _fields_ = [("plan", C.c_void_p * 2), ("m", C.c_void_p * 2), ("p", C.c_void_p * 2),
                ("resid", C.c_void_p * 2), ("dobs", C.c_void_p * 2), ("wd", C.c_void_p * 2),
                ("wdepth", C.c_void_p * 2), ("whard", C.c_void_p * 2), ("mapr", C.c_void_p * 2),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2), ("alpha0", C.c_double * 2),
                ("q", C.c_double * 2), ("alpha_min", C.c_double * 2), ("lambda_", C.c_double * 2),
                ("eps2", C.c_double), ("coupled", C.c_int), ("restart", C.c_int), ("p_norm", C.c_int),
                ("gramian_weighted", C.c_int), ("use_graph", C.c_int), ("anchor", C.c_int),
                ("mprev", C.c_void_p * 2)]


class RrcgScalars(C.Structure):
    _fields_ = [("alpha", C.c_double * 2), ("L_prev", C.c_double * 2), ("phi", C.c_double * 2),
                ("threshold", C.c_double), ("beta", C.c_double * 2), ("step", C.c_double * 2),
                ("gramian", C.c_double), ("frozen", C.c_int * 2), ("k", C.c_int), ("converged", C.c_int),
                ("nonfinite", C.c_int), ("similarity", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library (loaded once).  Raises ImportError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2112_15562_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i, d, ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
    sig = {
        "bttb_prism_kernels": [i, C.POINTER(Geometry), vp, vp],
        "bttb_setup": [vp, i, i, i, i, i, i, i, vp, C.POINTER(vp)],
        "bttb_matvec": [vp, vp, vp, vp],
        "bttb_rmatvec": [vp, vp, vp, vp],
        "bttb_apply": [vp, i, i, vp, ll, vp, ll, vp, vp, vp],
        "bttb_set_launch": [vp, i, i, i],
        "bttb_plan_info": [vp, C.POINTER(PlanDesc)],
        "bttb_plan_eigenvalues": [vp, vp, vp],
        "bttb_destroy": [vp],
        "rrcg_create": [C.POINTER(RrcgDesc), vp, C.POINTER(vp)],
        "rrcg_step": [vp, i, vp],
        "rrcg_read_scalars": [vp, C.POINTER(RrcgScalars), vp],
        "rrcg_write_scalars": [vp, C.POINTER(RrcgScalars), vp],
        "rrcg_refresh": [vp, vp],
        "rrcg_destroy": [vp],
        "bttb_timing_enable": [vp, i, i],
        "bttb_timing_read": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)],
        "bttb_group_create": [C.POINTER(vp), i, vp, C.POINTER(vp)],
        "bttb_group_apply": [vp, i, vp, vp, vp, vp, vp],
        "bttb_group_set_launch": [vp, i, i, i, i, vp],
        "bttb_group_info": [vp, C.POINTER(GroupDesc)],
        "bttb_group_destroy": [vp],
        "rrcg_group_create": [C.POINTER(RrcgDesc), i, vp, C.POINTER(vp)],
        "rrcg_group_step": [vp, i, vp],
        "rrcg_group_read_scalars": [vp, i, C.POINTER(RrcgScalars), vp],
        "rrcg_group_write_scalars": [vp, i, C.POINTER(RrcgScalars), vp],
        "rrcg_group_refresh": [vp, vp],
        "rrcg_group_set_launch": [vp, i, i, i, i, vp],
        "rrcg_group_products": [vp, C.POINTER(vp)],
        "rrcg_group_destroy": [vp],
        "bttb_autotune": [vp, i, vp, C.POINTER(TuneResult)],
        "bttb_group_autotune": [vp, i, vp, C.POINTER(TuneResult)],
        "rrcg_group_autotune": [vp, i, vp, C.POINTER(TuneResult)],
        "bttb_group_timing_enable": [vp, i, i],
        "bttb_group_timing_read": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)],
        "rrcg_products": [vp, C.POINTER(vp)],
        "rrcg_autotune": [vp, i, vp, C.POINTER(TuneResult)],
        "rrcg_prepare": [vp, i],
        "rrcg_group_prepare": [vp, i],
        "bttb_group_timing_list": [vp, i, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_int)],
        "bttb_apply_noalloc": [vp, i, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.bttb_strerror.argtypes = [i]
    L.bttb_strerror.restype = C.c_char_p
    L.bttb_last_error.argtypes = []
    L.bttb_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != BTTB_OK:
        L = lib()
        msg = L.bttb_last_error().decode(errors="replace")
        raise BTTBError(status, where, f"{L.bttb_strerror(status).decode()}: {msg}")
