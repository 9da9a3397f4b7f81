"""ctypes binding of libkpsb.so (argument marshalling only).

The structures mirror include/kpsb.h field by field. Device buffers are passed
as raw pointers (e.g. ``tensor.data_ptr()``), the stream as a hipStream_t
handle (``torch.cuda.current_stream().cuda_stream``). Nothing here computes.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkpsb.so")

KP_OK, KP_E_INVAL, KP_E_NOMEM, KP_E_DEVICE, KP_E_NUMERIC = 0, 1, 2, 3, 4
KP_E_BUSY, KP_E_TIMEOUT, KP_E_CANCELLED = 5, 6, 7
KP_W_BREAKDOWN = 100
KP_F64, KP_F32, KP_BF16, KP_F16, KP_F16X3 = 0, 1, 2, 3, 4
KP_METHOD_GKB, KP_METHOD_RSVD = 0, 1
KP_BC_ZERO, KP_BC_REFLEXIVE, KP_BC_PERIODIC = 0, 1, 2

STATUS_NAMES = {0: "KP_OK", 1: "KP_E_INVAL", 2: "KP_E_NOMEM", 3: "KP_E_DEVICE",
                4: "KP_E_NUMERIC", 5: "KP_E_BUSY", 6: "KP_E_TIMEOUT", 7: "KP_E_CANCELLED",
                100: "KP_W_BREAKDOWN"}

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTED = ["kp_ctx_create", "kp_ctx_destroy", "kp_last_error", "kp_version",
            "kp_prof_enable", "kp_prof_read",
            "kp_rmat_apply", "kp_svd_gkb", "kp_svd_rsvd", "kp_apply",
            "sb_solve_aniso", "sb_solve_iso", "kp_svd_batched",
            "kp_server_create", "kp_server_submit", "kp_server_wait", "kp_server_stats",
            "kp_server_destroy", "kp_tune_report", "kp_rmat_reorder", "kp_rmat_apply_stored",
            "kp_svd_gkb_stored", "kp_svd_rsvd_stored", "sb_solve_aniso_direct",
            "sb_solve_iso_direct", "kp_blur_matrix", "kp_rmat_apply_noalloc",
            "kp_ctx_workspace", "kp_request_footprint", "kp_cancel", "kp_server_cancel",
            "sb_solve_batched", "kp_blur_apply", "sb_solve_aniso_fft", "sb_solve_iso_fft"]


class kp_blur(C.Structure):
    _fields_ = [("n", C.c_int32), ("psf", C.POINTER(C.c_double)), ("pu", C.c_int32),
                ("pv", C.c_int32), ("cu", C.c_int32), ("cv", C.c_int32),
                ("psf_on_device", C.c_int32), ("bc", C.c_int32), ("compact", C.c_int32)]


class kp_gkb_opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("p", C.c_int32), ("k_min", C.c_int32),
                ("auto_k", C.c_int32), ("tau", C.c_double), ("literal_init", C.c_int32),
                ("reorth", C.c_int32), ("prec", C.c_int), ("seed", C.c_uint64),
                ("y0", C.POINTER(C.c_double)), ("bd_rel", C.c_double),
                ("block", C.c_int32)]


class kp_rsvd_opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("prec", C.c_int),
                ("refine", C.c_int32), ("seed", C.c_uint64), ("F", C.POINTER(C.c_double))]


class kp_diag(C.Structure):
    _fields_ = [("cap", C.c_int32), ("alpha", C.POINTER(C.c_double)),
                ("t", C.POINTER(C.c_double)), ("kp", C.c_int32), ("nbreak", C.c_int32),
                ("break_side", C.c_int32 * 128), ("break_step", C.c_int32 * 128),
                ("ms_total", C.c_double), ("basis_u", C.c_void_p), ("basis_v", C.c_void_p)]


class kp_factors(C.Structure):
    _fields_ = [("n", C.c_int32), ("k_cap", C.c_int32), ("k", C.c_int32),
                ("sigma", C.POINTER(C.c_double)), ("Ax", C.c_void_p), ("Ay", C.c_void_p),
                ("factor_prec", C.c_int), ("diag", C.POINTER(kp_diag))]


class sb_opts(C.Structure):
    _fields_ = [("lam", C.c_double), ("beta", C.c_double), ("L_max", C.c_int32),
                ("I_max", C.c_int32), ("tau_sb", C.c_double), ("tau_cgls", C.c_double)]


class kp_prof(C.Structure):
    _fields_ = [("ms", C.c_double * 4), ("launches", C.c_int64 * 4), ("flops", C.c_double * 4)]


class sb_stats(C.Structure):
    _fields_ = [("l_end", C.c_int32), ("iota_total", C.c_int32), ("rc_sb", C.c_double),
                ("graph_replays", C.c_int32), ("reserved", C.c_int32)]


class sb_problem(C.Structure):
    _fields_ = [("f", C.POINTER(kp_factors)), ("b", C.c_void_p), ("x", C.c_void_p),
                ("opts", sb_opts), ("iso", C.c_int32), ("reserved", C.c_int32)]


class kp_server_cfg(C.Structure):
    _fields_ = [("slots", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("max_pending", C.c_int32), ("cache_entries", C.c_int32)]


class kp_request(C.Structure):
    _fields_ = [("psf_key", C.c_uint64), ("blur", kp_blur), ("method", C.c_int32),
                ("gkb", kp_gkb_opts), ("rsvd", kp_rsvd_opts), ("k_cap", C.c_int32),
                ("iso", C.c_int32), ("sb", sb_opts), ("b", C.c_void_p), ("x", C.c_void_p)]


class kp_result(C.Structure):
    _fields_ = [("status", C.c_int), ("stats", sb_stats), ("k", C.c_int32),
                ("cache_hit", C.c_int32), ("queue_ms", C.c_double), ("factor_ms", C.c_double),
                ("solve_ms", C.c_double), ("total_ms", C.c_double), ("msg", C.c_char * 160)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2410_00233_amd.build`")
    # PyTorch (which owns device memory and streams here) ships its own HIP
    # runtime; one runtime serves the process, the first one loaded. Load
    # PyTorch's before the library so that both use it: with the system
    # runtime loaded first, PyTorch finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.kp_ctx_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(vp)]
    lib.kp_ctx_destroy.argtypes = [vp]
    lib.kp_last_error.argtypes = [vp]
    lib.kp_last_error.restype = C.c_char_p
    lib.kp_version.argtypes = []
    lib.kp_version.restype = C.c_char_p
    lib.kp_prof_enable.argtypes = [vp, C.c_int]
    lib.kp_prof_read.argtypes = [vp, C.POINTER(kp_prof), C.c_int]
    lib.kp_rmat_apply.argtypes = [vp, C.POINTER(kp_blur), C.c_int, C.c_int, C.c_int32, vp, vp, vp]
    lib.kp_rmat_apply_noalloc.argtypes = lib.kp_rmat_apply.argtypes
    lib.kp_ctx_workspace.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.kp_cancel.argtypes = [vp]
    lib.kp_server_cancel.argtypes = [vp, C.c_uint64]
    lib.kp_request_footprint.argtypes = [C.POINTER(kp_request), C.POINTER(C.c_size_t)]
    lib.kp_svd_gkb.argtypes = [vp, C.POINTER(kp_blur), C.POINTER(kp_gkb_opts),
                               C.POINTER(kp_factors), vp]
    lib.kp_svd_rsvd.argtypes = [vp, C.POINTER(kp_blur), C.POINTER(kp_rsvd_opts),
                                C.POINTER(kp_factors), vp]
    lib.kp_apply.argtypes = [vp, C.POINTER(kp_factors), C.c_int, vp, vp, vp]
    lib.sb_solve_aniso.argtypes = [vp, C.POINTER(kp_factors), vp, C.POINTER(sb_opts), vp,
                                   C.POINTER(sb_stats), vp]
    lib.sb_solve_iso.argtypes = lib.sb_solve_aniso.argtypes
    lib.kp_svd_batched.argtypes = [vp, C.c_int32, C.POINTER(kp_blur), C.POINTER(C.c_int32),
                                   C.POINTER(vp), C.POINTER(kp_factors), C.POINTER(C.c_int),
                                   C.c_int32, vp]
    lib.sb_solve_batched.argtypes = [vp, C.c_int32, C.POINTER(sb_problem), C.POINTER(sb_stats),
                                     C.POINTER(C.c_int), C.c_int32, vp]
    lib.kp_server_create.argtypes = [vp, C.POINTER(kp_server_cfg), C.POINTER(vp)]
    lib.kp_server_submit.argtypes = [vp, C.POINTER(kp_request), C.POINTER(C.c_uint64)]
    lib.kp_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(kp_result)]
    lib.kp_server_stats.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.kp_server_destroy.argtypes = [vp]
    lib.kp_tune_report.argtypes = [C.c_char_p, C.c_size_t]
    lib.kp_rmat_reorder.argtypes = [vp, C.c_int32, C.c_int, vp, vp, vp]
    lib.kp_blur_matrix.argtypes = [vp, C.POINTER(kp_blur), C.c_int, vp, vp]
    lib.kp_rmat_apply_stored.argtypes = [vp, C.c_int32, C.c_int, vp, C.c_int, C.c_int32, vp, vp,
                                         vp]
    lib.kp_svd_gkb_stored.argtypes = [vp, C.c_int32, vp, C.POINTER(kp_gkb_opts),
                                      C.POINTER(kp_factors), vp]
    lib.kp_svd_rsvd_stored.argtypes = [vp, C.c_int32, vp, C.POINTER(kp_rsvd_opts),
                                       C.POINTER(kp_factors), vp]
    lib.sb_solve_aniso_direct.argtypes = [vp, C.c_int32, vp, vp, C.POINTER(sb_opts), vp,
                                          C.POINTER(sb_stats), vp]
    lib.sb_solve_iso_direct.argtypes = lib.sb_solve_aniso_direct.argtypes
    lib.kp_blur_apply.argtypes = [vp, C.POINTER(kp_blur), C.c_int, vp, vp, vp]
    lib.sb_solve_aniso_fft.argtypes = [vp, C.POINTER(kp_blur), vp, C.POINTER(sb_opts), vp,
                                       C.POINTER(sb_stats), vp]
    lib.sb_solve_iso_fft.argtypes = lib.sb_solve_aniso_fft.argtypes
    for name in EXPORTED:
        if name not in ("kp_last_error", "kp_version"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
