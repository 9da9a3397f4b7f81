"""CPU checks of the C ABI: the library builds/loads, exports every function the
header declares, and the ctypes structures match the C layout (compiled with gcc
from include/kpsb.h). No compute call is made."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2410_00233_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpsb.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:kp_status|const char\*)\s+(\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2410_00233_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert sorted(_lib.EXPORTED) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in names:
        assert n in syms, n
        assert hasattr(lib, n)


def test_version_string(lib):
    assert lib.kp_version().startswith(b"kpsb")


def test_null_arguments_are_rejected(lib):
    assert lib.kp_ctx_create(0, 0, None) == _lib.KP_E_INVAL
    assert lib.kp_ctx_destroy(None) == _lib.KP_E_INVAL
    assert lib.kp_svd_gkb(None, None, None, None, None) == _lib.KP_E_INVAL
    assert lib.kp_last_error(None) == b"null context"
    assert lib.kp_svd_batched(None, 0, None, None, None, None, None, 0, None) == _lib.KP_E_INVAL
    assert lib.sb_solve_batched(None, 0, None, None, None, 0, None) == _lib.KP_E_INVAL
    assert lib.kp_server_create(None, None, None) == _lib.KP_E_INVAL
    assert lib.kp_server_submit(None, None, None) == _lib.KP_E_INVAL
    assert lib.kp_server_wait(None, 0, 0.0, None) == _lib.KP_E_INVAL
    assert lib.kp_server_stats(None, None) == _lib.KP_E_INVAL
    assert lib.kp_server_destroy(None) == _lib.KP_E_INVAL


def test_ctx_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = C.c_void_p()
    assert lib.kp_ctx_create(0, 0, C.byref(h)) == _lib.KP_E_DEVICE


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "kpsb.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
#define S(T) printf(#T " %zu\n", sizeof(T))
int main(void) {
  S(kp_blur); P(kp_blur, psf); P(kp_blur, cv); P(kp_blur, psf_on_device); P(kp_blur, bc); P(kp_blur, compact);
  S(kp_gkb_opts); P(kp_gkb_opts, tau); P(kp_gkb_opts, prec); P(kp_gkb_opts, seed); P(kp_gkb_opts, y0); P(kp_gkb_opts, bd_rel); P(kp_gkb_opts, block);
  S(kp_rsvd_opts); P(kp_rsvd_opts, prec); P(kp_rsvd_opts, seed); P(kp_rsvd_opts, F);
  S(kp_diag); P(kp_diag, alpha); P(kp_diag, kp); P(kp_diag, break_side); P(kp_diag, ms_total); P(kp_diag, basis_v);
  S(kp_factors); P(kp_factors, sigma); P(kp_factors, Ax); P(kp_factors, factor_prec); P(kp_factors, diag);
  S(sb_opts); P(sb_opts, L_max); P(sb_opts, tau_cgls);
  S(sb_stats); P(sb_stats, rc_sb); P(sb_stats, graph_replays);
  S(sb_problem); P(sb_problem, b); P(sb_problem, x); P(sb_problem, opts); P(sb_problem, iso);
  S(kp_prof); P(kp_prof, launches); P(kp_prof, flops);
  S(kp_server_cfg); P(kp_server_cfg, hbm_budget_bytes); P(kp_server_cfg, cache_entries);
  S(kp_request); P(kp_request, blur); P(kp_request, method); P(kp_request, gkb); P(kp_request, rsvd);
  P(kp_request, k_cap); P(kp_request, iso); P(kp_request, sb); P(kp_request, b); P(kp_request, x);
  S(kp_result); P(kp_result, stats); P(kp_result, k); P(kp_result, queue_ms); P(kp_result, total_ms);
  P(kp_result, msg);
  return 0;
}
"""


def test_ctypes_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    ref = dict(l.rsplit(" ", 1) for l in lines if l)
    m = {"kp_blur": _lib.kp_blur, "kp_gkb_opts": _lib.kp_gkb_opts, "kp_rsvd_opts": _lib.kp_rsvd_opts,
         "kp_diag": _lib.kp_diag, "kp_factors": _lib.kp_factors, "sb_opts": _lib.sb_opts,
         "sb_stats": _lib.sb_stats, "sb_problem": _lib.sb_problem, "kp_prof": _lib.kp_prof,
         "kp_server_cfg": _lib.kp_server_cfg, "kp_request": _lib.kp_request,
         "kp_result": _lib.kp_result}
    rename = {"lambda": "lam"}
    for key, val in ref.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(m[t], rename.get(f, f)).offset == int(val), key
        else:
            assert C.sizeof(m[key]) == int(val), key


def test_library_loads_after_torch():
    """PyTorch's HIP runtime must be the process's one (loaded before the
    library), or PyTorch finds no GPU once the library has initialised HIP:
    loading the library in a fresh process imports torch first."""
    import subprocess
    import sys
    code = ("import sys; from paper_2410_00233_amd import _lib; "
            "assert 'torch' not in sys.modules; _lib.load(); "
            "assert 'torch' in sys.modules; print('ok')")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=str(__import__("pathlib").Path(__file__).resolve().parents[1]),
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
