"""The oracle's pins have teeth: each plausible slip planted in a copy of the
oracle (never in the product path) must make a pin fail.

The split Bregman slips are judged by the certified-minimizer pin of
Algorithms 3/4 (tests/_sb_pins.py); the refinement slip by the rotated exact
subspace pin of the Rayleigh-Ritz refinement.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import operator as op

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def _mutant(name, old, new):
    """A fresh copy of oracle.<name> with ``old`` replaced by ``new`` (which
    must occur exactly once in its source)."""
    path = os.path.join(ORACLE, name + ".py")
    src = open(path).read()
    assert src.count(old) == 1, (name, old)
    spec = importlib.util.spec_from_loader(f"oracle._mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    mod.__file__ = path
    sys.modules[spec.name] = mod
    try:
        exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    finally:
        del sys.modules[spec.name]
    return mod


SB_MUTATIONS = [
    # (kind checked, original text, planted slip)
    ("aniso", "gx = cx - dx", "gx = dx - cx"),                       # Bregman update sign
    ("iso", "gy = cy - dy", "gy = dy - cy"),
    ("aniso", "dx = shrink(cx, 1.0 / gamma)", "dx = shrink(cx, 0.5 / gamma)"),   # threshold
    ("iso", "iso_shrink(cx, cy, 1.0 / gamma)", "iso_shrink(cx, cy, 0.5 / gamma)"),
    ("aniso", "cx = x_new @ L.T + gx", "cx = L @ x_new + gx"),       # wrong direction
    ("iso", "gamma = lam * lam / beta", "gamma = beta / (lam * lam)"),  # gamma inverted
    ("aniso", "bhat = (b, lam * (dx - gx), lam * (dy - gy))",
     "bhat = (b, lam * (gx - dx), lam * (dy - gy))"),                 # h = d - g sign
    ("iso", "L -= 0.5 * np.eye(n, k=1)", "L -= 0.5 * np.eye(n, k=-1)"),  # L transposed
]


def test_unmutated_oracle_passes_the_sb_pin():
    from _sb_pins import loop_error
    from oracle import sb
    assert loop_error(sb, "aniso") <= 1e-6


@pytest.mark.parametrize("kind,old,new", SB_MUTATIONS)
def test_sb_slip_fails_the_minimizer_pin(kind, old, new):
    from _sb_pins import loop_error
    err = loop_error(_mutant("sb", old, new), kind)
    assert not err <= 1e-6, f"slip {new!r} passed the pin (err {err:.2e})"


def _refine_subspace_error(kpsvd_mod):
    n, k = 20, 8
    P, cu, cv = wl.speckle_psf(n, seed=1005)
    R = lambda X: op.rmat_struct_apply(P, cu, cv, n, X)
    s_ex, U_ex, V_ex = op.exact_kpsvd(P, cu, cv, n, k)
    Qm, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((k, k)))
    out = kpsvd_mod.refine(R, V_ex @ Qm)
    e = 0.0
    for i in range(k):
        v = out["V"][:, i]
        e = max(e, min(np.abs(v - V_ex[:, i]).max(), np.abs(v + V_ex[:, i]).max()))
    e = max(e, np.linalg.norm(R(out["V"]) - out["U"] * out["sigma"]) / s_ex[0])
    return e


def test_refine_slip_fails_the_subspace_pin():
    from oracle import kpsvd
    assert _refine_subspace_error(kpsvd) <= 1e-10
    bad = _mutant("kpsvd", "V=Vo @ Zt.T", "V=Vo @ Zt")
    assert _refine_subspace_error(bad) > 1e-3
