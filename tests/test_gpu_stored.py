"""The explicit-matrix path: reorder of a stored blur matrix A into R(A)
(section 2.1), products and KP-SVDs of the stored R, and split Bregman with A
itself (the paper's method (i)), against the oracle. Covers the reflexive
boundary conditions of the paper's "Medium" example through an explicit A.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import kpsvd, operator as op, sb

pytestmark = pytest.mark.gpu


def _dev(a, dt="f64"):
    import torch
    return torch.tensor(np.ascontiguousarray(a),
                        dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [2, 5, 16, 33])
def test_reorder_is_the_literal_rearrangement(ctx, n, prec):
    A = np.random.default_rng(n).standard_normal((n * n, n * n))
    if prec == "f32":
        A = A.astype(np.float32).astype(np.float64)
    R = ctx.kp_rmat_reorder(n, _dev(A, prec)).cpu().numpy().astype(np.float64)
    assert np.array_equal(R, op.rearrange(A, n, n, n, n))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ncols", [1, 5, 32, 37])
@pytest.mark.parametrize("n", [7, 16, 40])
def test_stored_products_match_explicit_R(ctx, n, ncols, prec):
    import torch
    rng = np.random.default_rng(n + ncols)
    R = rng.standard_normal((n * n, n * n))
    X = rng.standard_normal((n * n, ncols))
    if prec == "f32":
        R = R.astype(np.float32).astype(np.float64)
        X = X.astype(np.float32).astype(np.float64)
    Rd = _dev(R, prec)
    Xd = _dev(X[:, 0] if ncols == 1 else X.T, prec)
    for tr in (False, True):
        Y = ctx.kp_rmat_apply_stored(n, Rd, Xd, transpose=tr)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy().astype(np.float64)
        Yh = Yh[:, None] if ncols == 1 else Yh.T
        M = R.T if tr else R
        ref, mag = M @ X, np.abs(M) @ np.abs(X)
        if prec == "f64":
            assert np.abs(Yh - ref).max() <= 1e-13 * mag.max()
        else:
            assert np.all(np.abs(Yh - ref) <= 2e-6 * mag + 1e-7 * mag.max())


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shift_R,shift_x", [(1, 0), (0, 1), (1, 1), (0, 0)])
def test_stored_gemv_on_offset_views(ctx, prec, shift_R, shift_x):
    """R and x as views one element into a larger buffer (not 16-byte aligned):
    the matrix-vector products must read them element-wise and agree with the
    aligned call to rounding order."""
    import torch
    n = 16
    N = n * n
    rng = np.random.default_rng(5 + shift_R + 2 * shift_x)
    R = rng.standard_normal((N, N))
    x = rng.standard_normal(N)
    if prec == "f32":
        R = R.astype(np.float32).astype(np.float64)
        x = x.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == "f64" else torch.float32
    Rbuf = torch.zeros(N * N + 1, dtype=dt, device="cuda")
    Rbuf[shift_R:shift_R + N * N] = torch.tensor(R.ravel(), dtype=dt, device="cuda")
    xbuf = torch.zeros(N + 1, dtype=dt, device="cuda")
    xbuf[shift_x:shift_x + N] = torch.tensor(x, dtype=dt, device="cuda")
    Rd = Rbuf[shift_R:shift_R + N * N].view(N, N)
    xd = xbuf[shift_x:shift_x + N]
    for tr in (False, True):
        y = ctx.kp_rmat_apply_stored(n, Rd, xd, transpose=tr)
        torch.cuda.synchronize()
        M = R.T if tr else R
        ref, mag = M @ x, np.abs(M) @ np.abs(x)
        err = np.abs(y.cpu().numpy().astype(np.float64) - ref)
        if prec == "f64":
            assert err.max() <= 1e-13 * mag.max()
        else:
            assert np.all(err <= 2e-6 * mag + 1e-7 * mag.max())


def _blur_problem(n, bc, seed):
    P, cu, cv = wl.random_psf(7, 9, seed, cu=3, cv=4)
    A = op.blur_matrix_reflexive(P, cu, cv, n) if bc == "reflexive" else op.blur_matrix(P, cu, cv, n)
    return P, cu, cv, A


@pytest.mark.parametrize("bc", ["zero", "reflexive"])
def test_stored_kpsvd_matches_oracle(ctx, bc):
    """EGKB and RSVD of the reordered A (FP64) against the oracle run on the
    explicit R with the same start vector / sketch (1e-12 sigma_1); for zero
    boundary conditions they also equal the generated-tile path."""
    from paper_2410_00233_amd import api
    n, k, p, q = 12, 5, 5, 1
    P, cu, cv, A = _blur_problem(n, bc, 3)
    R = op.rearrange(A, n, n, n, n)
    Rd = ctx.kp_rmat_reorder(n, _dev(A))
    apply_R, apply_Rt = (lambda X: R @ X), (lambda X: R.T @ X)
    y = wl.gaussian_block(n * n, 1, seed=11)[:, 0]
    F = wl.gaussian_block(n * n, k + p, seed=12)
    g = ctx.kp_svd_gkb(None, k, p, prec="f64", y0=y, stored=(n, Rd))
    ref = kpsvd.egkb(apply_R, apply_Rt, y, k, p, force_breakdown=set(g.breakdowns))
    s1 = ref["sigma"][0]
    assert np.abs(g.sigma[:k] - ref["sigma"]).max() <= 1e-12 * s1
    r = ctx.kp_svd_rsvd(None, k, p, q, prec="f64", F=F, stored=(n, Rd))
    ref_r = kpsvd.rsvd(apply_R, apply_Rt, F, k, q)
    assert np.abs(r.sigma[:k] - ref_r["sigma"]).max() <= 1e-12 * s1
    exact = np.linalg.svd(R, compute_uv=False)[:k]
    assert np.all(r.sigma[:k] <= exact * (1 + 1e-12) + 1e-14 * s1)      # interlacing
    if bc == "zero":
        gg = ctx.kp_svd_rsvd(api.Blur(P, cu, cv, n), k, p, q, prec="f64", F=F)
        assert np.abs(gg.sigma[:k] - r.sigma[:k]).max() <= 1e-12 * s1


def test_stored_f32_egkb_close_to_generated(ctx):
    from paper_2410_00233_amd import api
    n, k, p = 24, 6, 6
    P, cu, cv = wl.gaussian_psf(n)
    A = op.blur_matrix(P, cu, cv, n)
    Rd = ctx.kp_rmat_reorder(n, _dev(A, "f32"))
    y = wl.gaussian_block(n * n, 1, seed=5)[:, 0]
    s = ctx.kp_svd_gkb(None, k, p, prec="f32", y0=y, stored=(n, Rd))
    g = ctx.kp_svd_gkb(api.Blur(P, cu, cv, n), k, p, prec="f32", y0=y)
    assert np.abs(s.sigma[:k] - g.sigma[:k]).max() <= 1e-5 * g.sigma[0]


@pytest.mark.parametrize("kind", ["aniso", "iso"])
@pytest.mark.parametrize("bc", ["zero", "reflexive"])
def test_sb_with_A_itself_matches_oracle(ctx, kind, bc):
    n = 20
    P, cu, cv, A = _blur_problem(n, bc, 4)
    x_true = wl.rectangles_image(n, seed=7)
    vec = lambda M: M.flatten(order="F")
    unvec = lambda v: v.reshape((n, n), order="F")
    b = unvec(A @ vec(x_true))
    b = wl.add_noise(b, 0.01, seed=8)
    lam, beta = 0.115, 0.115 ** 2 / 2.0
    fn = ctx.sb_solve_aniso_direct if kind == "aniso" else ctx.sb_solve_iso_direct
    x, st = fn(n, _dev(A), _dev(b), lam, beta, L_max=6, I_max=15)
    ref = sb.split_bregman(kind, lambda X: unvec(A @ vec(X)), lambda X: unvec(A.T @ vec(X)), b,
                           lam, beta, L_max=6, I_max=15)
    xr = x.cpu().numpy()
    assert np.linalg.norm(xr - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
    assert st["l_end"] == 6 and st["iota_total"] == 6 * 15


def test_stored_path_rejects_bad_arguments(ctx):
    import torch
    from paper_2410_00233_amd import api
    n = 6
    A = _dev(np.eye(n * n))
    with pytest.raises(api.KPError):                 # R overlaps A
        ctx.kp_rmat_reorder(n, A, R=A)
    with pytest.raises(api.KPError):                 # 16-bit precision for a stored R
        ctx.kp_svd_rsvd(None, 3, 2, 1, prec="bf16", stored=(n, A))
    with pytest.raises(api.KPError):
        ctx.kp_rmat_apply_stored(1, A, torch.zeros(1, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("bc", ["zero", "reflexive"])
@pytest.mark.parametrize("n,shape,seed", [(6, (3, 5), 1), (13, (7, 9), 2), (20, (39, 39), 3)])
def test_blur_matrix_matches_oracle(ctx, bc, n, shape, seed):
    from paper_2410_00233_amd import api
    P, cu, cv = wl.random_psf(shape[0], shape[1], seed)
    A = ctx.kp_blur_matrix(api.Blur(P, cu, cv, n), bc=bc).cpu().numpy()
    ref = op.blur_matrix_reflexive(P, cu, cv, n) if bc == "reflexive" else op.blur_matrix(P, cu, cv, n)
    assert np.abs(A - ref).max() <= 1e-15 * np.abs(ref).max() * 9
