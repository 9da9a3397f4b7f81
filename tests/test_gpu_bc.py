"""Reflexive and periodic boundary conditions in the generator: R(A) of a blur
with non-zero boundary conditions, generated from the PSF (never stored),
against the oracle's R(A) built from the image-sum definition, and against
the explicit-matrix path (blur matrix built on the device, reordered, stored).

Tolerances: FP64 products 1e-13 of max(|R| |X|); FP32 1e-6 of it (four FP32
term products are added for reflexive boundary conditions); 16-bit inputs
1e-2. KP-SVDs: FP64 1e-12 sigma_1 against the oracle on the same start vector
or sketch, FP32 1e-5 sigma_1.
"""
import numpy as np
import pytest

import workloads as wl
from _replay import check_replayed_breakdowns
from oracle import kpsvd, operator as op

pytestmark = pytest.mark.gpu

BLUR_MATRIX = {"zero": op.blur_matrix, "reflexive": op.blur_matrix_reflexive,
               "periodic": op.blur_matrix_periodic}


def _dev(a, dt="f64"):
    import torch
    return torch.tensor(np.ascontiguousarray(a),
                        dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")


def _psf(kind, n, seed):
    """small: 7 x 9 off-centre; full: the (2n-1)^2 offset grid; reach2n: a PSF
    that reaches exactly 2n pixels from its centre (the largest allowed)."""
    if kind == "small":
        return wl.random_psf(7, 9, seed, cu=2, cv=6)
    if kind == "full":
        P = np.random.default_rng(seed).uniform(-0.2, 1.0, (2 * n - 1, 2 * n - 1))
        return P, n - 1, n - 1
    P = np.random.default_rng(seed).uniform(-0.2, 1.0, (4 * n + 1, 2 * n + 3))
    return P, 2 * n, 2 * n


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,kind,ncols", [(5, "small", 1), (5, "reach2n", 7), (12, "full", 1),
                                          (12, "small", 32), (33, "full", 40),
                                          (33, "small", 7)])
def test_generated_products_match_oracle(ctx, bc, prec, n, kind, ncols):
    import torch
    from paper_2410_00233_amd import api
    P, cu, cv = _psf(kind, n, 100 + n + ncols)
    blur = api.Blur(P, cu, cv, n, bc=bc)
    N = n * n
    R = op.rmat_entries(P, cu, cv, n, np.arange(N), np.arange(N), bc)
    X = np.random.default_rng(n).standard_normal((N, ncols))
    if prec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    Xd = _dev(X[:, 0] if ncols == 1 else X.T, prec)
    for tr in (False, True):
        Y = ctx.kp_rmat_apply(blur, Xd, transpose=tr, prec=prec)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy().astype(np.float64)
        Yh = Yh[:, None] if ncols == 1 else Yh.T
        M = R.T if tr else R
        ref, mag = M @ X, (np.abs(M) @ np.abs(X)).max()
        tol = 1e-13 if prec == "f64" else 1e-6
        assert np.abs(Yh - ref).max() <= tol * mag, (tr, np.abs(Yh - ref).max() / mag)


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_generated_16bit_products_match_oracle(ctx, bc):
    import torch
    from paper_2410_00233_amd import api
    n, ncols = 20, 9
    P, cu, cv = wl.random_psf(9, 9, 7, cu=4, cv=4)
    blur = api.Blur(P, cu, cv, n, bc=bc)
    N = n * n
    R = op.rmat_entries(P, cu, cv, n, np.arange(N), np.arange(N), bc)
    X = np.random.default_rng(3).standard_normal((N, ncols)).astype(np.float32)
    for prec in ("bf16", "f16"):
        for tr in (False, True):
            Y = ctx.kp_rmat_apply(blur, _dev(X.T, "f32"), transpose=tr, prec=prec)
            torch.cuda.synchronize()
            M = R.T if tr else R
            ref = M @ X.astype(np.float64)
            mag = (np.abs(M) @ np.abs(X)).max()
            assert np.abs(Y.cpu().numpy().T - ref).max() <= 1e-2 * mag


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_generated_equals_explicit_matrix_path(ctx, bc):
    """The matrix-free operator against the stored R of the device-built A."""
    import torch
    from paper_2410_00233_amd import api
    n = 40
    P, cu, cv = wl.speckle_psf(8, seed=1007)                 # 15 x 15
    blur = api.Blur(P, cu, cv, n, bc=bc)
    Rd = ctx.kp_rmat_reorder(n, ctx.kp_blur_matrix(blur, prec="f64"))
    X = _dev(np.random.default_rng(5).standard_normal((8, n * n)))
    for tr in (False, True):
        Yg = ctx.kp_rmat_apply(blur, X, transpose=tr, prec="f64")
        Ys = ctx.kp_rmat_apply_stored(n, Rd, X, transpose=tr)
        torch.cuda.synchronize()
        assert (Yg - Ys).abs().max().item() <= 1e-13 * Ys.abs().max().item()


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_blur_matrix_periodic_and_reflexive_match_oracle(ctx, bc):
    from paper_2410_00233_amd import api
    for n, (P, cu, cv) in [(6, wl.random_psf(3, 5, 1)), (5, _psf("reach2n", 5, 2)),
                           (9, _psf("full", 9, 3))]:
        A = ctx.kp_blur_matrix(api.Blur(P, cu, cv, n, bc=bc)).cpu().numpy()
        ref = BLUR_MATRIX[bc](P, cu, cv, n)
        assert np.abs(A - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_kpsvd_with_boundary_conditions_matches_oracle(ctx, bc):
    """EGKB, block EGKB and RSVD (FP64) of the generated R against the oracle
    on the explicit R with the same start vector / block / sketch."""
    from paper_2410_00233_amd import api
    n, k, p, q = 12, 5, 5, 1
    P, cu, cv = wl.random_psf(7, 9, 3, cu=3, cv=4)
    blur = api.Blur(P, cu, cv, n, bc=bc)
    R = op.rearrange(BLUR_MATRIX[bc](P, cu, cv, n), n, n, n, n)
    apply_R, apply_Rt = (lambda X: R @ X), (lambda X: R.T @ X)
    y = wl.gaussian_block(n * n, 1, seed=21)[:, 0]
    Y = wl.gaussian_block(n * n, 2, seed=22)
    F = wl.gaussian_block(n * n, k + p, seed=23)
    g = ctx.kp_svd_gkb(blur, k, p, prec="f64", y0=y)
    ref = kpsvd.egkb(apply_R, apply_Rt, y, k, p, force_breakdown=set(g.breakdowns))
    check_replayed_breakdowns(ref, "f64")
    s1 = ref["sigma"][0]
    assert np.abs(g.sigma[:k] - ref["sigma"]).max() <= 1e-12 * s1
    gb = ctx.kp_svd_gkb(blur, k, p, prec="f64", y0=Y, block=2)
    refb = kpsvd.block_egkb(apply_R, apply_Rt, Y, k, p, force_breakdown=set(gb.breakdowns))
    check_replayed_breakdowns(refb, "f64")
    assert np.abs(gb.sigma[:k] - refb["sigma"]).max() <= 1e-12 * s1
    r = ctx.kp_svd_rsvd(blur, k, p, q, prec="f64", F=F)
    refr = kpsvd.rsvd(apply_R, apply_Rt, F, k, q)
    assert np.abs(r.sigma[:k] - refr["sigma"]).max() <= 1e-12 * s1
    exact = np.linalg.svd(R, compute_uv=False)[:k]
    assert np.all(r.sigma[:k] <= exact * (1 + 1e-12) + 1e-14 * s1)


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_kpsvd_f32_with_boundary_conditions(ctx, bc):
    """FP32 RSVD and EGKB at n = 48 (15 x 15 speckle-like PSF) against the oracle
    on the explicit R."""
    from paper_2410_00233_amd import api
    n, k, p, q = 48, 10, 10, 1
    P, cu, cv = wl.speckle_psf(8, seed=1008)
    blur = api.Blur(P, cu, cv, n, bc=bc)
    N = n * n
    R = op.rmat_entries(P, cu, cv, n, np.arange(N), np.arange(N), bc)
    apply_R, apply_Rt = (lambda X: R @ X), (lambda X: R.T @ X)
    F = wl.gaussian_block(N, k + p, seed=31)
    y = wl.gaussian_block(N, 1, seed=32)[:, 0]
    r = ctx.kp_svd_rsvd(blur, k, p, q, prec="f32", F=F)
    refr = kpsvd.rsvd(apply_R, apply_Rt, F, k, q)
    s1 = refr["sigma"][0]
    assert np.abs(r.sigma[:k] - refr["sigma"]).max() <= 1e-5 * s1
    g = ctx.kp_svd_gkb(blur, k, p, prec="f32", y0=y, reorth=1)
    ref = kpsvd.egkb(apply_R, apply_Rt, y, k, p, force_breakdown=set(g.breakdowns))
    check_replayed_breakdowns(ref, "f32")
    assert np.abs(g.sigma[:k] - ref["sigma"]).max() <= 1e-5 * s1


def test_bf16_rsvd_with_refinement_reflexive(ctx):
    """BF16 block products plus the split-FP16 refinement product (four terms
    each) against the FP32 RSVD on the same sketch."""
    from paper_2410_00233_amd import api
    n, k, p, q = 64, 10, 10, 2
    P, cu, cv = wl.speckle_psf(8, seed=1009)
    blur = api.Blur(P, cu, cv, n, bc="reflexive")
    F = wl.gaussian_block(n * n, k + p, seed=41)
    f32 = ctx.kp_svd_rsvd(blur, k, p, q, prec="f32", F=F)
    for refine, tol in ((2, 1e-6), (1, 1e-6), (0, 1e-2)):
        fb = ctx.kp_svd_rsvd(blur, k, p, q, prec="bf16", refine=refine, F=F)
        err = np.abs(fb.sigma[:k] - f32.sigma[:k]).max() / f32.sigma[0]
        assert err <= tol, (refine, err)


@pytest.mark.parametrize("bc", ["reflexive", "periodic"])
def test_sampled_rows_at_n256(ctx, bc):
    """FP32 products at n = 256 (full-size launches) on sampled rows and
    columns of R computed one by one by the oracle."""
    import torch
    from paper_2410_00233_amd import api
    n, ncols = 256, 5
    P, cu, cv = wl.speckle_psf(8, seed=1010)
    blur = api.Blur(P, cu, cv, n, bc=bc)
    N = n * n
    rng = np.random.default_rng(6)
    X = rng.standard_normal((N, ncols)).astype(np.float32)
    sample = np.concatenate([np.arange(0, 2 * n, 37), rng.integers(0, N, 24), [N - 1, N - n]])
    for tr in (False, True):
        Y = ctx.kp_rmat_apply(blur, _dev(X.T, "f32"), transpose=tr, prec="f32")
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy().T.astype(np.float64)
        Rs = (op.rmat_entries(P, cu, cv, n, np.arange(N), sample, bc).T if tr
              else op.rmat_entries(P, cu, cv, n, sample, np.arange(N), bc))
        ref = Rs @ X.astype(np.float64)
        mag = (np.abs(Rs) @ np.abs(X)).max()
        assert np.abs(Yh[sample] - ref).max() <= 1e-6 * mag


def test_boundary_conditions_are_validated(ctx):
    from paper_2410_00233_amd import api
    n = 6
    P = np.ones((4 * n + 3, 3))
    with pytest.raises(api.KPError):           # reaches 2n + 1 pixels above the centre
        ctx.kp_rmat_apply(api.Blur(P, 2 * n + 1, 1, n, bc="reflexive"),
                          _dev(np.ones(n * n)), prec="f64")
    b = api.Blur(np.ones((3, 3)), 1, 1, n)
    b.s.bc = 7
    with pytest.raises(api.KPError):
        ctx.kp_rmat_apply(b, _dev(np.ones(n * n)), prec="f64")
    # the same PSF with zero boundary conditions is valid at any reach
    ctx.kp_rmat_apply(api.Blur(P, 2 * n + 1, 1, n), _dev(np.ones(n * n)), prec="f64")


def test_server_keys_factors_by_boundary_conditions(ctx):
    """Two requests with the same PSF key but different boundary conditions
    do not share cached factors."""
    import torch
    from paper_2410_00233_amd import api
    n = 16
    P, cu, cv = wl.random_psf(5, 5, 9)
    b = np.random.default_rng(1).uniform(0, 1, (n, n))
    bd = _dev(b)
    srv = api.Server(ctx, slots=1)
    res = []
    for bc in ("zero", "reflexive", "zero", "reflexive"):
        x = torch.empty_like(bd)
        r = srv.wait(srv.submit(api.Blur(P, cu, cv, n, bc=bc), bd, x, psf_key=77, method="rsvd",
                                k=4, p=4, q=1, prec="f32", seed=3, L_max=3, I_max=5))
        assert r["status"] == 0, r["msg"]
        res.append((r["cache_hit"], x.clone()))
    srv.close()
    assert [h for h, _ in res] == [False, False, True, True]
    assert torch.equal(res[0][1], res[2][1]) and torch.equal(res[1][1], res[3][1])
    assert not torch.equal(res[0][1], res[1][1])
