"""Parity of the generated-tile products R X / R^T X (block MFMA kernel and the
matrix-vector kernel) against the oracle, element by element.

Reference: explicit entries of R(A) from the oracle (section 2.1 rearrangement)
in float64. FP64 kernels: |err| <= 1e-13 max|ref|. FP32 kernels: the forward
error bound of a length-K dot product, |err| <= c K u (|R||X|) with u = 2^-24;
we use 4 * sqrt(K) * u as the statistical scale (rounding errors of FP32
accumulation are random-signed) with a floor of 2 K u max|.|, i.e. the test
allows |err| <= 2e-6 * (|R| |X|) + 1e-7 * max(|R||X|).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import operator as op

pytestmark = pytest.mark.gpu


def _run(ctx, P, cu, cv, n, X, transpose, prec):
    """X: (n^2,) or (n^2, b) host array; the device block is column-major, i.e. a
    (b, n^2) row-major tensor."""
    import torch
    from paper_2410_00233_amd import api
    dt = torch.float64 if prec == "f64" else torch.float32   # 16-bit modes take FP32 X
    Xt = torch.tensor(X if X.ndim == 1 else np.ascontiguousarray(X.T), dtype=dt, device="cuda")
    Y = ctx.kp_rmat_apply(api.Blur(P, cu, cv, n), Xt, transpose=transpose, prec=prec)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy().astype(np.float64)
    return Yh if X.ndim == 1 else Yh.T


def _check(Y, R, X, prec):
    ref = R @ X
    mag = np.abs(R) @ np.abs(X)
    if prec == "f64":
        assert np.abs(Y - ref).max() <= 1e-13 * max(mag.max(), 1e-300)
    else:
        assert np.all(np.abs(Y - ref) <= 2e-6 * mag + 1e-7 * mag.max())


CASES = [(2, (1, 1), 0), (5, (3, 4), 1), (12, (5, 7), 2), (16, (9, 9), 3), (20, (30, 30), 4),
         (33, (7, 40), 5), (48, (95, 95), 6)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ncols", [1, 3, 32, 37])
@pytest.mark.parametrize("n,shape,seed", CASES)
def test_product_matches_explicit_R(ctx, n, shape, seed, ncols, prec):
    P, cu, cv = wl.random_psf(shape[0], shape[1], seed)
    idx = np.arange(n * n)
    R = op.rmat_entries(P, cu, cv, n, idx, idx)
    X = np.random.default_rng(seed).standard_normal((n * n, ncols))
    if prec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    for tr in (False, True):
        Xin = X[:, 0] if ncols == 1 else X
        Y = _run(ctx, P, cu, cv, n, Xin, tr, prec)
        _check(Y.reshape(n * n, -1), (R.T if tr else R), X, prec)


@pytest.mark.parametrize("n,cp", [(48, 16), (33, 10), (70, 64), (16, 1)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_block_product_in_column_phases(ctx, n, cp, prec, monkeypatch):
    """The slab of grid columns reloaded per phase of cp column blocks (how large
    n fits the LDS), forced at small n, including a ragged last phase."""
    monkeypatch.setenv("KPSB_BLOCK_CP", str(cp))
    P, cu, cv = wl.random_psf(2 * n - 1, 2 * n - 1, n + cp)
    idx = np.arange(n * n)
    R = op.rmat_entries(P, cu, cv, n, idx, idx)
    X = np.random.default_rng(cp).standard_normal((n * n, 32))
    if prec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    for tr in (False, True):
        Y = _run(ctx, P, cu, cv, n, X, tr, prec).reshape(n * n, -1)
        _check(Y, (R.T if tr else R), X, prec)


@pytest.mark.parametrize("n,prec", [(256, "f32"), (512, "f32"), (128, "f64"), (1024, "f32")])
@pytest.mark.parametrize("ncols", [1, 32])
def test_product_full_size_sampled_rows(ctx, n, prec, ncols):
    # the configured workload: rotated Gaussian on the full (2n-1)^2 grid
    P, cu, cv = wl.gaussian_psf(n)
    X = np.random.default_rng(n).standard_normal((n * n, ncols))
    if prec == "f32":
        X = X.astype(np.float32).astype(np.float64)
    rows = np.unique(np.r_[0, n * n - 1, n - 1, n * (n - 1),
                           np.random.default_rng(n + 1).choice(n * n, 24, replace=False)])
    for tr in (False, True):
        Y = _run(ctx, P, cu, cv, n, X[:, 0] if ncols == 1 else X, tr, prec).reshape(n * n, -1)
        Rrows = op.rmat_entries(P.T, cv, cu, n, rows, np.arange(n * n)) if tr else \
            op.rmat_entries(P, cu, cv, n, rows, np.arange(n * n))
        _check(Y[rows], Rrows, X, prec)
        # every row agrees with the (exact-arithmetic-equal) structured product,
        # componentwise against |R| |X| = R(|P|) |X|
        Ys = op.rmat_struct_apply(P, cu, cv, n, X, transpose=tr)
        mag = op.rmat_struct_apply(np.abs(P), cu, cv, n, np.abs(X), transpose=tr)
        tol = 1e-12 if prec == "f64" else 2e-6
        assert np.all(np.abs(Y - Ys) <= tol * mag + 0.05 * tol * mag.max())


def _round16(a, prec):
    """Round like the kernel: FP64 -> FP32 -> 16-bit, round to nearest even."""
    a32 = np.asarray(a, dtype=np.float32)
    if prec == "f16":
        return a32.astype(np.float16).astype(np.float64)
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + (((u >> 16) & 1) + 0x7FFF)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n,shape,seed,ncols", [(5, (3, 4), 1, 3), (16, (9, 9), 3, 32),
                                                (33, (7, 40), 5, 37), (48, (95, 95), 6, 20)])
def test_product16_matches_rounded_explicit_R(ctx, n, shape, seed, ncols, prec):
    P, cu, cv = wl.random_psf(shape[0], shape[1], seed)
    idx = np.arange(n * n)
    X = np.random.default_rng(seed).standard_normal((n * n, ncols)).astype(np.float32).astype(np.float64)
    for tr in (False, True):
        R = op.rmat_entries(P, cu, cv, n, idx, idx)
        R = R.T if tr else R
        Y = _run(ctx, P, cu, cv, n, X, tr, prec).reshape(n * n, -1)
        R16, X16 = _round16(R, prec), _round16(X, prec)
        ref = R16 @ X16
        mag = np.abs(R16) @ np.abs(X16)
        assert np.all(np.abs(Y - ref) <= 2e-6 * mag + 1e-7 * mag.max())


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_product16_full_size_sampled_rows(ctx, prec):
    n = 512
    P, cu, cv = wl.gaussian_psf(n)
    X = np.random.default_rng(7).standard_normal((n * n, 30)).astype(np.float32).astype(np.float64)
    rows = np.unique(np.r_[0, n * n - 1, np.random.default_rng(8).choice(n * n, 16, replace=False)])
    Y = _run(ctx, P, cu, cv, n, X, False, prec).reshape(n * n, -1)
    R16 = _round16(op.rmat_entries(P, cu, cv, n, rows, np.arange(n * n)), prec)
    X16 = _round16(X, prec)
    ref = R16 @ X16
    mag = np.abs(R16) @ np.abs(X16)
    assert np.all(np.abs(Y[rows] - ref) <= 2e-6 * mag + 1e-7 * mag.max())


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("n,force,tr", [(400, "5", False), (417, "5", True), (417, None, False)])
def test_product16_slab_phases_ragged(ctx, n, force, tr, prec, monkeypatch):
    """16-bit products with 64 row blocks per workgroup (variant 5): the slab at
    n = 400 / 417 runs in phases of 256 column blocks, reloaded between X tiles;
    n = 417 leaves a ragged last row block. Sampled rows (and the first / last)
    against the FP64 product of the rounded operands, both orientations; the
    tuned shape at n = 417 as well."""
    if force is not None:
        monkeypatch.setenv("KPSB_TUNE_FORCE", force)
    P, cu, cv = wl.mixed_psf(n, "disk", np.random.default_rng(n))
    X = np.random.default_rng(n + 1).standard_normal((n * n, 21)).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(n + 2)
    rows = np.unique(np.r_[0, n - 1, n * n - n, n * n - 1, rng.choice(n * n, 14, replace=False)])
    Y = _run(ctx, P, cu, cv, n, X, tr, prec).reshape(n * n, -1)
    cols = np.arange(n * n)
    R = op.rmat_entries(P, cu, cv, n, cols, rows).T if tr else op.rmat_entries(P, cu, cv, n, rows, cols)
    R16, X16 = _round16(R, prec), _round16(X, prec)
    ref = R16 @ X16
    mag = np.abs(R16) @ np.abs(X16)
    assert np.all(np.abs(Y[rows] - ref) <= 2e-6 * mag + 1e-7 * mag.max())


@pytest.mark.parametrize("prec,nvar", [("f32", 18), ("f64", 18), ("bf16", 7)])
@pytest.mark.parametrize("n", [40, 256])
def test_autotuner_variants_agree_bitwise(ctx, prec, nvar, n, monkeypatch):
    """Every launch variant the autotuner chooses among computes the same bits."""
    import torch
    from paper_2410_00233_amd import api
    P, cu, cv = wl.gaussian_psf(n, (2.5, 1.2), 17.0)
    dt = torch.float64 if prec == "f64" else torch.float32
    X = torch.tensor(np.random.default_rng(n).standard_normal((30, n * n)), dtype=dt,
                     device="cuda")
    blur = api.Blur(P, cu, cv, n)
    outs = []
    for v in range(nvar):
        monkeypatch.setenv("KPSB_TUNE_FORCE", str(v))
        outs.append(ctx.kp_rmat_apply(blur, X, prec=prec).cpu())
    monkeypatch.delenv("KPSB_TUNE_FORCE")
    outs.append(ctx.kp_rmat_apply(blur, X, prec=prec).cpu())     # the tuned choice
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    rep = ctx.kp_tune_report()
    assert any(r["n"] == n for r in rep)


@pytest.mark.parametrize("n,k", [(96, 7), (256, 20)])
def test_apply_variants_agree_bitwise(ctx, n, k, monkeypatch):
    import torch
    from paper_2410_00233_amd import api
    rng = np.random.default_rng(n)
    f = api.Factors.from_arrays(rng.standard_normal((k, n, n)), rng.standard_normal((k, n, n)))
    X = torch.tensor(rng.standard_normal((n, n)), dtype=torch.float64, device="cuda")
    for tr in (False, True):
        outs = []
        for v in range(8):          # every Kronecker-apply launch variant
            monkeypatch.setenv("KPSB_TUNE_FORCE", str(v))
            outs.append(ctx.kp_apply(f, X, transpose=tr).cpu())
        for o in outs[1:]:
            assert torch.equal(o, outs[0])
