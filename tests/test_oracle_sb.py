"""Pins for the oracle's Kronecker apply (eq. "KPAx"), regularization operator
(eq. "deriv"), shrink formulas, CGLS (Algorithm 5) and split Bregman
(Algorithms 3 and 4), plus the quality metrics and the Philox generator."""
import json
import os

import numpy as np
import pytest
import scipy.optimize

import workloads as wl
from oracle import kpsvd, metrics, operator as op, philox, sb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _full_factors(P, cu, cv, n):
    s, U, V = op.exact_kpsvd(P, cu, cv, n)
    return kpsvd.kp_terms(s, U, V, n)


@pytest.mark.parametrize("n,seed", [(5, 1), (8, 2), (11, 3)])
def test_kp_apply_full_rank_equals_explicit_A(n, seed):
    P, cu, cv = wl.random_psf(5, 4, seed)
    A = op.blur_matrix(P, cu, cv, n)
    Ax, Ay = _full_factors(P, cu, cv, n)
    X = np.random.default_rng(seed).standard_normal((n, n))
    x = X.flatten(order="F")
    Y = sb.kp_apply(Ax, Ay, X)
    assert np.allclose(Y.flatten(order="F"), A @ x, rtol=0, atol=1e-13)
    Yt = sb.kp_apply(Ax, Ay, X, transpose=True)
    assert np.allclose(Yt.flatten(order="F"), A.T @ x, rtol=0, atol=1e-13)
    # and the direct convolution of the image
    assert np.allclose(Y, wl.blur_zero_bc(P, cu, cv, X), rtol=0, atol=1e-13)


def test_regularization_operator_orientation():
    n = 6
    L = sb.reg_matrix(n)
    x = np.arange(1.0, n + 1)
    assert np.allclose(L @ x, np.r_[-0.5 * np.ones(n - 1), 0.5 * n])
    X = np.random.default_rng(0).standard_normal((n, n))
    vx = X.flatten(order="F")
    # (L_x (x) I) vec(X) = vec(X L^T): horizontal differences along each row
    assert np.allclose(np.kron(L, np.eye(n)) @ vx, (X @ L.T).flatten(order="F"))
    assert np.allclose((X @ L.T)[:, 0], 0.5 * (X[:, 0] - X[:, 1]))
    # (I (x) L_y) vec(X) = vec(L X): vertical differences along each column
    assert np.allclose(np.kron(np.eye(n), L) @ vx, (L @ X).flatten(order="F"))
    assert np.allclose((L @ X)[0], 0.5 * (X[0] - X[1]))


def test_augmented_operator_adjoint_dot_test():
    n = 7
    P, cu, cv = wl.random_psf(3, 5, 4)
    Ax, Ay = _full_factors(P, cu, cv, n)
    aug = sb.Augmented(lambda X: sb.kp_apply(Ax, Ay, X),
                       lambda X: sb.kp_apply(Ax, Ay, X, True), n, 0.37)
    rng = np.random.default_rng(1)
    w = rng.standard_normal((n, n))
    r = tuple(rng.standard_normal((n, n)) for _ in range(3))
    lhs = sum(np.sum(a * b) for a, b in zip(aug.fwd(w), r))
    rhs = np.sum(w * aug.adj(r))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_cgls_converges_to_least_squares_and_residual_decreases():
    n = 6
    P, cu, cv = wl.random_psf(3, 3, 8)
    A = op.blur_matrix(P, cu, cv, n)
    L = sb.reg_matrix(n)
    lam = 0.3
    Ahat = np.vstack([A, lam * np.kron(L, np.eye(n)), lam * np.kron(np.eye(n), L)])
    rng = np.random.default_rng(2)
    bhat = tuple(rng.standard_normal((n, n)) for _ in range(3))
    bvec = np.concatenate([b.flatten(order="F") for b in bhat])
    x_ls = np.linalg.lstsq(Ahat, bvec, rcond=None)[0]
    aug = sb.Augmented(lambda X: (A @ X.flatten(order="F")).reshape(n, n, order="F"),
                       lambda X: (A.T @ X.flatten(order="F")).reshape(n, n, order="F"), n, lam)
    x, it, hist = sb.cgls(aug, bhat, I_max=200)
    assert np.allclose(x.flatten(order="F"), x_ls, rtol=0, atol=1e-8)
    assert np.all(np.diff(hist) <= 1e-12)


def test_cgls_delta_psf_without_regularization_is_one_step():
    n = 5
    b = np.random.default_rng(3).standard_normal((n, n))
    ident = lambda X: X
    aug = sb.Augmented(ident, ident, n, 0.0)
    x, it, _ = sb.cgls(aug, (b, 0 * b, 0 * b), I_max=1)
    assert it == 1 and np.allclose(x, b, atol=1e-15)


def test_aniso_shrink_solves_its_scalar_problem():
    # shrink(c, 1/gamma) minimizes (gamma/2)(d - c)^2 + |d|; the objective
    # gamma (d - c)^2 + |d| written beside eq. "d thresholding ani" would need
    # threshold 1/(2 gamma). The printed 1/gamma is implemented.
    gamma = 2.0
    for c in (-2.0, -0.7, -0.3, 0.0, 0.2, 0.45, 0.55, 3.0):
        d_brute = scipy.optimize.minimize_scalar(lambda d: 0.5 * gamma * (d - c) ** 2 + abs(d),
                                                 bounds=(-5, 5), method="bounded",
                                                 options={"xatol": 1e-12}).x
        assert abs(sb.shrink(np.array([c]), 1.0 / gamma)[0] - d_brute) < 1e-7
        d_half = scipy.optimize.minimize_scalar(lambda d: gamma * (d - c) ** 2 + abs(d),
                                                bounds=(-5, 5), method="bounded",
                                                options={"xatol": 1e-12}).x
        assert abs(sb.shrink(np.array([c]), 0.5 / gamma)[0] - d_half) < 1e-7


def test_iso_shrink_brute_force_and_reduction_to_aniso():
    gamma = 1.5
    rng = np.random.default_rng(5)
    for _ in range(6):
        c = rng.standard_normal(2)
        f = lambda d: 0.5 * gamma * np.sum((d - c) ** 2) + np.linalg.norm(d)
        d_b = scipy.optimize.minimize(f, c, method="Nelder-Mead",
                                      options={"xatol": 1e-12, "fatol": 1e-14}).x
        dx, dy = sb.iso_shrink(np.array([c[0]]), np.array([c[1]]), 1.0 / gamma)
        assert np.allclose([dx[0], dy[0]], d_b, atol=1e-6)
    cx = rng.standard_normal(50)
    dx, dy = sb.iso_shrink(cx, np.zeros(50), 0.4)
    assert np.allclose(dx, sb.shrink(cx, 0.4), atol=1e-15) and np.all(dy == 0)
    dx, dy = sb.iso_shrink(np.zeros(3), np.zeros(3), 0.4)
    assert np.all(dx == 0) and np.all(dy == 0)


@pytest.mark.parametrize("kind", ["aniso", "iso"])
def test_sb_with_full_rank_factors_equals_sb_with_explicit_A(kind):
    n = 16
    P, cu, cv = wl.gaussian_psf(n)
    A = op.blur_matrix(P, cu, cv, n)
    Ax, Ay = _full_factors(P, cu, cv, n)
    x_true = wl.rectangles_image(n, seed=2000)
    b = wl.add_noise(wl.blur_zero_bc(P, cu, cv, x_true), 0.01, seed=3000)
    lam, gamma = 0.115, 2.0
    beta = lam * lam / gamma
    fA = lambda X: (A @ X.flatten(order="F")).reshape(n, n, order="F")
    fAt = lambda X: (A.T @ X.flatten(order="F")).reshape(n, n, order="F")
    # I_max stays below the CGLS convergence point: past it the iteration runs
    # on rounding noise and two exact-arithmetic-equal operators drift apart.
    r1 = sb.split_bregman(kind, fA, fAt, b, lam, beta, L_max=8, I_max=12)
    r2 = sb.split_bregman(kind, lambda X: sb.kp_apply(Ax, Ay, X),
                          lambda X: sb.kp_apply(Ax, Ay, X, True), b, lam, beta,
                          L_max=8, I_max=12)
    assert np.linalg.norm(r1["x"] - r2["x"]) <= 1e-10 * np.linalg.norm(r1["x"])
    assert r1["iota_total"] == 96 and r1["l_end"] == 8
    # the restoration improves on the data
    assert metrics.rel_error(r2["x"], x_true) < metrics.rel_error(b, x_true)


def test_sb_tolerances_stop_early():
    n = 16
    P, cu, cv = wl.gaussian_psf(n)
    Ax, Ay = _full_factors(P, cu, cv, n)
    x_true = wl.rectangles_image(n, seed=2001)
    b = wl.add_noise(wl.blur_zero_bc(P, cu, cv, x_true), 0.01, seed=3001)
    out = sb.split_bregman("iso", lambda X: sb.kp_apply(Ax, Ay, X),
                           lambda X: sb.kp_apply(Ax, Ay, X, True), b, 0.115,
                           0.115 ** 2 / 2, L_max=50, tau_sb=1e-2, I_max=100, tau_cgls=1e-4)
    assert out["l_end"] < 50 and out["rc_sb"] < 1e-2
    assert all(rc >= 1e-2 for rc in out["rc_hist"][:-1])
    assert out["iota_total"] < 100 * out["l_end"]


def test_metrics_closed_forms():
    rng = np.random.default_rng(7)
    x_true = rng.standard_normal((8, 8))
    assert metrics.rel_error(2 * x_true, x_true) == pytest.approx(1.0)
    b = x_true + 0.1 * rng.standard_normal((8, 8))
    assert metrics.isnr(b, x_true, b) == pytest.approx(0.0)
    b_true = rng.standard_normal((8, 8))
    bn = wl.add_noise(b_true, 0.07, seed=9)
    assert metrics.snr(b_true, bn) == pytest.approx(-20 * np.log10(0.07))


def test_kp_rel_error_expansion_matches_explicit():
    n = 8
    P, cu, cv = wl.random_psf(5, 6, 12)
    R = op.rearrange(op.blur_matrix(P, cu, cv, n), n, n, n, n)
    U, s, Vt = np.linalg.svd(R)
    rng = np.random.default_rng(0)
    Up = U[:, :4] + 1e-2 * rng.standard_normal((n * n, 4))
    Vp = Vt[:4].T + 1e-2 * rng.standard_normal((n * n, 4))
    ref = np.linalg.norm(R - Up @ np.diag(s[:4]) @ Vp.T) / np.linalg.norm(R)
    assert metrics.kp_rel_error(P, cu, cv, n, s[:4], Up, Vp) == pytest.approx(ref, rel=1e-10)


def test_philox_known_answer_vectors():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        ctr = np.array([[int(v, 16) for v in case["ctr"]]], dtype=np.uint64)
        key = [int(v, 16) for v in case["key"]]
        out = philox.philox4x32_10(ctr, key)[0]
        assert [int(v) for v in out] == [int(v, 16) for v in case["out"]]


def test_philox_normals_are_standard_and_stream_distinct():
    z = philox.normals(400001, seed=123, stream=5)
    assert len(z) == 400001
    assert abs(z.mean()) < 5e-3 and abs(z.std() - 1) < 5e-3
    z2 = philox.normals(1000, seed=123, stream=6)
    assert not np.allclose(z[:1000], z2)
    assert np.array_equal(philox.normals(10, 123, 5), z[:10])


# ---------------------------------------------------------------------------
# the loop against the mathematics: Algorithms 3/4 converge to the minimizer of
# ||A x - b||^2 + 2 beta TV(x) (the factor 2 from the printed threshold 1/gamma),
# computed independently through the Lagrange dual and certified by its
# duality gap (tests/_sb_pins.py)

@pytest.mark.parametrize("kind", ["aniso", "iso"])
def test_sb_converges_to_certified_tv_minimizer(kind):
    from _sb_pins import loop_error
    err = loop_error(sb, kind)
    assert err <= 1e-6, err


@pytest.mark.parametrize("kind", ["aniso", "iso"])
def test_tv_minimizer_changes_with_beta(kind):
    # the pin resolves the regularization weight: doubling beta (the printed
    # threshold's factor 2, or gamma inverted) moves the minimizer by far more
    # than the 1e-6 gate
    from _sb_pins import BETA, problem, tv_minimizer
    A, b = problem()
    x1, _ = tv_minimizer(kind, A, b, BETA)
    x2, _ = tv_minimizer(kind, A, b, 2 * BETA)
    assert np.linalg.norm(x1 - x2) >= 1e-2 * np.linalg.norm(x1)
