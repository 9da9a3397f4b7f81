"""Pins for the oracle's EGKB (Algorithm 1), RSVD (Algorithm 2), Rayleigh-Ritz
refinement and Kronecker terms (eq. "KP approx").

Pins: the Lanczos relation B Q = S C, orthogonality, exactness once the
Krylov/sketch space contains the range (rank(R) <= k_p), interlacing, the
Eckart-Young optimum, a hand-computed firing index of the nu rule, and the
Kronecker-product theorem for the assembled terms.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import kpsvd, operator as op
from oracle.metrics import kp_rel_error


def _ops(P, cu, cv, n):
    return (lambda X: op.rmat_struct_apply(P, cu, cv, n, X),
            lambda X: op.rmat_struct_apply(P, cu, cv, n, X, transpose=True))


@pytest.mark.parametrize("reorth", ["full", "one_sided"])
def test_egkb_lanczos_relation_and_orthogonality(reorth):
    n = 24
    P, cu, cv = wl.speckle_psf(n, seed=1001)
    R, Rt = _ops(P, cu, cv, n)
    y = wl.gaussian_block(n * n, 1, seed=4001)[:, 0]
    out = kpsvd.egkb(R, Rt, y, k=8, p=8, reorth=reorth)
    S, Q, C = out["S"], out["Q"], out["C"]
    s1 = op.exact_kpsvd(P, cu, cv, n, 1)[0][0]
    assert S.shape == (n * n, 17) and Q.shape == (n * n, 16) and C.shape == (17, 16)
    assert np.linalg.norm(R(Q) - S @ C) <= 1e-12 * s1
    assert np.abs(Q.T @ Q - np.eye(16)).max() <= 1e-12
    if reorth == "full":
        assert np.abs(S.T @ S - np.eye(17)).max() <= 1e-12
    # C is lower bidiagonal with non-negative entries
    assert np.all(np.triu(C, 1) == 0) and np.all(np.tril(C, -2) == 0)
    assert np.all(np.diag(C) >= 0) and np.all(np.diag(C, -1) >= 0)
    # first right Lanczos vector is the normalized R^T y
    q1 = Rt(y)
    assert np.allclose(Q[:, 0], q1 / np.linalg.norm(q1), atol=1e-14)


def test_egkb_ritz_values_interlace_and_converge():
    n = 24
    P, cu, cv = wl.speckle_psf(n, seed=1002)
    R, Rt = _ops(P, cu, cv, n)
    y = wl.gaussian_block(n * n, 1, seed=4002)[:, 0]
    s_ex = op.exact_kpsvd(P, cu, cv, n)[0]
    out = kpsvd.egkb(R, Rt, y, k=5, p=15)
    sig = out["sigma_all"]
    assert np.all(sig <= s_ex[:len(sig)] * (1 + 1e-12) + 1e-14)
    assert np.allclose(out["sigma"], s_ex[:5], rtol=1e-8)
    # one-sided and full reorthogonalization agree in float64
    out1 = kpsvd.egkb(R, Rt, y, k=5, p=15, reorth="one_sided")
    assert np.allclose(out1["sigma"], out["sigma"], rtol=1e-10)


def test_egkb_exact_when_krylov_space_contains_range_with_breakdown():
    # The r=8 disk has Kronecker rank 6: with k_p = 8 > 6 the process breaks
    # down; the restart keeps the relation and the 6 nonzero sigmas are exact.
    n = 20
    P, cu, cv = wl.disk_psf(n)
    R, Rt = _ops(P, cu, cv, n)
    y = wl.gaussian_block(n * n, 1, seed=4003)[:, 0]
    out = kpsvd.egkb(R, Rt, y, k=6, p=2, seed=7)
    s_ex = op.exact_kpsvd(P, cu, cv, n)[0]
    assert out["breakdowns"], "expected a breakdown beyond the Kronecker rank"
    assert np.allclose(out["sigma"], s_ex[:6], rtol=1e-12)
    assert np.linalg.norm(R(out["Q"]) - out["S"] @ out["C"]) <= 1e-12 * s_ex[0]
    assert np.abs(out["Q"].T @ out["Q"] - np.eye(out["Q"].shape[1])).max() <= 1e-12
    err = kp_rel_error(P, cu, cv, n, out["sigma"], out["U"], out["V"])
    assert err <= 1e-7


def test_egkb_forced_breakdown_follows_requested_steps():
    n = 16
    P, cu, cv = wl.speckle_psf(n, seed=1003)
    R, Rt = _ops(P, cu, cv, n)
    y = wl.gaussian_block(n * n, 1, seed=4004)[:, 0]
    out = kpsvd.egkb(R, Rt, y, k=4, p=4, force_breakdown={("s", 3)}, seed=3)
    assert out["breakdowns"] == [("s", 3)]
    assert out["t"][2] == 0.0
    assert np.abs(out["S"].T @ out["S"] - np.eye(9)).max() <= 1e-12


def _bidiag(alpha, t):
    """Lower bidiagonal B ((m+1) x m) whose GKB from e_1 reproduces alpha, t."""
    m = len(alpha)
    B = np.zeros((m + 1, m))
    for i in range(m):
        B[i, i] = alpha[i]
        B[i + 1, i] = t[i + 1]
    return B


def test_nu_rule_fires_at_hand_computed_index():
    # t_j = 1, alpha_j = zeta_j. nu_{j+1} = sqrt(zeta_j zeta_{j-1}):
    # nu3 = .707, nu4 = .387, nu5 = .245, nu6 = .224, nu7 = sqrt(.4*.25) = .316
    # -> first rise at j = 6, so k = 6 and k_p = 6 + p.
    zeta = [1.0, 0.5, 0.3, 0.2, 0.25, 0.4, 0.1, 0.05, 0.04, 0.03, 0.02, 0.01, 0.01, 0.01]
    B = _bidiag(zeta, [1.0] * (len(zeta) + 1))
    y = np.zeros(B.shape[0])
    y[0] = 1.0
    R = lambda X: B @ X
    Rt = lambda X: B.T @ X
    out = kpsvd.egkb(R, Rt, y, k=10, p=2, auto_k=True)
    assert np.allclose(out["alpha"][:6], zeta[:6], atol=1e-15)
    assert out["k"] == 6 and out["kp"] == 8
    # k_min guard postpones the test until j > k_min
    out2 = kpsvd.egkb(R, Rt, y, k=10, p=2, auto_k=True, k_min=6)
    # after j = 6: nu8 = sqrt(.1*.4) = .2 < nu7 (.316); nu9 = sqrt(.05*.1) = .0707;
    # nu10 = sqrt(.04*.05) = .0447; nu11 = .0346; nu12 = .0245; nu13 = .0141;
    # nu14 = sqrt(.01*.01) = .01 < .0141; never rises -> k stays 10
    assert out2["k"] == 10 and out2["kp"] == 12
    # threshold clause: nu_j < tau fires at the first j > k_min with nu_j < tau
    out3 = kpsvd.egkb(R, Rt, y, k=10, p=2, auto_k=True, k_min=6, tau=0.05)
    # j = 7: nu7 = .316; j = 8: nu8 = .2; j = 9: nu9 = .0707; j = 10: nu10 = .0447 < .05
    assert out3["k"] == 10
    out4 = kpsvd.egkb(R, Rt, y, k=12, p=2, auto_k=True, k_min=6, tau=0.05)
    assert out4["k"] == 10 and out4["kp"] == 12
    # the printed initialisation (zeta_1 = 1, nu_2 = 100) gives the same index here
    out5 = kpsvd.egkb(R, Rt, y, k=10, p=2, auto_k=True, literal_init=True)
    assert out5["k"] == 6


def test_rsvd_exact_for_low_rank_and_bounds():
    n = 20
    P, cu, cv = wl.disk_psf(n)
    R, Rt = _ops(P, cu, cv, n)
    F = wl.gaussian_block(n * n, 8, seed=4005)
    out = kpsvd.rsvd(R, Rt, F, k=6, q=1)
    s_ex = op.exact_kpsvd(P, cu, cv, n)[0]
    assert np.allclose(out["sigma"], s_ex[:6], rtol=1e-12)
    # general case: sigma_bar_i <= sigma_i and error >= Eckart-Young optimum
    P, cu, cv = wl.speckle_psf(n, seed=1004)
    R, Rt = _ops(P, cu, cv, n)
    s_ex = op.exact_kpsvd(P, cu, cv, n)[0]
    for q in (0, 1, 2):
        out = kpsvd.rsvd(R, Rt, wl.gaussian_block(n * n, 12, seed=4006), k=8, q=q)
        assert np.all(out["sigma"] <= s_ex[:8] * (1 + 1e-12))
        err = kp_rel_error(P, cu, cv, n, out["sigma"], out["U"], out["V"])
        opt = np.sqrt(np.sum(s_ex[8:] ** 2) / np.sum(s_ex ** 2))
        assert err >= opt * (1 - 1e-9)
        if q == 2:
            assert err <= 1.01 * opt
    # orthonormal factors
    assert np.abs(out["U"].T @ out["U"] - np.eye(8)).max() < 1e-12
    assert np.abs(out["V"].T @ out["V"] - np.eye(8)).max() < 1e-12
    # R V = U S on the converged leading triplet
    assert np.linalg.norm(R(out["V"][:, :1]) - out["U"][:, :1] * out["sigma"][0]) < 1e-6 * s_ex[0]


def test_refine_recovers_exact_triplets_and_improves_perturbed_subspace():
    n = 20
    P, cu, cv = wl.speckle_psf(n, seed=1005)
    R, Rt = _ops(P, cu, cv, n)
    s_ex, U_ex, V_ex = op.exact_kpsvd(P, cu, cv, n, 10)
    out = kpsvd.refine(R, V_ex)
    assert np.allclose(out["sigma"], s_ex, rtol=1e-12)
    # columns perturbed by ~1e-3 in norm: the Ritz values err at second order
    pert = V_ex + 1e-3 / n * np.random.default_rng(0).standard_normal(V_ex.shape)
    out = kpsvd.refine(R, pert)
    e_ref = np.abs(out["sigma"] - s_ex).max() / s_ex[0]
    assert e_ref < 1e-5
    assert np.all(out["sigma"] <= s_ex * (1 + 1e-12))


def test_refine_on_a_rotated_exact_subspace_returns_the_exact_triplets():
    # V = V_exact Q with a random orthogonal Q spans the exact subspace but
    # mixes its directions: the refinement must undo the mixing, giving the
    # exact right and left singular vectors (up to sign) and B V_r = U_r S_r
    n = 20
    P, cu, cv = wl.speckle_psf(n, seed=1005)
    R, Rt = _ops(P, cu, cv, n)
    k = 8
    s_ex, U_ex, V_ex = op.exact_kpsvd(P, cu, cv, n, k)
    assert np.all(np.diff(s_ex) < -1e-3 * s_ex[0])           # distinct sigma
    Qm, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((k, k)))
    out = kpsvd.refine(R, V_ex @ Qm)
    assert np.allclose(out["sigma"], s_ex, rtol=1e-12)
    for i in range(k):
        sg = np.sign(out["V"][:, i] @ V_ex[:, i])
        assert np.abs(out["V"][:, i] - sg * V_ex[:, i]).max() <= 1e-10
        assert np.abs(out["U"][:, i] - sg * U_ex[:, i]).max() <= 1e-10


def test_refine_triplets_satisfy_b_v_equals_u_sigma_on_a_perturbed_subspace():
    n = 20
    P, cu, cv = wl.speckle_psf(n, seed=1006)
    R, Rt = _ops(P, cu, cv, n)
    k = 10
    s_ex, _, V_ex = op.exact_kpsvd(P, cu, cv, n, k)
    rng = np.random.default_rng(4)
    V = V_ex @ np.linalg.qr(rng.standard_normal((k, k)))[0] + 1e-2 * rng.standard_normal(V_ex.shape) / n
    out = kpsvd.refine(R, V)
    Vr, Ur, sr = out["V"], out["U"], out["sigma"]
    assert np.linalg.norm(R(Vr) - Ur * sr) <= 1e-12 * s_ex[0]
    assert np.abs(Vr.T @ Vr - np.eye(k)).max() <= 1e-13
    assert np.abs(Ur.T @ Ur - np.eye(k)).max() <= 1e-13
    # the refined directions lie in range(V)
    Qv = np.linalg.qr(V)[0]
    assert np.linalg.norm(Vr - Qv @ (Qv.T @ Vr)) <= 1e-13


def test_kp_terms_reconstruct_A_with_full_rank():
    n = 6
    P, cu, cv = wl.random_psf(4, 5, 21)
    A = op.blur_matrix(P, cu, cv, n)
    s, U, V = op.exact_kpsvd(P, cu, cv, n)
    Ax, Ay = kpsvd.kp_terms(s, U, V, n)
    assert np.abs(kpsvd.kp_approx_matrix(Ax, Ay) - A).max() <= 1e-13
    # sign convention: the largest-magnitude entry of every A_y is positive
    for t in range(Ay.shape[0]):
        flat = Ay[t].flatten(order="F")
        assert flat[np.argmax(np.abs(flat))] > 0


# ---------------------------------------------------------------------------
# block Golub-Kahan (the block analogue of Algorithm 1)

@pytest.mark.parametrize("b", [2, 4, 5])
def test_block_egkb_relation_orthogonality_and_structure(b):
    n = 16
    P, cu, cv = wl.speckle_psf(n, seed=1003)
    R, Rt = _ops(P, cu, cv, n)
    Y = wl.gaussian_block(n * n, b, seed=4003)
    out = kpsvd.block_egkb(R, Rt, Y, k=6, p=6)
    U, V, C, kp = out["Ub"], out["Vb"], out["C"], out["kp"]
    s1 = op.exact_kpsvd(P, cu, cv, n, 1)[0][0]
    assert kp % b == 0 and kp >= 12 and U.shape[1] == kp + b and V.shape[1] == kp
    assert np.linalg.norm(R(V) - U @ C) <= 1e-12 * s1          # B V = U C
    assert np.abs(U.T @ U - np.eye(kp + b)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(kp)).max() <= 1e-12
    # C is block lower bidiagonal: lower-triangular L_j on the diagonal,
    # upper-triangular R_j below it, zero elsewhere
    for j in range(kp // b):
        for i in range(kp // b + 1):
            blk = C[i * b:(i + 1) * b, j * b:(j + 1) * b]
            if i == j:
                assert np.all(np.triu(blk, 1) == 0)
            elif i == j + 1:
                assert np.all(np.tril(blk, -1) == 0)
            else:
                assert np.all(blk == 0)
    # the first right block spans B^T Y
    G = Rt(Y)
    assert np.linalg.norm(G - V[:, :b] @ (V[:, :b].T @ G)) <= 1e-12 * np.linalg.norm(G)


def test_block_egkb_with_one_vector_is_egkb():
    n = 12
    P, cu, cv = wl.speckle_psf(n, seed=1004)
    R, Rt = _ops(P, cu, cv, n)
    y = wl.gaussian_block(n * n, 1, seed=4004)
    blk = kpsvd.block_egkb(R, Rt, y, k=5, p=5)
    ref = kpsvd.egkb(R, Rt, y[:, 0], k=5, p=5, reorth="full")
    s1 = ref["sigma"][0]
    assert np.abs(blk["sigma"] - ref["sigma"]).max() <= 1e-12 * s1
    # the bidiagonal itself: alpha on the diagonal, t on the subdiagonal
    assert np.allclose(np.diag(blk["C"]), ref["alpha"], atol=1e-12 * s1)
    assert np.allclose(np.diag(blk["C"], -1), ref["t"][1:], atol=1e-12 * s1)


def test_block_egkb_exact_for_low_rank_and_interlacing():
    """kp >= rank(B): the Ritz values are the singular values (the disk PSF
    has Kronecker rank 6); below that they interlace."""
    n = 20
    P, cu, cv = wl.disk_psf(n, 8.0)
    R, Rt = _ops(P, cu, cv, n)
    exact = op.exact_kpsvd(P, cu, cv, n, 8)[0]
    Y = wl.gaussian_block(n * n, 3, seed=4005)
    out = kpsvd.block_egkb(R, Rt, Y, k=6, p=3)          # kp = 9 >= 6, breakdowns follow
    assert np.abs(out["sigma"][:6] - exact[:6]).max() <= 1e-12 * exact[0]
    assert len(out["breakdowns"]) > 0
    P2, cu2, cv2 = wl.speckle_psf(n, seed=1005)
    R2, Rt2 = _ops(P2, cu2, cv2, n)
    ex2 = op.exact_kpsvd(P2, cu2, cv2, n, 6)[0]
    out2 = kpsvd.block_egkb(R2, Rt2, Y, k=6, p=3)
    assert np.all(out2["sigma"] <= ex2 * (1 + 1e-12))


def test_block_egkb_forced_breakdown_keeps_the_relation():
    """A breakdown forced at one column of each basis stores 0 on C's diagonal
    there, restarts from the stated Philox stream and keeps both bases
    orthonormal (B V = U C no longer holds: the forced columns' residuals, which
    are not negligible here, are dropped)."""
    n, b = 14, 3
    P, cu, cv = wl.speckle_psf(n, seed=1006)
    R, Rt = _ops(P, cu, cv, n)
    Y = wl.gaussian_block(n * n, b, seed=4006)
    force = {("v", 4), ("u", 7)}
    out = kpsvd.block_egkb(R, Rt, Y, k=5, p=4, force_breakdown=force, seed=9)
    U, V, C, kp = out["Ub"], out["Vb"], out["C"], out["kp"]
    s1 = op.exact_kpsvd(P, cu, cv, n, 1)[0][0]
    assert sorted(out["breakdowns"]) == sorted(force)
    assert C[4, 4] == 0.0                      # column 4 of V: L_2^T diagonal
    assert C[7, 4] == 0.0                      # column 7 of U: R_2 diagonal (block 1 of V)
    assert np.abs(U.T @ U - np.eye(kp + b)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(kp)).max() <= 1e-12
    # columns before the first forced one still satisfy the relation
    assert np.linalg.norm(R(V[:, :3]) - U @ C[:, :3]) <= 1e-12 * s1
    # the restart direction is the stream-2(m+1)+1 Philox vector made orthogonal
    # to V[:, :4]: V[:, 4] is its normalized residual
    from oracle import philox
    g = philox.normals(n * n, 9, 2 * 5 + 1)
    g = g - V[:, :4] @ (V[:, :4].T @ g)
    assert np.allclose(V[:, 4], g / np.linalg.norm(g), atol=1e-12)


def test_block_stopping_rule_with_one_vector_is_algorithm_1():
    """With b = 1 the block rule is Algorithm 1's (same k, k_p, sigma), with
    the default and the printed initialization and with a tau clause."""
    zeta = [1.0, 0.5, 0.3, 0.2, 0.25, 0.4, 0.1, 0.05, 0.04, 0.03, 0.02, 0.01, 0.01, 0.01]
    B = _bidiag(zeta, [1.0] * (len(zeta) + 1))
    y = np.zeros(B.shape[0])
    y[0] = 1.0
    R = lambda X: B @ X
    Rt = lambda X: B.T @ X
    for kw in (dict(), dict(literal_init=True), dict(tau=0.3), dict(k_min=6)):
        ref = kpsvd.egkb(R, Rt, y, k=10, p=2, auto_k=True, **kw)
        blk = kpsvd.block_egkb(R, Rt, y[:, None], k=10, p=2, auto_k=True, **kw)
        assert (blk["k"], blk["kp"]) == (ref["k"], ref["kp"]), kw
        assert np.allclose(blk["sigma"], ref["sigma"], rtol=1e-13, atol=1e-15)


def test_block_stopping_rule_fires_at_hand_computed_block():
    """b = 2 on the direct sum of two bidiagonals started from their first
    rows: the block process interleaves the two single-vector processes, so
    block J holds the columns with alpha = a1[J-1], a2[J-1] and t = 1, and its
    zeta is sqrt(a1 a2) = (1, .5, .3, .2, .4, ...) by construction. Then
    nu_{J+1} = sqrt(zeta_J zeta_{J-1}) = .707, .387, .245, .283: the first rise
    is nu_6 > nu_5, at block 5, so k = 10, k_p = 12 -> 6 blocks of 2."""
    zb = np.array([1.0, 0.5, 0.3, 0.2, 0.4, 0.1, 0.05, 0.04, 0.03, 0.02])
    f = np.array([1.2, 1.2, 0.8, 1.5, 0.9, 1.1, 1.0, 1.3, 0.7, 1.0])
    a1, a2 = zb * f, zb / f
    B1 = _bidiag(a1, [1.0] * 11)
    B2 = _bidiag(a2, [1.0] * 11)
    B = np.zeros((22, 20))
    B[:11, :10] = B1
    B[11:, 10:] = B2
    Y = np.zeros((22, 2))
    Y[0, 0] = Y[11, 1] = 1.0
    R, Rt = (lambda X: B @ X), (lambda X: B.T @ X)
    out = kpsvd.block_egkb(R, Rt, Y, k=12, p=2, auto_k=True)
    assert out["k"] == 10 and out["kp"] == 12
    assert np.allclose([out["zeta"][J] for J in range(1, 6)], zb[:5], rtol=1e-14)
    # without the rule the same run keeps k = 12, k_p = 14
    out0 = kpsvd.block_egkb(R, Rt, Y, k=12, p=2)
    assert out0["k"] == 12 and out0["kp"] == 14
    # a tau above nu_3 = .707 fires at block 3 (the test at block 2 compares
    # nu_2 = +inf), so k = 6, k_p = 8
    out1 = kpsvd.block_egkb(R, Rt, Y, k=12, p=2, auto_k=True, tau=0.8)
    assert out1["k"] == 6 and out1["kp"] == 8
    # k_min = 10 postpones the test to blocks with J b > 10: none rises there
    # (zeta = .1, .05, ...), so k stays 12
    out2 = kpsvd.block_egkb(R, Rt, Y, k=12, p=2, auto_k=True, k_min=10)
    assert out2["k"] == 12
    # Ritz values: the decoupled Krylov spaces of the fired run are the leading
    # 6 x 7 sections of B1 and B2
    s1 = np.linalg.svd(B1[:7, :6], compute_uv=False)
    s2 = np.linalg.svd(B2[:7, :6], compute_uv=False)
    assert np.allclose(out["sigma_all"], np.sort(np.concatenate([s1, s2]))[::-1], rtol=1e-12)
