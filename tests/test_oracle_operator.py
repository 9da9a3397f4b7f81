"""Pins for the oracle's blur operator, rearrangement and exact Kronecker SVD.

Each check ties the oracle to something other than itself: the paper's literal
reordering (eq. "initial rearrange A"), an independent convolution routine,
the Kronecker-product SVD theorem (Theorem 12.3.1 of Golub-Van Loan as cited in
section 2.1), LAPACK on explicit matrices, and closed forms.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import operator as op

CASES = [(4, (3, 5), 1), (5, (5, 5), 2), (8, (6, 9), 3), (12, (23, 23), 4), (7, (2, 3), 5)]


def _psf(shape, seed):
    return wl.random_psf(shape[0], shape[1], seed)


@pytest.mark.parametrize("n,shape,seed", CASES)
def test_generator_equals_literal_reorder(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    A = op.blur_matrix(P, cu, cv, n)
    R = op.rearrange(A, n, n, n, n)
    idx = np.arange(n * n)
    Rg = op.rmat_entries(P, cu, cv, n, idx, idx)
    assert np.array_equal(R, Rg)


@pytest.mark.parametrize("n,shape,seed", CASES)
def test_blur_matrix_matches_independent_convolution(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    A = op.blur_matrix(P, cu, cv, n)
    X = np.random.default_rng(seed).standard_normal((n, n))
    B = wl.blur_zero_bc(P, cu, cv, X)
    Bm = (A @ X.flatten(order="F")).reshape(n, n, order="F")
    assert np.allclose(Bm, B, rtol=0, atol=1e-13)


def test_delta_psf_shifts_down_one_row():
    n = 6
    P = np.zeros((3, 3))
    P[2, 1] = 1.0          # vertical offset +1 from centre (1, 1)
    X = np.random.default_rng(0).standard_normal((n, n))
    A = op.blur_matrix(P, 1, 1, n)
    B = (A @ X.flatten(order="F")).reshape(n, n, order="F")
    assert np.array_equal(B[1:], X[:-1])
    assert np.array_equal(B[0], np.zeros(n))


@pytest.mark.parametrize("n,shape,seed", CASES[:4])
def test_kp_theorem_full_sum_reconstructs_A(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    A = op.blur_matrix(P, cu, cv, n)
    R = op.rearrange(A, n, n, n, n)
    U, s, Vt = np.linalg.svd(R)
    Ak = np.zeros_like(A)
    for i in range(len(s)):
        Ui = U[:, i].reshape(n, n, order="F")
        Vi = Vt[i].reshape(n, n, order="F")
        Ak += s[i] * np.kron(Ui, Vi)
    assert np.abs(Ak - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("n,shape,seed", CASES[:4])
def test_van_loan_pitsianis_identity(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    A = op.blur_matrix(P, cu, cv, n)
    R = op.rearrange(A, n, n, n, n)
    U, s, Vt = np.linalg.svd(R)
    for r in (1, 2, 3):
        Ar = sum(s[i] * np.kron(U[:, i].reshape(n, n, order="F"),
                                Vt[i].reshape(n, n, order="F")) for i in range(r))
        lhs = np.linalg.norm(A - Ar, "fro") ** 2
        rhs = np.sum(s[r:] ** 2)
        assert abs(lhs - rhs) <= 1e-12 * np.sum(s ** 2)


@pytest.mark.parametrize("n,shape,seed", CASES)
def test_exact_kpsvd_matches_lapack_on_explicit_R(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    R = op.rearrange(op.blur_matrix(P, cu, cv, n), n, n, n, n)
    s_ref = np.linalg.svd(R, compute_uv=False)
    s, U, V = op.exact_kpsvd(P, cu, cv, n)
    m = len(s)
    assert m == 2 * n - 1
    assert np.allclose(s, s_ref[:m], rtol=0, atol=1e-14 * s_ref[0])
    assert np.all(s_ref[m:] <= 1e-13 * s_ref[0])       # rank R(A) <= 2n - 1
    # singular vectors: R v_i = s_i u_i and orthonormality
    keep = s > 1e-10 * s[0]
    assert np.allclose(R @ V[:, keep], U[:, keep] * s[keep], atol=1e-13 * s[0])
    assert np.allclose(U[:, keep].T @ U[:, keep], np.eye(keep.sum()), atol=1e-12)


def test_separable_psf_is_rank_one_with_closed_form():
    n = 10
    a = np.array([0.1, 0.3, 0.4, 0.2])
    b = np.array([0.25, 0.5, 0.25, 0.05, 0.7])
    P, cu, cv = wl.separable_psf(a, b)
    s, U, V = op.exact_kpsvd(P, cu, cv, n)
    # closed form: R = E M E^T with M[d1, d2] = b[cv + d1] a[cu + d2], so
    # sigma_1 = sqrt(sum_d (n-|d|) b_d^2) sqrt(sum_d (n-|d|) a_d^2)
    d_a = np.arange(len(a)) - cu
    d_b = np.arange(len(b)) - cv
    s1 = np.sqrt(np.sum((n - np.abs(d_b)) * b ** 2)) * np.sqrt(np.sum((n - np.abs(d_a)) * a ** 2))
    assert abs(s[0] - s1) <= 1e-14 * s1
    assert s[1] <= 1e-14 * s[0]
    R = op.rearrange(op.blur_matrix(P, cu, cv, n), n, n, n, n)
    s_ref = np.linalg.svd(R, compute_uv=False)
    assert abs(s_ref[0] - s1) <= 1e-13 * s1 and s_ref[1] <= 1e-13 * s1


def test_motion_blur_along_axis_is_rank_one():
    n = 16
    P, cu, cv = wl.motion_psf(n, length=7, theta=0.0)
    s, _, _ = op.exact_kpsvd(P, cu, cv, n)
    assert s[1] <= 1e-14 * s[0]


def test_delta_psf_identity():
    n = 7
    P = np.ones((1, 1))
    s, U, V = op.exact_kpsvd(P, 0, 0, n)
    assert abs(s[0] - n) <= 1e-14 * n
    assert s[1] <= 1e-14
    Ui = U[:, 0].reshape(n, n, order="F")
    Vi = V[:, 0].reshape(n, n, order="F")
    assert np.allclose(np.abs(Ui), np.eye(n) / np.sqrt(n), atol=1e-15)
    assert np.allclose(np.abs(Vi), np.eye(n) / np.sqrt(n), atol=1e-15)
    A = op.blur_matrix(P, 0, 0, n)
    assert np.array_equal(A, np.eye(n * n))


def test_transpose_flip_and_scale_symmetries():
    n = 9
    P, cu, cv = wl.random_psf(5, 7, 11)
    s, U, V = op.exact_kpsvd(P, cu, cv, n)
    # transposed PSF with swapped centre gives R(A)^T: same sigma, roles swapped
    sT, UT, VT = op.exact_kpsvd(P.T, cv, cu, n)
    assert np.allclose(sT, s, atol=1e-14 * s[0])
    Rt = op.rmat_entries(P.T, cv, cu, n, np.arange(n * n), np.arange(n * n))
    R = op.rmat_entries(P, cu, cv, n, np.arange(n * n), np.arange(n * n))
    assert np.array_equal(Rt, R.T)
    # point reflection P(-u, -v) and scaling
    sF, _, _ = op.exact_kpsvd(P[::-1, ::-1], P.shape[0] - 1 - cu, P.shape[1] - 1 - cv, n)
    assert np.allclose(sF, s, atol=1e-14 * s[0])
    sS, _, _ = op.exact_kpsvd(3.5 * P, cu, cv, n)
    assert np.allclose(sS, 3.5 * s, atol=1e-14 * 3.5 * s[0])


@pytest.mark.parametrize("n,shape,seed", CASES)
def test_dense_and_struct_products_equal_explicit(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    R = op.rearrange(op.blur_matrix(P, cu, cv, n), n, n, n, n)
    X = np.random.default_rng(seed + 100).standard_normal((n * n, 3))
    for tr in (False, True):
        ref = (R.T if tr else R) @ X
        d = op.rmat_dense_apply(P, cu, cv, n, X, transpose=tr, row_chunk=7)
        s = op.rmat_struct_apply(P, cu, cv, n, X, transpose=tr)
        assert np.allclose(d, ref, rtol=0, atol=1e-13)
        assert np.allclose(s, ref, rtol=0, atol=1e-13)
        sv = op.rmat_struct_apply(P, cu, cv, n, X[:, 0], transpose=tr)
        assert np.allclose(sv, ref[:, 0], rtol=0, atol=1e-13)


def test_struct_product_matches_generated_rows_at_n128():
    n = 128
    P, cu, cv = wl.gaussian_psf(n)
    X = np.random.default_rng(3).standard_normal((n * n, 2))
    Y = op.rmat_struct_apply(P, cu, cv, n, X)
    rows = np.random.default_rng(4).choice(n * n, 40, replace=False)
    ref = op.rmat_entries(P, cu, cv, n, rows, np.arange(n * n)) @ X
    assert np.allclose(Y[rows], ref, rtol=0, atol=1e-13)
    Yt = op.rmat_struct_apply(P, cu, cv, n, X, transpose=True)
    cols = rows
    reft = op.rmat_entries(P, cu, cv, n, np.arange(n * n), cols).T @ X
    assert np.allclose(Yt[cols], reft, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n,shape,seed", CASES)
def test_frobenius_norm_closed_form(n, shape, seed):
    P, cu, cv = _psf(shape, seed)
    A = op.blur_matrix(P, cu, cv, n)
    assert abs(op.rmat_fro_norm2(P, cu, cv, n) - np.sum(A * A)) <= 1e-13 * np.sum(A * A)


def test_configured_psfs_are_normalized_and_nonseparable():
    n = 32
    for P, cu, cv in (wl.gaussian_psf(n), wl.disk_psf(n), wl.speckle_psf(n, seed=1000),
                      wl.motion_psf(n, theta=0.3)):
        assert P.shape == (2 * n - 1, 2 * n - 1) and (cu, cv) == (n - 1, n - 1)
        assert abs(P.sum() - 1.0) < 1e-12 and P.min() >= 0
        s, _, _ = op.exact_kpsvd(P, cu, cv, n)
        assert s[1] > 1e-6 * s[0]
    # The Kronecker rank equals rank(P). The r=8 disk (pixel-centre inclusion)
    # has rows that are centred intervals of half-widths 8, 7, 6, 5, 3, 0 (the
    # floor of sqrt(64 - u^2)), i.e. 6 distinct independent rows.
    P, cu, cv = wl.disk_psf(n)
    widths = {int(np.floor(np.sqrt(64 - u * u))) for u in range(-8, 9)}
    assert len(widths) == 6
    s, _, _ = op.exact_kpsvd(P, cu, cv, n)
    assert s[5] > 1e-8 * s[0] and s[6] < 1e-12 * s[0]


@pytest.mark.parametrize("n,shape,seed", [(6, (3, 5), 1), (9, (7, 7), 2), (12, (11, 5), 3)])
def test_reflexive_blur_matrix_is_ndimage_reflect_convolution(n, shape, seed):
    """Reflexive boundary conditions (half-sample symmetric extension): the
    explicit matrix against scipy.ndimage.convolve(mode="reflect"), an
    independent implementation; mode="constant" reproduces the zero-BC matrix."""
    import scipy.ndimage as nd
    rng = np.random.default_rng(seed)
    P = rng.uniform(0, 1, shape)
    cu, cv = shape[0] // 2, shape[1] // 2          # ndimage's kernel centre
    X = rng.standard_normal((n, n))
    Ar = op.blur_matrix_reflexive(P, cu, cv, n)
    Az = op.blur_matrix(P, cu, cv, n)
    vec = lambda M: M.flatten(order="F")
    assert np.allclose(Ar @ vec(X), vec(nd.convolve(X, P, mode="reflect")), rtol=0, atol=1e-12)
    assert np.allclose(Az @ vec(X), vec(nd.convolve(X, P, mode="constant", cval=0.0)),
                       rtol=0, atol=1e-12)
    # the reflected part is a nonzero, separately structured correction
    assert np.abs(Ar - Az).max() > 1e-3


def test_reflexive_blur_of_constant_image_is_constant():
    """With a unit-sum PSF whose extent is below n, reflection preserves a
    constant image exactly (no boundary darkening, unlike zero BC)."""
    n = 10
    P = np.random.default_rng(4).uniform(0, 1, (5, 7))
    P /= P.sum()
    Ar = op.blur_matrix_reflexive(P, 2, 3, n)
    assert np.allclose(Ar @ np.ones(n * n), 1.0, atol=1e-13)


@pytest.mark.parametrize("n,shape,centre,seed", [(6, (3, 5), None, 1), (5, (9, 9), None, 2),
                                                 (5, (13, 11), None, 3), (3, (13, 13), (6, 6), 4),
                                                 (4, (3, 9), (0, 8), 5)])
def test_periodic_blur_matrix_is_circular_convolution(n, shape, centre, seed):
    """Periodic boundary conditions: A is block circulant with circulant
    blocks, i.e. a circular convolution with the PSF aliased onto the n x n
    torus, computed here by the 2-D FFT. PSFs reaching up to 2n pixels from
    their centre (the extent the image set covers) are included."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(-1, 1, shape)
    cu, cv = centre if centre else (shape[0] // 2, shape[1] // 2)
    Ap = op.blur_matrix_periodic(P, cu, cv, n)
    K = np.zeros((n, n))
    for u in range(shape[0]):
        for v in range(shape[1]):
            K[(u - cu) % n, (v - cv) % n] += P[u, v]
    X = rng.standard_normal((n, n))
    Y = np.real(np.fft.ifft2(np.fft.fft2(K) * np.fft.fft2(X)))
    vec = lambda M: M.flatten(order="F")
    assert np.allclose(Ap @ vec(X), vec(Y), rtol=0, atol=1e-12)
    if centre is None:                   # ndimage's kernel centre convention
        import scipy.ndimage as nd
        assert np.allclose(Ap @ vec(X), vec(nd.convolve(X, P, mode="grid-wrap")), rtol=0,
                           atol=1e-12)


@pytest.mark.parametrize("n,shape,seed", [(5, (9, 9), 6), (4, (9, 7), 7), (5, (13, 11), 8)])
def test_reflexive_blur_matrix_with_psf_larger_than_the_image(n, shape, seed):
    """PSFs larger than the image reflect more than once; the image set of
    the oracle still reproduces scipy.ndimage.convolve(mode="reflect")."""
    import scipy.ndimage as nd
    rng = np.random.default_rng(seed)
    P = rng.uniform(0, 1, shape)
    Ar = op.blur_matrix_reflexive(P, shape[0] // 2, shape[1] // 2, n)
    X = rng.standard_normal((n, n))
    vec = lambda M: M.flatten(order="F")
    assert np.allclose(Ar @ vec(X), vec(nd.convolve(X, P, mode="reflect")), rtol=0, atol=1e-12)


@pytest.mark.parametrize("bc", ["zero", "reflexive", "periodic"])
def test_rmat_entries_with_boundary_conditions_are_the_rearranged_matrix(bc):
    """R(A) entries generated from the PSF equal the literal reorder of the
    explicit blur matrix (integer PSF, so every sum is exact)."""
    n = 7
    rng = np.random.default_rng(9)
    P = rng.integers(-5, 6, (9, 13)).astype(np.float64)
    cu, cv = 2, 9
    A = {"zero": op.blur_matrix, "reflexive": op.blur_matrix_reflexive,
         "periodic": op.blur_matrix_periodic}[bc](P, cu, cv, n)
    R = op.rearrange(A, n, n, n, n)
    N = n * n
    assert np.array_equal(op.rmat_entries(P, cu, cv, n, np.arange(N), np.arange(N), bc), R)
    X = rng.standard_normal((N, 3))
    assert np.allclose(op.rmat_dense_apply(P, cu, cv, n, X, bc=bc, row_chunk=10), R @ X,
                       rtol=0, atol=1e-12)
    assert np.allclose(op.rmat_dense_apply(P, cu, cv, n, X, transpose=True, bc=bc, row_chunk=10),
                       R.T @ X, rtol=0, atol=1e-12)


def test_periodic_blur_of_constant_image_is_constant():
    """A unit-sum PSF of any extent up to 2n maps a constant image to itself
    under periodic boundary conditions."""
    n = 4
    P = np.random.default_rng(10).uniform(0, 1, (15, 11))
    P /= P.sum()
    Ap = op.blur_matrix_periodic(P, 7, 3, n)
    assert np.allclose(Ap @ np.ones(n * n), 1.0, atol=1e-13)


@pytest.mark.parametrize("n,shape,seed", [(2, (1, 1), 0), (7, (3, 5), 1), (12, (9, 13), 2),
                                          (16, (31, 31), 3), (10, (4, 25), 4)])
def test_window_product_equals_explicit_R(n, shape, seed):
    """The window form of the dense product (blocks of R read as windows of the
    padded transposed PSF) against the explicit R(A) of the paper's
    rearrangement, including PSFs smaller and larger than the image and
    off-centre centres, and a subset of block rows."""
    P, cu, cv = wl.random_psf(shape[0], shape[1], seed)
    A = op.blur_matrix(P, cu, cv, n)
    R = op.rearrange(A, n, n, n, n)
    X = np.random.default_rng(seed).standard_normal((n * n, 3))
    Y = op.rmat_window_apply(P, cu, cv, n, X)
    assert np.abs(Y - R @ X).max() <= 1e-13 * max(1.0, np.abs(R @ X).max())
    js = range(1, n, 2)
    Yb = op.rmat_window_apply(P, cu, cv, n, X[:, 0], blocks=js)
    rows = np.concatenate([np.arange(n * j, n * j + n) for j in js])
    assert np.allclose(Yb[rows], (R @ X[:, 0])[rows], rtol=0, atol=1e-13)
    other = np.setdiff1d(np.arange(n * n), rows)
    assert np.all(Yb[other] == 0.0)
