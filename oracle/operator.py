"""Blur operator A, its rearrangement R(A), and exact Kronecker SVD (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Notation (section 2.1 of the paper, with m1 = m2 = n1 = n2 = n as in its
experimental design): A is N x N with N = n^2, partitioned into n x n blocks
A_{i,j} (eq. "block A for KP"); vec is column-major; row i + n*j of R(A) is
vec(A_{i,j})^T (eq. "initial rearrange A").

The zero-boundary blur with PSF P (centre (cu, cv)) has entries
A[r + n*i, c + n*j] = P[cu + r - c, cv + i - j] (0 outside P), so
R[i + n*j, r + n*c] = P[cu + r - c, cv + i - j].
"""
from __future__ import annotations

import numpy as np


def _psf_at(P, cu, cv, du, dv):
    """P[cu + du, cv + dv] with zeros outside the array (arrays du, dv)."""
    pu, pv = P.shape
    uu, vv = np.broadcast_arrays(cu + np.asarray(du), cv + np.asarray(dv))
    ok = (uu >= 0) & (uu < pu) & (vv >= 0) & (vv < pv)
    out = np.zeros(uu.shape, dtype=P.dtype)
    out[ok] = P[uu[ok], vv[ok]]
    return out


def blur_matrix(P, cu, cv, n):
    """Explicit zero-BC blur matrix A (n^2 x n^2), block by block.

    Block A_{i,j} (block row i, block column j) has entries
    A_{i,j}[r, c] = P[cu + r - c, cv + i - j]: the image pixel (r, i) of the
    output (r vertical) collects pixel (c, j) of the input.
    """
    N = n * n
    A = np.zeros((N, N), dtype=P.dtype)
    r = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    for i in range(n):
        for j in range(n):
            A[n * i:n * i + n, n * j:n * j + n] = _psf_at(P, cu, cv, r - c,
                                                         np.full((1, 1), i - j))
    return A


def _reflect_images(k, n):
    """Positions that the half-sample symmetric (reflexive) extension of a
    length-n signal maps onto index k: k + 2nm and -1 - k + 2nm, m = -1, 0, 1
    (enough for PSF extents below 3n)."""
    return [k + 2 * n * m for m in (-1, 0, 1)] + [-1 - k + 2 * n * m for m in (-1, 0, 1)]


def blur_matrix_reflexive(P, cu, cv, n):
    """Explicit reflexive-BC blur matrix (n^2 x n^2): the image is extended
    beyond its edges by reflection about the edge of the last pixel
    (x[-1 - k] = x[k], x[n + k] = x[n - 1 - k]), so

        A[r + n*i, c + n*j] = sum over images c~ of c and j~ of j of
                              P[cu + r - c~, cv + i - j~].
    """
    N = n * n
    A = np.zeros((N, N), dtype=P.dtype)
    r = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    cimg = _reflect_images(c, n)           # list of (1, n) arrays
    for i in range(n):
        for j in range(n):
            blk = np.zeros((n, n), dtype=P.dtype)
            for jj in _reflect_images(j, n):
                for cc in cimg:
                    blk += _psf_at(P, cu, cv, r - cc, np.full((1, 1), i - jj))
            A[n * i:n * i + n, n * j:n * j + n] = blk
    return A


def _periodic_images(k, n):
    """Positions that the periodic extension of a length-n signal maps onto
    index k: k + nm, m = -2 .. 2 (enough for PSFs reaching at most 2n pixels
    from their centre)."""
    return [k + n * m for m in (-2, -1, 0, 1, 2)]


def blur_matrix_periodic(P, cu, cv, n):
    """Explicit periodic-BC blur matrix (n^2 x n^2): the image repeats with
    period n in both directions (x[k + n] = x[k]), so

        A[r + n*i, c + n*j] = sum over images c~ of c and j~ of j of
                              P[cu + r - c~, cv + i - j~].
    """
    N = n * n
    A = np.zeros((N, N), dtype=P.dtype)
    r = np.arange(n)[:, None]
    c = np.arange(n)[None, :]
    cimg = _periodic_images(c, n)
    for i in range(n):
        for j in range(n):
            blk = np.zeros((n, n), dtype=P.dtype)
            for jj in _periodic_images(j, n):
                for cc in cimg:
                    blk += _psf_at(P, cu, cv, r - cc, np.full((1, 1), i - jj))
            A[n * i:n * i + n, n * j:n * j + n] = blk
    return A


def _images(bc, k, n):
    if bc == "zero":
        return [k]
    if bc == "reflexive":
        return _reflect_images(k, n)
    if bc == "periodic":
        return _periodic_images(k, n)
    raise ValueError(bc)


def rearrange(A, m1, n1, m2, n2):
    """R(A) by the literal reordering of eq. "initial rearrange A".

    A is (m1*m2) x (n1*n2) with blocks A_{i,j} of size m2 x n2; row i + m1*j
    of R(A) is vec(A_{i,j})^T with vec column-major.
    """
    R = np.zeros((m1 * n1, m2 * n2), dtype=A.dtype)
    for j in range(n1):
        for i in range(m1):
            blk = A[i * m2:(i + 1) * m2, j * n2:(j + 1) * n2]
            R[i + m1 * j, :] = blk.flatten(order="F")
    return R


def rmat_entries(P, cu, cv, n, rows, cols, bc="zero"):
    """Entries R[rows, cols] of R(A) from the PSF (outer product of indices).

    rows index i + n*j, cols index r + n*c; R[i+n*j, r+n*c] = A[r+n*i, c+n*j],
    which for zero boundary conditions is P[cu+r-c, cv+i-j] and otherwise the
    sum of P[cu+r-c~, cv+i-j~] over the images c~ of c and j~ of j of the
    extended image (bc = "reflexive" or "periodic", as in blur_matrix_*).
    """
    rows = np.asarray(rows)[:, None]
    cols = np.asarray(cols)[None, :]
    i, j = rows % n, rows // n
    r, c = cols % n, cols // n
    if bc == "zero":
        return _psf_at(P, cu, cv, r - c, i - j)
    out = np.zeros(np.broadcast(rows, cols).shape, dtype=P.dtype)
    for jj in _images(bc, j, n):
        for cc in _images(bc, c, n):
            out += _psf_at(P, cu, cv, r - cc, i - jj)
    return out


def rmat_dense_apply(P, cu, cv, n, X, transpose=False, row_chunk=256, bc="zero"):
    """Y = R X (or R^T X) as a dense product over generated row blocks of R.

    The paper treats B = R(A) as an unstructured matrix (section 4.1); this is
    that product, with R's rows produced ``row_chunk`` at a time from the PSF
    (boundary conditions ``bc`` as in rmat_entries) and multiplied with BLAS.
    X may be 1-D or 2-D.
    """
    N = n * n
    X = np.asarray(X)
    vec = X.ndim == 1
    Xm = X[:, None] if vec else X
    dt = np.result_type(P.dtype, Xm.dtype)
    cols = np.arange(N)
    if not transpose:
        Y = np.zeros((N, Xm.shape[1]), dtype=dt)
        for r0 in range(0, N, row_chunk):
            rows = np.arange(r0, min(N, r0 + row_chunk))
            Y[rows] = rmat_entries(P, cu, cv, n, rows, cols, bc).astype(dt) @ Xm
    else:
        Y = np.zeros((N, Xm.shape[1]), dtype=dt)
        for r0 in range(0, N, row_chunk):
            rows = np.arange(r0, min(N, r0 + row_chunk))
            Y += rmat_entries(P, cu, cv, n, rows, cols, bc).astype(dt).T @ Xm[rows]
    return Y[:, 0] if vec else Y


def rmat_window_apply(P, cu, cv, n, X, blocks=None, dtype=np.float64):
    """Y = R X (zero boundary conditions) as the same dense product, with each
    n x n block of R read straight from the PSF instead of gathered entry by
    entry: block (j, c) of R (rows i + n j, columns r + n c) has entries
    R[i + n j, r + n c] = P[cu + r - c, cv + i - j], i.e. it is the n x n window
    of the zero-padded transposed PSF whose top-left corner sits at
    (cv - j, cu - c). Each window is multiplied with BLAS as a strided view (no
    copy) in ``dtype``; every block of R is visited, so the work is the dense
    2 N^2 flops per column.

    blocks: optional range of block rows j (rows n*j .. n*j + n - 1 of Y) to
    compute; the other rows of Y are left zero. X: N x b (or N).
    """
    N = n * n
    X = np.asarray(X)
    vec = X.ndim == 1
    Xm = np.ascontiguousarray((X[:, None] if vec else X).astype(dtype, copy=False))
    pu, pv = P.shape
    Tp = np.zeros((pv + 2 * (n - 1), pu + 2 * (n - 1)), dtype=dtype)
    Tp[n - 1:n - 1 + pv, n - 1:n - 1 + pu] = np.asarray(P, dtype=dtype).T
    Y = np.zeros((N, Xm.shape[1]), dtype=dtype)
    for j in (range(n) if blocks is None else blocks):
        acc = np.zeros((n, Xm.shape[1]), dtype=dtype)
        a0 = cv - j + n - 1
        for c in range(n):
            b0 = cu - c + n - 1
            acc += Tp[a0:a0 + n, b0:b0 + n] @ Xm[n * c:n * c + n]
        Y[n * j:n * j + n] = acc
    return Y[:, 0] if vec else Y


def offset_matrix(P, cu, cv, n):
    """M[d1 + n-1, d2 + n-1] = P[cu + d2, cv + d1] on the (2n-1)^2 offset grid.

    With E[(i,j), d] = [i - j = d] (an n^2 x (2n-1) 0/1 matrix) this gives
    R(A) = E M E^T (block-Toeplitz structure of a shift-invariant blur).
    """
    d = np.arange(-(n - 1), n)
    return _psf_at(P, cu, cv, d[None, :], d[:, None])


def diag_sums(X, n):
    """E^T X: for every offset d in [-(n-1), n-1], sum of X[a + n*b] over a - b = d."""
    Xm = X.reshape(n, n, -1, order="F") if X.ndim == 2 else X.reshape(n, n, 1, order="F")
    out = np.zeros((2 * n - 1, Xm.shape[2]), dtype=X.dtype)
    for d in range(-(n - 1), n):
        a = np.arange(max(0, d), min(n, n + d))
        out[d + n - 1] = Xm[a, a - d, :].sum(axis=0)
    return out


def diag_spread(Z, n):
    """E Z: the vector with entry Z[a - b + n-1] at index a + n*b."""
    a = np.arange(n)[:, None]
    b = np.arange(n)[None, :]
    idx = (a - b + n - 1).flatten(order="F")
    return Z[idx]


def rmat_struct_apply(P, cu, cv, n, X, transpose=False):
    """Y = R X (or R^T X) via R = E M E^T; algebraically identical to the dense
    product (checked against it in the tests) and fast at any n."""
    X = np.asarray(X)
    vec = X.ndim == 1
    Xm = X[:, None] if vec else X
    M = offset_matrix(P, cu, cv, n)
    if transpose:
        M = M.T
    Y = diag_spread(M @ diag_sums(Xm, n), n)
    return Y[:, 0] if vec else Y


def exact_kpsvd(P, cu, cv, n, K=None):
    """Exact leading singular triplets of R(A), hence the optimal K-term
    Kronecker approximation (Theorem "Kronecker Product SVD" + Eckart-Young).

    Since E^T E = W = diag(n - |d|), R = (E W^-1/2)(W^1/2 M W^1/2)(E W^-1/2)^T
    with E W^-1/2 orthonormal, so sigma(R) = sigma(W^1/2 M W^1/2) and the
    singular vectors are E W^-1/2 times those of the weighted (2n-1)^2 matrix.
    Returns (sigma, U, V) with U, V of shape (n^2, K).
    """
    d = np.arange(-(n - 1), n)
    w = np.sqrt(n - np.abs(d)).astype(np.float64)
    M = offset_matrix(P, cu, cv, n).astype(np.float64)
    Uw, s, Vwt = np.linalg.svd(w[:, None] * M * w[None, :])
    if K is None:
        K = len(s)
    U = diag_spread(Uw[:, :K] / w[:, None], n)
    V = diag_spread(Vwt[:K].T / w[:, None], n)
    return s[:K], U, V


def rmat_fro_norm2(P, cu, cv, n):
    """||R(A)||_F^2 = ||A||_F^2 = sum_{d1,d2} (n-|d1|)(n-|d2|) M[d1,d2]^2."""
    d = np.arange(-(n - 1), n)
    w = (n - np.abs(d)).astype(np.float64)
    M = offset_matrix(P, cu, cv, n).astype(np.float64)
    return float((w[:, None] * w[None, :] * M * M).sum())
