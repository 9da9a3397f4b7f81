"""Kronecker apply, CGLS and split Bregman (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Images are n x n arrays X[row, col] (row vertical); x = vec(X) column-major.

Readings of open passages:
* L (eq. "deriv") is square n x n: (L x)_i = (x_i - x_{i+1})/2 for i < n and
  (L x)_n = x_n / 2 (P = N, as the paper's T = N + 2P = 30000 at n = 100
  implies). (L_x (x) I) vec(X) = vec(X L^T) acts along rows (horizontal
  differences); (I (x) L_y) vec(X) = vec(L X) acts along columns (vertical).
* The anisotropic shrink uses the printed threshold 1/gamma with
  gamma = lambda^2/beta (eq. "d thresholding ani"); the isotropic one uses
  (c/s) max(s - 1/gamma~, 0) (eq. "d thresholding iso") with d = 0 where s = 0.
* RC_CGLS = ||mu w|| / ||x^(iota+1)|| (eq. "RC" divides by ||x^(iota)||, which
  is 0 at the first step).
* CGLS starts from x = 0 at every outer iteration (Algorithm 5).
* tau_cgls = 0 or tau_sb = 0 means a fixed iteration count.

With the x-update solved exactly, a fixed point of Algorithms 3/4 has d = L x
and g a subgradient of (beta / lambda^2) TV at L x, so the loop converges to
the minimizer of ||A x - b||^2 + 2 beta TV(x) (anisotropic: the l1 norms of the
two difference images; isotropic: the sum of the pixelwise gradient lengths).
The tests check this against the minimizer computed through the Lagrange dual.
"""
from __future__ import annotations

import numpy as np


def kp_apply(Ax, Ay, X, transpose=False):
    """array(A_k x) = sum_i A_y,i X A_x,i^T (eq. "KPAx"); the transpose is
    array(A_k^T y) = sum_i A_y,i^T Y A_x,i."""
    out = np.zeros_like(X, dtype=np.result_type(Ax.dtype, X.dtype))
    for i in range(Ax.shape[0]):
        if transpose:
            out += Ay[i].T @ X @ Ax[i]
        else:
            out += Ay[i] @ X @ Ax[i].T
    return out


def reg_matrix(n):
    """L = 1/2 * bidiag(1, -1), n x n (eq. "deriv", square reading)."""
    L = 0.5 * np.eye(n)
    L -= 0.5 * np.eye(n, k=1)
    return L


def shrink(c, thr):
    """shrink(w, v) = sign(w) max(|w| - v, 0)."""
    return np.sign(c) * np.maximum(np.abs(c) - thr, 0.0)


def iso_shrink(cx, cy, thr):
    """(c/s) max(s - thr, 0), s = sqrt(cx^2 + cy^2); 0 where s == 0."""
    s = np.sqrt(cx * cx + cy * cy)
    scale = np.zeros_like(s)
    nz = s > 0
    scale[nz] = np.maximum(s[nz] - thr, 0.0) / s[nz]
    return cx * scale, cy * scale


class Augmented:
    """A-hat = [A; lam (L_x (x) I); lam (I (x) L_y)] acting on images (eq. "agu A")."""

    def __init__(self, apply_A, apply_At, n, lam):
        self.A, self.At, self.n, self.lam = apply_A, apply_At, n, lam
        self.L = reg_matrix(n)

    def fwd(self, W):
        return (self.A(W), self.lam * (W @ self.L.T), self.lam * (self.L @ W))

    def adj(self, r):
        r1, r2, r3 = r
        return self.At(r1) + self.lam * (r2 @ self.L) + self.lam * (self.L.T @ r3)


def _nrm2(parts):
    return float(sum(np.sum(p * p) for p in parts))


def cgls(op: Augmented, bhat, I_max, tau=0.0):
    """CGLS (Algorithm 5) for min ||A-hat x - b-hat||; x^(0) = 0.

    Returns (x, iterations, history of ||r||).
    """
    n = op.n
    x = np.zeros((n, n))
    r = tuple(np.array(p, dtype=np.float64) for p in bhat)
    f = op.adj(r)
    w = f.copy()
    tau_i = float(np.sum(f * f))
    hist = [np.sqrt(_nrm2(r))]
    it = 0
    while it < I_max:
        if tau_i == 0.0:
            break
        z = op.fwd(w)
        mu = tau_i / _nrm2(z)
        step = mu * w
        x = x + step
        r = tuple(ri - mu * zi for ri, zi in zip(r, z))
        f = op.adj(r)
        tau_new = float(np.sum(f * f))
        delta = tau_new / tau_i
        w = f + delta * w
        tau_i = tau_new
        it += 1
        hist.append(np.sqrt(_nrm2(r)))
        if tau > 0.0:
            rc = np.linalg.norm(step) / np.linalg.norm(x)
            if rc < tau:
                break
    return x, it, hist


def split_bregman(kind, apply_A, apply_At, b, lam, beta, L_max, tau_sb=0.0,
                  I_max=100, tau_cgls=0.0):
    """Split Bregman TV deblurring: Algorithm 3 (kind="aniso") or Algorithm 4
    (kind="iso"), with lambda_x = lambda_y = lam and beta_x = beta_y = beta.

    Returns dict(x, l_end, iota_total, rc_sb, rc_hist).
    """
    n = b.shape[0]
    op = Augmented(apply_A, apply_At, n, lam)
    L = op.L
    x = b.copy()                         # x^(0) = b
    dx = np.zeros_like(b)
    dy = np.zeros_like(b)
    gx = np.zeros_like(b)
    gy = np.zeros_like(b)
    gamma = lam * lam / beta
    iota_total = 0
    rc_hist = []
    l_end = 0
    for ell in range(L_max):
        bhat = (b, lam * (dx - gx), lam * (dy - gy))
        x_new, it, _ = cgls(op, bhat, I_max, tau_cgls)
        iota_total += it
        cx = x_new @ L.T + gx
        cy = L @ x_new + gy
        if kind == "aniso":
            dx = shrink(cx, 1.0 / gamma)
            dy = shrink(cy, 1.0 / gamma)
        elif kind == "iso":
            dx, dy = iso_shrink(cx, cy, 1.0 / gamma)
        else:
            raise ValueError(kind)
        gx = cx - dx
        gy = cy - dy
        rc = np.linalg.norm(x_new - x) / np.linalg.norm(x)
        rc_hist.append(rc)
        x = x_new
        l_end = ell + 1
        if tau_sb > 0.0 and rc < tau_sb:
            break
    return dict(x=x, l_end=l_end, iota_total=iota_total,
                rc_sb=rc_hist[-1] if rc_hist else 0.0, rc_hist=rc_hist)
