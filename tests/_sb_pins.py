"""Independent checks of the split Bregman loop (Algorithms 3 and 4).

At a fixed point of Algorithm 3/4 with the x-update solved exactly, the
g-update forces d = L x, the shrink (threshold 1/gamma = beta/lambda^2) makes
g a subgradient of (beta/lambda^2) * TV at L x, and the normal equations of
eq. "x in 2d" then read A^T (A x - b) + beta L^T s = 0 with s in the
subdifferential of the TV term. So the loop converges to the minimizer of

    F(x) = ||A x - b||^2 + 2 beta TV(x),
    TV_aniso(x) = ||(L_x (x) I) x||_1 + ||(I (x) L_y) x||_1,
    TV_iso(x)   = sum_i sqrt(((L_x (x) I) x)_i^2 + ((I (x) L_y) x)_i^2),

(the factor 2 is what the printed threshold 1/gamma implies; the exact
minimizer of the printed d-subproblem would threshold at 1/(2 gamma)).

The minimizer is computed here by a route that shares nothing with the loop:
for square invertible A the Lagrange dual of F is

    max_z  ||b||^2 - ||b - beta K z||^2,   K = A^-T D^T,  D = [L_x (x) I; I (x) L_y],

over |z_i| <= 1 (aniso: a box, solved exactly by bounded-variable least
squares) or ||(z_x, z_y)_i|| <= 1 (iso: disks, solved by SLSQP and then
polished by Newton's method on the primal), and x(z) = A^-1 (b - beta K z).
The duality gap F(x) - G(z) >= sigma_min(A)^2 ||x - x*||^2 (F is
sigma_min^2-strongly convex) certifies the reference.
"""
import numpy as np
import scipy.optimize as so


def problem(n=5, seed=7):
    """A small, well-conditioned, non-symmetric blur (cond(A) ~ 2) and a
    noisy blurred two-rectangle image; returns (A, b) with b an n x n image."""
    from oracle import operator as op
    rng = np.random.default_rng(seed)
    P = 0.15 * rng.random((3, 4))
    P[1, 1] += 1.0
    A = op.blur_matrix(P, 1, 1, n)
    X = np.zeros((n, n))
    X[1:3, 0:2] = 1.0
    X[n - 2:, n - 3:] = 0.6
    b = (A @ X.flatten(order="F")).reshape(n, n, order="F") + 0.05 * rng.standard_normal((n, n))
    return A, b


def diff_ops(n):
    """(L_x (x) I, I (x) L_y) as explicit matrices, L = 1/2 bidiag(1, -1)
    written out entry by entry from eq. "deriv" (square reading)."""
    L = np.zeros((n, n))
    for i in range(n):
        L[i, i] = 0.5
        if i + 1 < n:
            L[i, i + 1] = -0.5
    return np.kron(L, np.eye(n)), np.kron(np.eye(n), L)


def objective(kind, A, b, beta, x):
    """F(x) for an image x (n x n)."""
    n = b.shape[0]
    Dx, Dy = diff_ops(n)
    v = x.flatten(order="F")
    r = A @ v - b.flatten(order="F")
    gx, gy = Dx @ v, Dy @ v
    tv = np.sum(np.abs(gx)) + np.sum(np.abs(gy)) if kind == "aniso" else \
        np.sum(np.sqrt(gx * gx + gy * gy))
    return float(r @ r + 2.0 * beta * tv)


def _polish_iso(A, b, beta, v, tol=1e-7):
    """Newton's method on F restricted to {x : (D x)_i = 0 for i in I0}, I0 the
    pixels where the approximate minimizer v has (numerically) zero gradient;
    elsewhere the TV term is smooth. Returns (x, I0)."""
    n = b.shape[0]
    N = n * n
    Dx, Dy = diff_ops(n)
    bv = b.flatten(order="F")
    s = np.sqrt((Dx @ v) ** 2 + (Dy @ v) ** 2)
    I0 = s <= tol * s.max()
    act = ~I0
    Z = np.eye(N)
    if I0.any():
        _, sv, Vt = np.linalg.svd(np.vstack([Dx[I0], Dy[I0]]))
        Z = Vt[int(np.sum(sv > 1e-12 * sv[0])):].T          # null space basis
    Da, Db = Dx[act], Dy[act]
    y = Z.T @ v
    for _ in range(50):
        x = Z @ y
        u, w = Da @ x, Db @ x
        nr = np.sqrt(u * u + w * w)
        g = 2 * A.T @ (A @ x - bv) + 2 * beta * (Da.T @ (u / nr) + Db.T @ (w / nr))
        H = 2 * A.T @ A
        for i in range(len(nr)):
            d = np.vstack([Da[i], Db[i]])
            uv = np.array([u[i], w[i]])
            H += 2 * beta * d.T @ ((np.eye(2) - np.outer(uv, uv) / nr[i] ** 2) / nr[i]) @ d
        step = np.linalg.solve(Z.T @ H @ Z, Z.T @ g)
        y = y - step
        if np.linalg.norm(step) <= 1e-15 * np.linalg.norm(y):
            break
    return Z @ y, I0


def tv_minimizer(kind, A, b, beta):
    """Minimizer of F via its dual. Returns (x, bound) where bound is the
    certified upper bound on ||x - x*|| from the duality gap (its absolute
    value, so a gap at the rounding level still bounds the error)."""
    n = b.shape[0]
    N = n * n
    Dx, Dy = diff_ops(n)
    K = np.linalg.solve(A.T, np.hstack([Dx.T, Dy.T]))
    bv = b.flatten(order="F")
    M = beta * K
    if kind == "aniso":
        z = so.lsq_linear(M, bv, bounds=(-1.0, 1.0), method="bvls", tol=1e-15).x
        z = np.clip(z, -1.0, 1.0)
        x = np.linalg.solve(A, bv - M @ z)
    else:
        cons = {"type": "ineq", "fun": lambda z: 1.0 - z[:N] ** 2 - z[N:] ** 2,
                "jac": lambda z: np.hstack([np.diag(-2 * z[:N]), np.diag(-2 * z[N:])])}
        z = so.minimize(lambda z: float(np.sum((bv - M @ z) ** 2)), np.zeros(2 * N),
                        jac=lambda z: -2.0 * M.T @ (bv - M @ z), constraints=[cons],
                        method="SLSQP", options={"ftol": 1e-16, "maxiter": 2000}).x
        x, I0 = _polish_iso(A, b, beta, np.linalg.solve(A, bv - M @ z))
        # dual point from the polished x: unit gradients where they are
        # nonzero, and on I0 the SLSQP multipliers moved onto the affine set
        # of the stationarity equation A^T (A x - b) + beta D^T z = 0
        act = ~I0
        u, w = Dx @ x, Dy @ x
        nr = np.sqrt(u * u + w * w)
        zx, zy = z[:N].copy(), z[N:].copy()
        zx[act], zy[act] = u[act] / nr[act], w[act] / nr[act]
        if I0.any():
            rhs = -(A.T @ (A @ x - bv)) / beta - Dx[act].T @ zx[act] - Dy[act].T @ zy[act]
            DI = np.hstack([Dx[I0].T, Dy[I0].T])
            zI = np.concatenate([zx[I0], zy[I0]])
            zI = zI + np.linalg.lstsq(DI, rhs - DI @ zI, rcond=None)[0]
            m = int(I0.sum())
            zx[I0], zy[I0] = zI[:m], zI[m:]
        sc = np.maximum(1.0, np.sqrt(zx * zx + zy * zy))      # feasible
        z = np.concatenate([zx / sc, zy / sc])
    x = x.reshape(n, n, order="F")
    dual = float(bv @ bv - np.sum((bv - M @ z) ** 2))
    gap = objective(kind, A, b, beta, x) - dual
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    return x, np.sqrt(abs(gap)) / smin


def run_loop(sbmod, kind, A, b, lam, beta, L_max=200):
    """The oracle's split Bregman with the explicit A and CGLS run well past
    convergence (I_max = 3 N)."""
    n = b.shape[0]
    fA = lambda X: (A @ X.flatten(order="F")).reshape(n, n, order="F")
    fAt = lambda X: (A.T @ X.flatten(order="F")).reshape(n, n, order="F")
    with np.errstate(all="ignore"):
        out = sbmod.split_bregman(kind, fA, fAt, b, lam, beta, L_max=L_max, I_max=3 * n * n)
    return out["x"]


LAM, BETA = 0.7, 0.05


def loop_error(sbmod, kind, n=5):
    """Relative distance of the loop's result to the certified minimizer."""
    A, b = problem(n)
    x_ref, bound = tv_minimizer(kind, A, b, BETA)
    assert bound <= 1e-6 * np.linalg.norm(x_ref), bound
    x = run_loop(sbmod, kind, A, b, LAM, BETA)
    return float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))
