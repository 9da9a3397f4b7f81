"""EGKB, RSVD, Rayleigh-Ritz refinement and Kronecker terms (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

``apply_R(X)`` / ``apply_Rt(X)`` are callables giving B X and B^T X for the
matrix B = R(A) (any of the products in ``oracle.operator``). Everything here
runs in float64 unless ``dtype`` asks otherwise.

Readings of passages the paper leaves open (each is also listed in the design
notes):

* nu: the algorithm's index with the text's square root,
  nu_{j+1} = sqrt(zeta_j zeta_{j-1}) (Algorithm 1 vs eq. "stopnu").
* initialisation: zeta_1 = alpha_1 t_1 and nu_2 = +inf (scale-invariant);
  ``literal_init=True`` restores the printed zeta_1 = 1, nu_2 = 100.
* the garbled loop condition: iterate j = 2 .. k_p + 1 with the current k_p;
  the auto-k test fires at most once, only while j > k_min and j - 1 != k_p,
  and sets k = min(j, k_input), k_p = k + p.
* svds(C, k_p) = full thin SVD of the (k_p+1) x k_p bidiagonal C.
* output: U_k = S_{(k_p+1)} U[:, :k], V_k = Q_{k_p} V[:, :k] (all k_p+1 Lanczos
  vectors enter the left factor).
* breakdown (t_j or alpha_j <= ``bd_rel`` * the largest entry of C accepted so
  far; t_1 = ||y|| is not an entry of C and its size is arbitrary, so it is not
  part of the scale; alpha_1 breaks down only when it is 0): the coefficient is
  stored as 0 and the vector is replaced by a Philox normal vector (stream 2j
  for s_j, 2j+1 for q_j), orthogonalized twice (classical Gram-Schmidt) against
  the basis built so far, and normalized.
"""
from __future__ import annotations

import numpy as np

from . import philox


def _norm(x):
    return float(np.sqrt(np.dot(x, x)))


def mgs(v, basis):
    """One pass of modified Gram-Schmidt of v against the columns in ``basis``
    (step "one-sided reorthogonalization" of Algorithm 1)."""
    for b in basis:
        v = v - np.dot(v, b) * b
    return v


def cgs2(v, basis):
    """Classical Gram-Schmidt applied twice (used only for restart vectors)."""
    if len(basis) == 0:
        return v
    Bm = np.stack(basis, axis=1)
    for _ in range(2):
        v = v - Bm @ (Bm.T @ v)
    return v


def egkb(apply_R, apply_Rt, y, k, p, *, reorth="full", auto_k=False, k_min=0,
         tau=0.0, literal_init=False, bd_rel=None, seed=0, dtype=np.float64,
         force_breakdown=None):
    """Enlarged Golub-Kahan bidiagonalization (Algorithm 1, section 2.2).

    reorth: "one_sided" = step 6 only (q_j against Q, the paper's DP run);
            "full" = also s_j against S (the paper's SP runs, section 4.4).
    force_breakdown: optional set of ("s"|"q", j) forcing the breakdown branch
            at exactly those steps (and nowhere else), so the oracle can follow
            a run whose breakdown decisions were taken in another precision.
    Returns a dict with sigma (k), U (M x k), V (N x k), S, Q, C, alpha, t, nu,
    k, kp, breakdowns.
    """
    eps = np.finfo(dtype).eps / 2
    if bd_rel is None:
        bd_rel = 1e2 * eps
    k_in = k
    kp = k + p
    y = np.asarray(y, dtype=dtype)

    forced = []    # (side, j, own norm, scale) at each forced step

    def is_bd(side, j, val, scale):
        if force_breakdown is not None:
            if (side, j) in force_breakdown:
                forced.append((side, j, float(val), float(scale)))
                return True
            return False
        return val <= bd_rel * scale or val == 0.0

    def restart(side, j, basis, size):
        g = philox.normals(size, seed, 2 * j + (0 if side == "s" else 1)).astype(dtype)
        g = cgs2(g, basis)
        return g / _norm(g)

    breakdowns = []
    t = [_norm(y)]
    S = [y / t[0]]
    q = apply_Rt(S[0])
    alpha = [_norm(q)]
    if is_bd("q", 1, alpha[0], 0.0):
        breakdowns.append(("q", 1))
        alpha[0] = 0.0
        Q = [restart("q", 1, [], q.shape[0])]
    else:
        Q = [q / alpha[0]]
    zeta = {1: 1.0 if literal_init else alpha[0] * t[0]}
    nu = {2: 100.0 if literal_init else np.inf}
    scale = alpha[0]
    fired = False
    j = 2
    while j <= kp + 1:
        s = apply_R(Q[-1]) - alpha[-1] * S[-1]
        if reorth == "full":
            s = mgs(s, S)
        tj = _norm(s)
        if is_bd("s", j, tj, scale):
            breakdowns.append(("s", j))
            tj = 0.0
            s = restart("s", j, S, s.shape[0])
        else:
            s = s / tj
        S.append(s)
        t.append(tj)
        scale = max(scale, tj)
        if j <= kp:
            q = apply_Rt(s) - tj * Q[-1]
            q = mgs(q, Q)
            aj = _norm(q)
            if is_bd("q", j, aj, scale):
                breakdowns.append(("q", j))
                aj = 0.0
                q = restart("q", j, Q, q.shape[0])
            else:
                q = q / aj
            Q.append(q)
            alpha.append(aj)
            scale = max(scale, aj)
            zeta[j] = aj * tj
            nu[j + 1] = float(np.sqrt(zeta[j] * zeta[j - 1]))
            if auto_k and not fired and j > k_min and (j - 1) != kp:
                if nu[j + 1] > nu[j] or nu[j] < tau:
                    fired = True
                    k = min(j, k_in)
                    kp = k + p
        j += 1
    # S has kp+1 columns, Q has kp columns (the loop ran to the final kp+1).
    Sm = np.stack(S[:kp + 1], axis=1)
    Qm = np.stack(Q[:kp], axis=1)
    C = np.zeros((kp + 1, kp), dtype=np.float64)
    for i in range(kp):
        C[i, i] = alpha[i]
        C[i + 1, i] = t[i + 1]
    Uc, sc, Vct = np.linalg.svd(C, full_matrices=False)
    U = Sm @ Uc[:, :k]
    V = Qm @ Vct[:k].T
    return dict(sigma=sc[:k].copy(), sigma_all=sc, U=U, V=V, S=Sm, Q=Qm, C=C,
                alpha=np.array(alpha[:kp]), t=np.array(t[:kp + 1]), nu=nu,
                k=k, kp=kp, breakdowns=breakdowns, Uc=Uc, Vc=Vct.T, forced=forced)


def _gs_column(w, basis, passes=2):
    """Classical Gram-Schmidt of w against the columns of ``basis`` (N x m),
    ``passes`` times; returns (w orthogonalized, total coefficients)."""
    h = np.zeros(basis.shape[1])
    for _ in range(passes):
        if basis.shape[1] == 0:
            break
        hp = basis.T @ w
        w = w - basis @ hp
        h += hp
    return w, h


def block_egkb(apply_R, apply_Rt, Y, k, p, *, bd_rel=None, seed=0, dtype=np.float64,
               force_breakdown=None, auto_k=False, k_min=0, tau=0.0, literal_init=False):
    """Block Golub-Kahan bidiagonalization with b = Y.shape[1] start vectors
    (Golub, Luk & Overton 1981): the block analogue of Algorithm 1 with full
    reorthogonalization, enlarged to k_p = k + p columns rounded up to whole
    blocks (nb blocks of b).

        U_1 = qr(Y),             V_1 L_1^T = B^T U_1,
        U_{j+1} R_j = B V_j - U_j L_j,     V_{j+1} L_{j+1}^T = B^T U_{j+1} - V_j R_j^T,

    so that B [V_1 .. V_nb] = [U_1 .. U_nb+1] C with C block lower bidiagonal
    (L_j on the diagonal, R_j below). Each new block is orthonormalized column
    by column with classical Gram-Schmidt applied twice against all previous
    vectors of its basis (which subtracts U_j L_j and V_j R_j^T and
    reorthogonalizes in one step); the coefficients on the block's own earlier
    columns and the norms form R_j (resp. L_{j+1}^T). With b = 1 this is
    Algorithm 1 with full reorthogonalization.

    Breakdown: a norm that is 0 or <= bd_rel times the largest norm accepted so
    far in C stores 0 and replaces the column by a Philox normal vector
    orthogonalized twice against its basis (stream 2(m+1) for column m of U,
    2(m+1)+1 for column m of V: for b = 1 the streams of Algorithm 1's s_{m+1},
    q_{m+1}). The start block's own factor is not part of C (as t_1).
    force_breakdown: optional set of ("u"|"v", m) taking the breakdown branch at
    exactly those columns (and nowhere else), to follow a run whose decisions
    were taken in another precision.

    auto_k: the stopping rule of Algorithm 1 (eq. "stopnu") with one value per
    block: zeta_J (J = 1 .. nb) is the geometric mean over the b columns m of
    block J of alpha_m t_m, where alpha_m = C[m, m] (the diagonal of L_J) and
    t_m is the stored norm of column m of U (the start block's own norms for
    J = 1, the diagonal of R_{J-1} after), i.e. (|det L_J| |det R_{J-1}|)^(1/b).
    nu_{J+1} = sqrt(zeta_J zeta_{J-1}), zeta_1 as computed and nu_2 = +inf
    (literal_init: 1 and 100). The first block J >= 2 with J b > k_min and
    nu_{J+1} > nu_J or nu_J < tau sets k = min(J b, k), k_p = k + p and
    nb = ceil(k_p / b). With b = 1 these are Algorithm 1's alpha, t and rule.
    (Column by column the rule would fire at the first block boundary, where a
    block's first column is always larger than the last of the previous one.)
    Returns dict(sigma, U, V, Ub, Vb, C, kp, k, breakdowns, zeta, nu).
    """
    eps = np.finfo(dtype).eps / 2
    if bd_rel is None:
        bd_rel = 1e2 * eps
    Y = np.asarray(Y, dtype=dtype)
    N, b = Y.shape
    nb = -(-(k + p) // b)
    kp = nb * b
    breakdowns = []
    forced = []    # (side, m, own norm, scale) at each forced column
    scale = [0.0]

    def orth_block(W, basis, side, col0, in_c):
        """Columns of W against `basis` then each other; returns (Q, own R)."""
        Q = np.zeros_like(W)
        Rown = np.zeros((W.shape[1], W.shape[1]))
        for c in range(W.shape[1]):
            full = np.concatenate([basis, Q[:, :c]], axis=1)
            w, h = _gs_column(W[:, c], full)
            nr = _norm(w)
            Rown[:c, c] = h[basis.shape[1]:]
            m = col0 + c
            if force_breakdown is not None:
                broken = (side, m) in force_breakdown
                if broken:
                    forced.append((side, m, float(nr), float(scale[0])))
            else:
                broken = nr == 0.0 or (in_c and nr <= bd_rel * scale[0])
            if broken:
                breakdowns.append((side, m))
                g = philox.normals(W.shape[0], seed,
                                   2 * (m + 1) + (0 if side == "u" else 1)).astype(dtype)
                g, _ = _gs_column(g, full)
                w, nr_store = g / _norm(g), 0.0
            else:
                w, nr_store = w / nr, nr
                if in_c:
                    scale[0] = max(scale[0], nr)
            Rown[c, c] = nr_store
            Q[:, c] = w
        return Q, Rown

    U = np.zeros((N, 0), dtype=dtype)
    V = None                                # sized by the first product with B^T
    U1, R0 = orth_block(Y, U, "u", 0, False)
    U = U1
    tcol = list(np.diag(R0))                # t of every U column, in order
    C = np.zeros((kp + b, kp))
    k_in = k
    zeta, nu = {}, {}
    fired = False
    j = 0
    while j < nb:
        W = apply_Rt(U[:, j * b:(j + 1) * b])
        if V is None:
            V = np.zeros((W.shape[0], 0), dtype=dtype)
        Vj, Lt = orth_block(W, V, "v", j * b, True)
        V = np.concatenate([V, Vj], axis=1)
        C[j * b:(j + 1) * b, j * b:(j + 1) * b] = Lt.T
        # the stopping rule on block J = j + 1
        J = j + 1
        prods = np.array([Lt[c, c] * tcol[j * b + c] for c in range(b)])
        with np.errstate(divide="ignore"):
            zeta[J] = float(np.exp(np.mean(np.log(prods))))
        if J == 1:
            if literal_init:
                zeta[1] = 1.0
            nu[2] = 100.0 if literal_init else np.inf
        else:
            nu[J + 1] = float(np.sqrt(zeta[J] * zeta[J - 1]))
            if auto_k and not fired and J * b > k_min:
                if nu[J + 1] > nu[J] or nu[J] < tau:
                    fired = True
                    k = min(J * b, k_in)
                    kp = k + p
                    nb = -(-kp // b)
        Z = apply_R(Vj)
        Uj, Rj = orth_block(Z, U, "u", (j + 1) * b, True)
        U = np.concatenate([U, Uj], axis=1)
        tcol.extend(np.diag(Rj))
        C[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = Rj
        j += 1
    kp = nb * b
    U, V, C = U[:, :kp + b], V[:, :kp], C[:kp + b, :kp]
    Uc, sc, Vct = np.linalg.svd(C, full_matrices=False)
    return dict(sigma=sc[:k].copy(), sigma_all=sc, U=U @ Uc[:, :k], V=V @ Vct[:k].T, Ub=U,
                Vb=V, C=C, kp=kp, k=k, breakdowns=breakdowns, zeta=zeta, nu=nu, forced=forced)


def orth(X):
    """Orthonormal basis of range(X) (Householder QR, reduced)."""
    Qm, _ = np.linalg.qr(X)
    return Qm


def rsvd(apply_R, apply_Rt, F, k, q=1):
    """Randomized SVD (Algorithm 2, section 2.3) with orthonormalization after
    every application of B or B^T (the paper's practical remark).

    F is the N x k_p Gaussian sketch. Returns dict(sigma, U, V, Y, H).
    """
    Y = orth(apply_R(F))
    for _ in range(q):
        Z = orth(apply_Rt(Y))
        Y = orth(apply_R(Z))
    Ht = apply_Rt(Y)                       # (Q^T B)^T
    Uh, s, Vt = np.linalg.svd(Ht.T, full_matrices=False)
    return dict(sigma=s[:k].copy(), sigma_all=s, U=Y @ Uh[:, :k], V=Vt[:k].T,
                Y=Y, Ht=Ht)


def refine(apply_R, V):
    """One-sided Rayleigh-Ritz refinement of a right factor V (N x k).

    V is re-orthonormalized, W = B V is formed and its thin SVD
    W = U~ S~ Z^T gives the refined triplets (U~, S~, V Z): the best rank-k
    approximation of B restricted to range(V).
    """
    Vo = orth(V)
    W = apply_R(Vo)
    Uw, s, Zt = np.linalg.svd(W, full_matrices=False)
    return dict(sigma=s, U=Uw, V=Vo @ Zt.T)


def sign_fix(U, V):
    """Flip each pair (u_i, v_i) so that the largest-magnitude entry of v_i is
    positive (ties to the lowest index). Returns new arrays."""
    U = U.copy()
    V = V.copy()
    for i in range(V.shape[1]):
        m = int(np.argmax(np.abs(V[:, i])))
        if V[m, i] < 0:
            U[:, i] = -U[:, i]
            V[:, i] = -V[:, i]
    return U, V


def kp_terms(sigma, U, V, n):
    """Kronecker factors (eq. "KP approx"): A_x,i = sigma_i array(u_i, n, n),
    A_y,i = array(v_i, n, n), array column-major. Returns (Ax, Ay) with shape
    (k, n, n)."""
    U, V = sign_fix(U, V)
    k = len(sigma)
    Ax = np.stack([sigma[i] * U[:, i].reshape(n, n, order="F") for i in range(k)])
    Ay = np.stack([V[:, i].reshape(n, n, order="F") for i in range(k)])
    return Ax, Ay


def kp_approx_matrix(Ax, Ay):
    """Explicit A_k = sum_i A_x,i (x) A_y,i (small n only)."""
    return sum(np.kron(Ax[i], Ay[i]) for i in range(Ax.shape[0]))
