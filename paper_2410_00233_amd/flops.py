"""Algorithmic flop counts of the method (section 4, "Computational costs").

These are the paper's dense cost models, used to turn measured times into
TFLOP/s. They count the work the method must do on an unstructured B = R(A)
(the paper's assumption), not what a structure-exploiting algorithm would do.
Sizes: m1 = m2 = n1 = n2 = n, M_bar = N_bar = N = n^2.
"""
from __future__ import annotations


def rmat_product(n: int, ncols: int) -> float:
    """Y = R X or R^T X with X of ncols columns: 2 M_bar N_bar per column."""
    N = n * n
    return 2.0 * N * N * ncols


def egkb(n: int, k: int, p: int, full: bool = False) -> float:
    """EGKB (eq. "EGKB cost1"): 4 M N k_p dominant term; with full=True the
    lower-order terms 2 M k^2 + 2 N (k^2 + k_p^2) + 12 k_p^3 are added."""
    N = n * n
    kp = k + p
    f = 4.0 * N * N * kp
    if full:
        f += 2.0 * N * k * k + 2.0 * N * (k * k + kp * kp) + 12.0 * kp ** 3
    return f


def rsvd(n: int, k: int, p: int, q: int = 1) -> float:
    """RSVD with q power iterations: (2q + 2) products with B or B^T on k_p
    columns, i.e. (4q + 4) M N k_p; q = 1 gives the paper's 8 M N k_p
    (eq. "RSVD cost")."""
    N = n * n
    return (4.0 * q + 4.0) * N * N * (k + p)


def kp_apply(n: int, k: int) -> float:
    """One apply of the k-term Kronecker sum (eq. "KPAx"): 2 (m2 N + M n1) k."""
    N = n * n
    return 2.0 * (n * N + N * n) * k


def cgls_iteration_kp(n: int, k: int) -> float:
    """One CGLS iteration with A_k: an apply and a transposed apply."""
    return 2.0 * kp_apply(n, k)


def cgls_iteration_direct(n: int, P: int | None = None) -> float:
    """One CGLS iteration with A itself (Table 1, row (i)): 4 T N, T = N + 2P."""
    N = n * n
    P = N if P is None else P
    return 4.0 * (N + 2 * P) * N


def sb_speedup(n: int, k: int, P: int | None = None) -> float:
    """Ratio of Table 1's CGLS column, direct A over A_k (eq. "ratio of cost")."""
    return cgls_iteration_direct(n, P) / cgls_iteration_kp(n, k)


def alg_speedup(n: int, kp: int, iota_total: int, rho: int = 1, P: int | None = None) -> float:
    """Table 1, column 4 (direct CGLS) over column 2 (TSVD of B), eq.
    "ratio of alg cost": 4 (N + 2P) N iota / (4 rho N^2 k_p)."""
    N = n * n
    P = N if P is None else P
    return 4.0 * (N + 2 * P) * N * iota_total / (4.0 * rho * N * N * kp)
