"""Quality metrics (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np

from .operator import rmat_fro_norm2, rmat_struct_apply


def rel_error(x, x_true):
    """RE(x) = ||x - x_true|| / ||x_true|| (eq. "RE")."""
    return float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))


def isnr(x, x_true, b):
    """ISNR(x) = 20 log10(||b - x_true|| / ||x - x_true||) (eq. "ISNR")."""
    return float(20.0 * np.log10(np.linalg.norm(b - x_true) / np.linalg.norm(x - x_true)))


def snr(b_true, b):
    """SNR = 10 log10(||b_true||^2 / ||b_true - b||^2) (eq. "SNR")."""
    return float(10.0 * np.log10(np.sum(b_true ** 2) / np.sum((b_true - b) ** 2)))


def kp_rel_error(P, cu, cv, n, sigma, U, V):
    """||R - U diag(sigma) V^T||_F / ||R||_F, equal to ||A - A_k||_F / ||A||_F
    since R(.) only permutes entries. Expanded in float64 as
    ||R||^2 - 2 sum_i s_i u_i^T R v_i + sum_{i,j} s_i s_j (u_i^T u_j)(v_i^T v_j)."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    r2 = rmat_fro_norm2(P, cu, cv, n)
    RV = rmat_struct_apply(P, cu, cv, n, V)
    cross = float(np.sum(s * np.einsum("ij,ij->j", U, RV)))
    G = (U.T @ U) * (V.T @ V)
    quad = float(s @ G @ s)
    val = max(r2 - 2.0 * cross + quad, 0.0)
    return float(np.sqrt(val / r2))
