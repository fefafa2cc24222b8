"""Oracle: open-system Gebhart matrix method.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gebhart's recursion B_ij = eps_j F_ij + sum_k F_ik rho_k B_kj (Sec. 4.2.3,
eq. 4.5) in matrix form K B = E (App. B.1, eq. B.1-B.5), extended to open
systems with the space column B_i,inf = F_i,inf + sum_k F_ik rho_k B_k,inf
(App. B.2, eq. B.6-B.11):

    K = I - F_sq diag(rho)            (N x N, eq. B.9)
    E = [F_sq diag(eps) | F_inf]      (N x (N+1), eq. B.8)
    B = K^{-1} E                      (eq. B.11)

Readings: eps and rho are independent per-face inputs; the space column has no
emissivity factor and space does not reflect (eq. B.6); the last row of K as
printed (-rho_2 F_2N) is read as -rho_2 F_N2, the pattern of every other
entry.  This oracle solves with LAPACK's partially pivoted LU (scipy
``lu_factor``/``lu_solve``), the plain definition of the solve.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def form_k_e(f: np.ndarray, eps: np.ndarray, rho: np.ndarray):
    """K and E of eq. B.8-B.9 (float64)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    fs = f[:, :n]
    k = np.eye(n) - fs * np.asarray(rho, dtype=np.float64)[None, :]
    e = np.empty((n, n + 1))
    e[:, :n] = fs * np.asarray(eps, dtype=np.float64)[None, :]
    e[:, n] = f[:, n]
    return k, e


def gebhart_ref(f: np.ndarray, eps: np.ndarray, rho: np.ndarray, return_factors: bool = False):
    """REF matrix B (N x (N+1)) of eq. B.11 by a pivoted LU solve."""
    k, e = form_k_e(f, eps, rho)
    lu = sla.lu_factor(k, check_finite=True)
    b = sla.lu_solve(lu, e)
    if return_factors:
        return b, lu
    return b


def ref_closure_residual(b: np.ndarray) -> float:
    """max_i |sum_j B_ij + B_i,inf - 1| (eq. 4.3 with space included)."""
    return float(np.abs(np.asarray(b).sum(axis=1) - 1.0).max())


def ref_reciprocity_residual(b: np.ndarray, eps: np.ndarray, area: np.ndarray) -> float:
    """max_ij |eps_i A_i B_ij - eps_j A_j B_ji| (eq. 4.4) on the square block."""
    n = b.shape[0]
    g = (np.asarray(eps) * np.asarray(area))[:, None] * np.asarray(b)[:, :n]
    return float(np.abs(g - g.T).max())
