"""Oracle: iterative closure and reciprocity enforcer for open systems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thesis Sec. 3.5.5, "Iterative closure and reciprocity enforcer": each iteration
enforces reciprocity on the square N x N part with the fractional-variance
method (Sec. 3.5.3, eq. 3.18-3.25), keeps the environment column of the
previous iterate, then enforces closure on the full N x (N+1) matrix with
least-squares smoothing for open systems (Sec. 3.5.4, eq. 3.36-3.40) using the
weights omega_ij = eta_ij recommended in Sec. 3.5.4.

Readings taken where the text is silent or garbled:

* The worked example (Sec. 6.2, eq. 6.4 -> 6.6 and 6.9) is reproduced only by
  the equal-weight estimator kappa = 1/2; eq. 3.25 with any equal or
  area-proportional ray counts does not give the printed digits.  Both rules are
  provided: ``kappa="half"`` and ``kappa="fracvar"`` (eq. 3.25).
* The variances of eq. 3.23 are evaluated on the current iterate.  z cancels
  in eq. 3.25.  A zero exchange coefficient has infinite variance (kappa puts
  all weight on the other one); when both are zero, or both variances vanish,
  kappa = 1/2.
* Eq. 3.40's numerator is read with the *prior* coefficients eta (the printed
  hat makes it identically zero by the constraint).  With omega = eta the step
  is an exact row normalisation over all N+1 columns.
* The paper does not state its stopping rule.  Here an iteration ends the loop
  when the closure defect the reciprocity step introduced, max_i |s_i - 1|
  with s_i the row sums after that step, is <= ``tol``; tol = 1e-7 gives the
  paper's 13 iterations on its example.  ``tol = 0`` runs exactly ``max_iter``
  iterations.
"""
from __future__ import annotations

import numpy as np


def kappa_fracvar(f: np.ndarray, area: np.ndarray, n_rays: np.ndarray) -> np.ndarray:
    """Eq. 3.25: kappa_ij = s2_ji / (s2_ij + s2_ji), s2 from eq. 3.23 (z dropped).

    s2_ij = Omega_i^2 (1 - F_ij) / (N_i F_ij) with Omega_i = A_i.
    """
    n = f.shape[0]
    fs = f[:, :n]
    with np.errstate(divide="ignore", invalid="ignore"):
        s2 = (area[:, None] ** 2) * (1.0 - fs) / (n_rays[:, None] * fs)
    s2 = np.where(fs > 0.0, s2, np.inf)
    s2t = s2.T
    with np.errstate(divide="ignore", invalid="ignore"):
        kap = s2t / (s2 + s2t)
    both_inf = np.isinf(s2) & np.isinf(s2t)
    kap = np.where(np.isinf(s2) & ~both_inf, 0.0, kap)
    kap = np.where(np.isinf(s2t) & ~both_inf, 1.0, kap)
    kap = np.where(both_inf | ((s2 == 0.0) & (s2t == 0.0)), 0.5, kap)
    return kap


def reciprocity_step(f: np.ndarray, area: np.ndarray, n_rays=None, kappa: str = "fracvar") -> np.ndarray:
    """One reciprocity half-step on the square block (eq. 3.18-3.20).

    eta_ij = Omega_i F_ij (eq. 3.18); for each pair i < j the single estimator
    eta^_ij = kappa eta_ij + (1 - kappa) eta_ji (eq. 3.20) is used for both
    directions, so eq. 3.19 holds by construction.  The diagonal and the
    environment column are left as they are.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    eta = area[:, None] * f[:, :n]                                  # eq. 3.18
    if kappa == "half":
        kap = np.full((n, n), 0.5)
    elif kappa == "fracvar":
        kap = kappa_fracvar(f, area, np.asarray(n_rays, dtype=np.float64))
    else:
        raise ValueError(kappa)
    eta_hat_upper = kap * eta + (1.0 - kap) * eta.T                  # eq. 3.20
    iu = np.triu_indices(n, 1)
    eta_hat = np.zeros((n, n))
    eta_hat[iu] = eta_hat_upper[iu]
    eta_hat = eta_hat + eta_hat.T
    out = f.copy()
    off = ~np.eye(n, dtype=bool)
    out[:, :n][off] = (eta_hat / area[:, None])[off]
    return out


def closure_step(f: np.ndarray, area=None) -> np.ndarray:
    """Least-squares smoothing for open systems (eq. 3.36-3.40), omega = eta.

    lambda_i = (Omega_i - sum_j eta_ij) / sum_j omega_ij over all N+1 columns,
    eta^_ij = eta_ij + omega_ij lambda_i (eq. 3.39), F^_ij = eta^_ij / Omega_i.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    omega_i = np.ones(n) if area is None else np.asarray(area, dtype=np.float64)
    eta = omega_i[:, None] * f
    omega = eta
    denom = omega.sum(axis=1)
    if np.any(denom <= 0.0):
        raise ValueError("a row of the view-factor matrix sums to zero")
    lam = (omega_i - eta.sum(axis=1)) / denom                        # eq. 3.40
    eta_hat = eta + omega * lam[:, None]                             # eq. 3.39
    return eta_hat / omega_i[:, None]


def enforce_vf(f: np.ndarray, area: np.ndarray, n_rays=None, kappa: str = "fracvar",
               tol: float = 0.0, max_iter: int = 100):
    """Iterative enforcer (Sec. 3.5.5).  Returns (F, info).

    info: ``iters`` run, ``closure_defect`` = max_i |s_i - 1| of the last
    reciprocity step (s_i = row sums after it), ``recip_err`` = relative
    reciprocity error max_ij |eta_ij - eta_ji| / max eta of the matrix that
    entered the last iteration, and ``converged`` (tol > 0 and met).
    """
    f = np.array(f, dtype=np.float64, copy=True)
    n = f.shape[0]
    if f.shape != (n, n + 1):
        raise ValueError("expected an N x (N+1) open-system matrix")
    area = np.asarray(area, dtype=np.float64)
    info = {"iters": 0, "closure_defect": float("nan"), "recip_err": float("nan"), "converged": False}
    for k in range(1, max_iter + 1):
        eta = area[:, None] * f[:, :n]
        emax = np.abs(eta).max()
        info["recip_err"] = float(np.abs(eta - eta.T).max() / emax) if emax > 0 else 0.0
        g = reciprocity_step(f, area, n_rays, kappa)
        s = g.sum(axis=1)
        info["closure_defect"] = float(np.abs(s - 1.0).max())
        f = closure_step(g, area)
        info["iters"] = k
        if tol > 0.0 and info["closure_defect"] <= tol:
            info["converged"] = True
            break
    return f, info


def mae(f: np.ndarray, f_exact: np.ndarray) -> float:
    """Mean absolute error over all N(N+1) entries (Table 6.1's metric)."""
    return float(np.abs(np.asarray(f) - np.asarray(f_exact)).mean())
