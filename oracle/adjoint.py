"""Oracle: gradients of an objective of the REF matrix w.r.t. eps and rho.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With B = K^{-1} E, K = I - F_sq diag(rho), E = [F_sq diag(eps) | F_inf]
(App. B.2, eq. B.8-B.11) and G = dJ/dB (N x (N+1)), the chain rule gives
dJ = <G, K^{-1}(dE - dK B)> = <Lambda, dE> - <Lambda, dK B> with
Lambda = K^{-T} G.  Since dE_ik = F_ik d eps_k and dK_ik = -F_ik d rho_k:

    dJ/d eps_k = sum_i Lambda_ik F_ik
    dJ/d rho_k = sum_i sum_j F_ik Lambda_ij B_kj  = sum_j B_kj (F_sq^T Lambda)_kj

(only the dependence through B; an objective that also contains eps or rho
explicitly adds its own partial derivatives).  The oracle evaluates these
plain definitions: a LAPACK transposed solve and dense products.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gebhart import form_k_e


def gebhart_ref_adjoint(f: np.ndarray, eps: np.ndarray, rho: np.ndarray, b: np.ndarray, g: np.ndarray):
    """Returns (grad_eps, grad_rho, Lambda) for G = dJ/dB."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    k, _ = form_k_e(f, eps, rho)
    lam = sla.lu_solve(sla.lu_factor(k), np.asarray(g, dtype=np.float64), trans=1)
    fs = f[:, :n]
    grad_eps = (lam[:, :n] * fs).sum(axis=0)
    ftl = fs.T @ lam
    grad_rho = (np.asarray(b, dtype=np.float64) * ftl).sum(axis=1)
    return grad_eps, grad_rho, lam
