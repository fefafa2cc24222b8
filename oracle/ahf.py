"""Oracle: absorbed heat fluxes from REFs and direct heat fluxes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gebhart's formula (Sec. 4.2.3, eq. 4.6): the heat absorbed by face i is the
part of the direct flux on i that i absorbs, plus, for every face j, the
part of the direct flux on j that j reflects diffusely and that ends up
absorbed by i (the REF B_ji accounts for every chain of reflections):

    Q^(a)_i = A_i eps_i Q^(d)_i + sum_{j=1..N} B_ji A_j rho_j Q^(d)_j

Readings: Q^(d) is the direct heat flux per unit area on each face (so
A_i Q^(d)_i is the incident power and Q^(a)_i a power); several load cases
are the columns of an N x m array.  Only the N x N block of B enters (space
absorbs nothing and does not reflect).
"""
from __future__ import annotations

import numpy as np


def absorbed_flux(b: np.ndarray, eps: np.ndarray, rho: np.ndarray, area: np.ndarray, qd: np.ndarray) -> np.ndarray:
    """Q^(a) (N x m, or N for a 1-D qd) of eq. 4.6 (float64)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    qd = np.asarray(qd, dtype=np.float64)
    vec = qd.ndim == 1
    q = qd[:, None] if vec else qd
    eps = np.asarray(eps, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    area = np.asarray(area, dtype=np.float64)
    direct = (area * eps)[:, None] * q
    reflected = b[:, :n].T @ ((area * rho)[:, None] * q)
    qa = direct + reflected
    return qa[:, 0] if vec else qa
