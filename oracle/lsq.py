"""Oracle: least-squares optimum closure + reciprocity enforcer for open systems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.5.5 (eq. 3.41-3.52) with the non-negativity rectification (NNR,
App. A.1) and small positive value avoidance (SPVA, App. A.2).  Unknowns are
the view factors F_ij in row-major order, space column included (N (N+1)
values).  The restrictions A x = b are the N closure rows R_C (row i sums to
one, eq. 3.42) and the N (N-1) / 2 reciprocity rows R_R (Omega_i F_ij -
Omega_j F_ji = 0 for i < j, the pattern of eq. 3.43 with the weights of
eta_ij = Omega_i F_ij).
The estimate is the row-space solution plus the null-space component closest
to the MCRT coefficients (eq. 3.47-3.52):

    x_hat = A^T (A A^T)^{-1} b + N_b (N_b^T N_b)^{-1} N_b^T (x - x_r).

Removing a coefficient (NNR: it came out negative; SPVA: it was zero in the
MCRT input) fixes it at zero and deletes its column from A; rows of A left
all zero are deleted with their entries of b; NNR repeats until no
coefficient is negative.  SPVA is applied once, before the NNR loop.

Readings: the text states the problem on eta = Omega F; the printed worked
example (eq. 6.7-6.8) is reproduced when the deviation is measured on F
itself (the Euclidean projection on eta gives a different answer there), so
the restrictions are written on F as above (the same affine set).  Eq. 3.41
gives A N(N-1) columns; the unknowns and eq. 3.42 need N (N+1).  NNR
removes the negative coefficients' columns, as SPVA does (a reciprocity row
with one partner removed stays and holds the other at zero, which keeps
reciprocity; that partner is then exactly zero, which is set explicitly so
that a rounding-level negative cannot trigger NNR).  Each round projects the
MCRT input restricted to the coefficients still active.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import null_space


def restriction_matrix(n: int, omega: np.ndarray):
    """A (eq. 3.41-3.43, written on F) and b for N surfaces."""
    omega = np.asarray(omega, dtype=np.float64)
    nc = n * (n + 1)
    rc = np.zeros((n, nc))
    for i in range(n):
        rc[i, i * (n + 1):(i + 1) * (n + 1)] = 1.0
    rr = np.zeros((n * (n - 1) // 2, nc))
    row = 0
    for i in range(n):
        for j in range(i + 1, n):
            rr[row, j + (n + 1) * i] = omega[i]
            rr[row, i + (n + 1) * j] = -omega[j]
            row += 1
    a = np.vstack([rc, rr])
    b = np.concatenate([np.ones(n), np.zeros(rr.shape[0])])
    return a, b


def _project(a: np.ndarray, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Eq. 3.47-3.52 on the reduced system."""
    keep = np.abs(a).sum(axis=1) > 0
    a, b = a[keep], b[keep]
    xr = a.T @ np.linalg.solve(a @ a.T, b)
    nb = null_space(a)
    if nb.shape[1] == 0:
        return xr
    w = np.linalg.solve(nb.T @ nb, nb.T @ (x - xr))
    return xr + nb @ w


def enforce_lsq(f: np.ndarray, omega: np.ndarray, nnr: bool = True, spva: bool = False, max_rounds: int = 100):
    """Returns (F_hat, info); info['rounds'] = least-squares solves run,
    info['active'] = the coefficients left free (n x (n+1) bool)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    omega = np.asarray(omega, dtype=np.float64)
    x = f.reshape(-1).copy()
    a, b = restriction_matrix(n, omega)
    active = np.ones(x.size, dtype=bool)
    if spva:
        active &= x != 0.0
    xh = np.zeros_like(x)
    rounds = 0
    while True:
        rounds += 1
        xh = np.zeros_like(x)
        xh[active] = _project(a[:, active], b, x[active])
        # an entry whose reciprocal partner is held at zero is zero by its
        # reciprocity row (Omega_i F_ik = 0): set it exactly, so that rounding
        # of the projection cannot decide the NNR test
        am = active.reshape(n, n + 1)
        lone = am[:, :n] & ~am[:, :n].T
        np.fill_diagonal(lone, False)
        xh.reshape(n, n + 1)[:, :n][lone] = 0.0
        neg = active & (xh < 0.0)
        if not nnr or not neg.any() or rounds >= max_rounds:
            break
        active &= ~neg
    xh[~active] = 0.0
    return xh.reshape(n, n + 1), {"rounds": rounds, "removed": int((~active).sum()),
                                  "active": active.reshape(n, n + 1).copy()}
