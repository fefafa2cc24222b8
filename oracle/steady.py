"""Oracle: radiation-only steady-state node temperatures.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The discrete node heat equation (Sec. 3.4.4, eq. 3.14) at steady state
(dT/dt = 0) and without conductive couplings: for every node i whose
temperature is not prescribed, the net power radiated from i to all nodes j
and to deep space equals the power put into i,

    sum_{j=1..N} GR_ij (T_i^4 - T_j^4) + GR_i,space (T_i^4 - T_space^4) = Q_i,

with q_ij = GR_ij (T_i^4 - T_j^4) the power from i to j (eq. 3.12) and, by
the Gebhart method, GR_ij = sigma eps_i A_i B_ij from the REFs (eq. 4.2;
Sec. 4.2.3: REFs replace view factors and absorbed fluxes replace direct
fluxes in eq. 3.14).  Q_i is everything the node receives (absorbed
environmental fluxes, dissipation, heaters minus coolers).

Readings: the printed eq. 3.14 writes the exchange sums with the same sign as
the heat inputs; the balance above takes the physical sign of eq. 3.12 (power
leaving i).  Nodes may hold a prescribed temperature (a boundary node, as the
bottom plate of Sec. 6.3); their balance is not imposed.  The balance is
linear in x_i = T_i^4, so the plain definition is one linear solve in x (the
Newton iteration on T^4 converges in one step); T_i = x_i^(1/4).
"""
from __future__ import annotations

import numpy as np

SIGMA = 5.670374419e-8


def steady_temperature(y: np.ndarray, weight: np.ndarray, q: np.ndarray, t_fixed=None, t_space: float = 3.0,
                       sigma: float = SIGMA) -> np.ndarray:
    """Steady node temperatures (K) of the radiation-only balance.

    y: N x (N+1) REF matrix (column N = deep space), face or node level;
    weight: eps_i A_i per node (W_G after aggregation), so GR = sigma w_i y_ij;
    q: heat input per node (W), N values or N x m load cases;
    t_fixed: None or N values, > 0 holds node i at that temperature, 0 = free.
    Returns T with the shape of q.
    """
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    w = np.asarray(weight, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    vec = q.ndim == 1
    qm = q[:, None] if vec else q
    fixed = np.zeros(n, dtype=bool) if t_fixed is None else np.asarray(t_fixed, dtype=np.float64) > 0.0
    tf = np.zeros(n) if t_fixed is None else np.asarray(t_fixed, dtype=np.float64)
    gr = sigma * w[:, None] * y                      # eq. 4.2, N x (N+1)
    # balance row i in x = T^4: (sum_j GR_ij + GR_i,space) x_i - sum_j GR_ij x_j
    #                           = Q_i + GR_i,space T_space^4   (the j = i terms cancel)
    a = -gr[:, :n].copy()
    a[np.arange(n), np.arange(n)] += gr.sum(axis=1)
    rhs = qm + (gr[:, n] * t_space ** 4)[:, None]
    free = ~fixed
    x = np.empty_like(qm)
    x[fixed] = (tf[fixed] ** 4)[:, None]
    if free.any():
        r = rhs[free] - a[np.ix_(free, fixed)] @ x[fixed]
        x[free] = np.linalg.solve(a[np.ix_(free, free)], r)
    t = np.where(x > 0.0, np.abs(x) ** 0.25, np.nan)
    return t[:, 0] if vec else t


def net_radiated_power(y: np.ndarray, weight: np.ndarray, t: np.ndarray, t_space: float = 3.0,
                       sigma: float = SIGMA) -> np.ndarray:
    """Left-hand side of the balance, sum_j q_ij + q_i,space per node (eq. 3.12-3.13)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    t = np.asarray(t, dtype=np.float64)
    tm = t[:, None] if t.ndim == 1 else t
    gr = sigma * np.asarray(weight, dtype=np.float64)[:, None] * y
    x = tm ** 4
    out = np.empty_like(tm)
    for c in range(tm.shape[1]):
        out[:, c] = (gr[:, :n] * (x[:, c][:, None] - x[:, c][None, :])).sum(axis=1) \
            + gr[:, n] * (x[:, c] - t_space ** 4)
    return out[:, 0] if t.ndim == 1 else out
