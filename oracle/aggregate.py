"""Oracle: multi-node aggregation of sub-face factors to faces / nodes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Thesis Sec. 5.2.3, eq. 5.6-5.7 (and the first two rows of eq. 5.28): for a
surface n made of sub-surfaces n_i with areas S_{n_i}, S_n = sum_i S_{n_i},

    F_nm   = sum_{i in n} sum_{j in m} F_{n_i m_j} S_{n_i} / S_n
    F_n,inf = sum_{i in n} F_{n_i,inf} S_{n_i} / S_n

One-sided faces only (C_n = 1, where eq. 5.17 is the identity).  The weight is
a per-row input: w_i = S_i for view factors.  For REF matrices the paper gives
no rule; the reading used here is w_i = eps_i S_i, the same substitution
Omega_i = eps_i A_i the paper makes to enforce REFs (Sec. 4.2.3), which keeps
eps_G A_G B_GH = sum eps_i A_i B_ij (the parallel-path sum of App. C, eq. C.2).
"""
from __future__ import annotations

import numpy as np


def aggregate_nodes(x: np.ndarray, weight: np.ndarray, group: np.ndarray, g: int):
    """Returns (Y, W): Y is g x (g+1), W_G = sum_{i in G} w_i."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    group = np.asarray(group, dtype=np.int64)
    w = np.asarray(weight, dtype=np.float64)
    if x.shape != (n, n + 1) or group.shape != (n,) or w.shape != (n,):
        raise ValueError("shape mismatch")
    if group.min() < 0 or group.max() >= g:
        raise ValueError("group id out of range")
    big_w = np.zeros(g)
    np.add.at(big_w, group, w)
    # rows: sum_{i in G} w_i X_ij
    rows = np.zeros((g, n + 1))
    np.add.at(rows, group, w[:, None] * x)
    # columns: sum_{j in H} (.)_Gj, space column kept
    y = np.zeros((g, g + 1))
    np.add.at(y.T, group, rows[:, :n].T)
    y[:, g] = rows[:, n]
    return y / big_w[:, None], big_w
