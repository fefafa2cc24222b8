"""Oracle: two-sided multi-node relations (view fractions, node emissivity).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A node is a sub-surface n_i with C_n faces (one, A, or two, A and B, of the
same area S_{n_i}); the MCRT and the Gebhart solve work on faces.  The rows
and columns of the face-level matrices here are faces, ``group[a]`` names the
node of face a, and column nf is deep space.

* Node factors (Sec. 5.2.4-5.2.6, eq. 5.17 / 5.28): F_ij = (1/C_n) sum over
  the face pairs (X, Y) of F^{X->Y}_{n_i m_j}; this is the area-weighted
  aggregation of ``oracle.aggregate`` with the face areas as weights (W_G =
  C_n S_{n_i}, the node area of eq. 5.36), written out here as the plain sum.
* View fractions (eq. 5.27 / 5.29): the share of one face pair in the node
  pair's total, f^{X->Y}_{n_i m_j} = F^{X->Y}_{n_i m_j} / sum_{X', Y'}
  F^{X'->Y'}_{n_i m_j}, and likewise for deep space.
* Node emissivity (App. C, eq. C.2-C.4): the emissivity that makes
  GR_ij = eps_ij C_i S_i B_ij hold with the node REF B_ij of eq. 5.17,
  eps_ij = sum_X eps^X sum_Y B^{X->Y} / sum_{X,Y} B^{X->Y}; it depends on
  the node pair through the view fractions of B.

Readings: a node pair without exchange (zero denominator) gets view fraction
0 and, for the emissivity, the area-weighted mean emissivity of node i (any
value gives GR_ij = 0).
"""
from __future__ import annotations

import numpy as np


def _pair_sums(x: np.ndarray, group: np.ndarray, g: int, row_weight=None) -> np.ndarray:
    """S[G, H] = sum_{a in G} r_a sum_{b in H} x_ab (H = g is deep space), as
    products with the face-to-node incidence matrix P (P[a, G] = 1 if a in G)."""
    nf = x.shape[0]
    r = np.ones(nf) if row_weight is None else np.asarray(row_weight, dtype=np.float64)
    p = np.zeros((nf, g))
    p[np.arange(nf), group] = 1.0
    cols = np.empty((nf, g + 1))
    cols[:, :g] = x[:, :nf] @ p
    cols[:, g] = x[:, nf]
    return p.T @ (r[:, None] * cols)


def node_view_factors(f: np.ndarray, group, g: int):
    """Eq. 5.17: F_ij = (1/C_n) sum over face pairs; returns (F_node, C)."""
    f = np.asarray(f, dtype=np.float64)
    group = np.asarray(group, dtype=np.int64)
    c = np.bincount(group, minlength=g).astype(np.float64)
    return _pair_sums(f, group, g) / c[:, None], c


def view_fractions(f: np.ndarray, group, g: int) -> np.ndarray:
    """Eq. 5.29 per face pair (face-level shape nf x (nf+1))."""
    f = np.asarray(f, dtype=np.float64)
    group = np.asarray(group, dtype=np.int64)
    nf = f.shape[0]
    tot = _pair_sums(f, group, g)
    cols = np.append(group, g)
    den = tot[group][:, cols]
    out = np.zeros((nf, nf + 1))
    nz = den != 0.0
    out[nz] = f[nz] / den[nz]
    return out


def node_emissivity(b: np.ndarray, eps, area, group, g: int) -> np.ndarray:
    """Eq. C.4 for every node pair (g x (g+1)) from face-level REFs."""
    b = np.asarray(b, dtype=np.float64)
    group = np.asarray(group, dtype=np.int64)
    eps = np.asarray(eps, dtype=np.float64)
    s = np.asarray(area, dtype=np.float64)
    num = _pair_sums(b, group, g, eps * s)
    den = _pair_sums(b, group, g, s)
    mean = np.bincount(group, weights=eps * s, minlength=g) / np.bincount(group, weights=s, minlength=g)
    out = np.repeat(mean[:, None], g + 1, axis=1)
    nz = den != 0.0
    out[nz] = num[nz] / den[nz]
    return out
