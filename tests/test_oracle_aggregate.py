"""Pins for the oracle's multi-node aggregation (thesis Sec. 5.2-5.3)."""
import numpy as np
import pytest

import oracle
from synth import geometry as geo
from synth import workloads as W


def test_additivity_reproduces_whole_square_closed_form():
    # sub-face exact F of two 4x4-meshed unit squares -> two whole squares
    inst = W.config1()
    y, wg = oracle.aggregate_nodes(inst.f_exact, inst.area, inst.groups[0], 2)
    assert abs(y[0, 1] - geo.parallel_vf(0, 1, 0, 1, 0, 1, 0, 1, 1.0)) < 1e-14
    assert abs(y[0, 2] - (1 - 0.19982489569838732)) < 1e-13
    assert np.allclose(wg, [1.0, 1.0], rtol=0, atol=1e-15)


def test_closed_cube_aggregates_to_coarse_mesh():
    fine = geo.open_box(1, 1, 1, 3, 3, 3, open_top=False)
    coarse = geo.open_box(1, 1, 1, 1, 1, 1, open_top=False)
    groups = np.repeat(np.arange(6), 9).astype(np.int32)
    y, _ = oracle.aggregate_nodes(fine.exact_vf(), fine.areas(), groups, 6)
    assert np.abs(y - coarse.exact_vf()).max() < 1e-14


def _enforced(seed=0):
    inst = W.small_box(4, 2, seed=seed)
    f, _ = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-15, max_iter=600)
    return inst, f


def test_closure_and_reciprocity_preserved():
    inst, f = _enforced()
    n = inst.n
    g = np.random.default_rng(0).integers(0, 7, n).astype(np.int32)
    g[:7] = np.arange(7)
    y, wg = oracle.aggregate_nodes(f, inst.area, g, 7)
    assert np.abs(y.sum(1) - 1).max() < 1e-14          # eq. 5.31-5.33
    s = wg[:, None] * y[:, :7]
    assert np.abs(s - s.T).max() < 1e-14                # eq. 5.35-5.36


def test_composition_and_identity():
    inst, f = _enforced(1)
    n = inst.n
    rng = np.random.default_rng(1)
    g1 = rng.integers(0, 10, n).astype(np.int32); g1[:10] = np.arange(10)
    g2 = rng.integers(0, 3, 10).astype(np.int32); g2[:3] = np.arange(3)
    y1, w1 = oracle.aggregate_nodes(f, inst.area, g1, 10)
    y2, _ = oracle.aggregate_nodes(y1, w1, g2, 3)
    yd, _ = oracle.aggregate_nodes(f, inst.area, g2[g1], 3)
    assert np.abs(y2 - yd).max() < 1e-15
    yi, _ = oracle.aggregate_nodes(f, inst.area, np.arange(n, dtype=np.int32), n)
    assert np.abs(yi - f).max() < 1e-16


def test_ref_aggregation_keeps_gebhart_relations():
    inst, f = _enforced(2)
    n = inst.n
    eps, rho = inst.eps[0], inst.rho[0]
    b = oracle.gebhart_ref(f, eps, rho)
    g = (np.arange(n) % 5).astype(np.int32)
    y, wg = oracle.aggregate_nodes(b, eps * inst.area, g, 5)
    assert np.abs(y.sum(1) - 1).max() < 1e-13
    s = wg[:, None] * y[:, :5]  # eps_G A_G B_GH
    assert np.abs(s - s.T).max() < 1e-14
