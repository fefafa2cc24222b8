"""Pins for the oracle's iterative enforcer (thesis Sec. 3.5.3-3.5.5, Sec. 6.2)."""
import math

import numpy as np
import pytest

import oracle
from oracle.enforce import kappa_fracvar
from synth import workloads as W
from tests.golden.loader import load

E1 = load("e1_discs_enforcer.txt")


def test_fixture_analytic_matrix_matches_disc_formula():
    # eq. 6.1-6.2 with R1 = 1, R2 = 2 (the reading of the areas used by every E1 pin)
    r1, r2 = 1.0, 2.0
    x = 1.0 + (1.0 + r2 * r2) / (r1 * r1)
    f12 = 0.5 * (x - math.sqrt(x * x - 4.0 * (r2 / r1) ** 2))
    assert abs(f12 - 0.763932) < 5e-7
    assert abs(f12 / 4.0 - 0.190983) < 5e-7  # reciprocity with A2 = 4 A1


def test_closure_only_leaves_mcrt_matrix_unchanged():
    # eq. 6.4 -> 6.5: MCRT rows already close
    f2 = oracle.closure_step(E1["F1_mcrt"], E1["areas"])
    assert np.abs(f2 - E1["F2_closure"]).max() < 1e-12


def test_one_reciprocity_step_matches_eq_6_6():
    f3 = oracle.reciprocity_step(E1["F1_mcrt"], E1["areas"], kappa="half")
    assert np.abs(f3 - E1["F3_reciprocity"]).max() < 1e-6
    # Sec. 6.2: the line sums of F3's first two rows are 0.99964 and 1.00009
    s = f3.sum(1)
    assert abs(s[0] - 0.99964) < 6e-6 and abs(s[1] - 1.00009) < 6e-6


def test_iterative_enforcer_matches_eq_6_9_in_13_iterations():
    f, info = oracle.enforce_vf(E1["F1_mcrt"], E1["areas"], kappa="half", tol=1e-7, max_iter=100)
    assert info["iters"] == int(E1["iterations"]) and info["converged"]
    assert np.abs(f - E1["F6_iterative"]).max() < 1e-6


def test_mae_table_6_1():
    t = E1["mae_table_6_1"]
    fe = E1["F_analytical"]
    assert abs(oracle.mae(E1["F1_mcrt"], fe) - t[0]) < 5e-8
    f2 = oracle.closure_step(E1["F1_mcrt"], E1["areas"])
    assert abs(oracle.mae(f2, fe) - t[1]) < 5e-8
    f3 = oracle.reciprocity_step(E1["F1_mcrt"], E1["areas"], kappa="half")
    assert abs(oracle.mae(f3, fe) - t[2]) < 5e-8
    f6, _ = oracle.enforce_vf(E1["F1_mcrt"], E1["areas"], kappa="half", tol=1e-7, max_iter=100)
    assert abs(oracle.mae(f6, fe) - t[5]) < 1e-7


def _random_closed_reciprocal(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 2.0, n)
    s = rng.uniform(0, 1, (n, n))
    s = s + s.T
    np.fill_diagonal(s, 0)
    f = s / a[:, None]
    f = f / (f.sum(1, keepdims=True) * rng.uniform(1.05, 2.0, (n, 1)))
    # reciprocity broken by the rescale: restore it by min-scaling the symmetric part
    eta = a[:, None] * f
    eta = np.minimum(eta, eta.T)
    f = eta / a[:, None]
    out = np.empty((n, n + 1))
    out[:, :n] = f
    out[:, n] = 1 - f.sum(1)
    return out, a


@pytest.mark.parametrize("mode", ["half", "fracvar"])
def test_exact_input_is_fixed_point(mode):
    f, a = _random_closed_reciprocal(7, 1)
    assert (f >= 0).all()
    g, info = oracle.enforce_vf(f, a, n_rays=np.full(7, 1e4), kappa=mode, max_iter=5)
    assert np.abs(g - f).max() < 1e-15 * 10
    assert info["closure_defect"] < 1e-15 * 10


def test_fracvar_kappa_minimises_estimator_variance():
    # eq. 3.24 -> 3.25: brute-force the variance over kappa in [0, 1]
    inst = W.small_box(3, 1, rays=500, seed=2)
    f, a, nr = inst.f_noisy, inst.area * np.linspace(0.5, 2, inst.n), inst.n_rays * np.linspace(1, 3, inst.n)
    n = inst.n
    kap = kappa_fracvar(f, a, nr)
    grid = np.linspace(0, 1, 20001)
    checked = 0
    for i in range(n):
        for j in range(n):
            if i == j or f[i, j] <= 0 or f[j, i] <= 0:
                continue
            s_ij = (a[i] * math.sqrt((1 - f[i, j]) / (nr[i] * f[i, j]))) ** 2  # eq. 3.23 (z = 1)
            s_ji = (a[j] * math.sqrt((1 - f[j, i]) / (nr[j] * f[j, i]))) ** 2
            var = grid ** 2 * s_ij + (1 - grid) ** 2 * s_ji                   # eq. 3.24
            assert abs(grid[np.argmin(var)] - kap[i, j]) <= 1e-4
            assert abs(kap[i, j] + kap[j, i] - 1) < 1e-14
            checked += 1
    assert checked > 10


def test_fracvar_limits():
    f = np.array([[0, 0.3, 0.0, 0.7], [0.2, 0, 0.5, 0.3], [0.0, 0.4, 0, 0.6]])
    a = np.array([1.0, 2.0, 1.5])
    nr = np.full(3, 1e4)
    kap = kappa_fracvar(f, a, nr)
    # both zero -> 1/2 ; one zero -> all weight on the other
    assert kap[0, 2] == 0.5 and kap[2, 0] == 0.5
    g = oracle.reciprocity_step(f, a, nr, "fracvar")
    assert g[0, 2] == 0 and g[2, 0] == 0
    f2 = f.copy(); f2[1, 0] = 0.0; f2[1, 3] = 0.5
    kap2 = kappa_fracvar(f2, a, nr)
    assert kap2[1, 0] == 0.0 and kap2[0, 1] == 1.0
    g2 = oracle.reciprocity_step(f2, a, nr, "fracvar")
    assert abs(a[1] * g2[1, 0] - a[0] * f2[0, 1]) < 1e-16 and g2[0, 1] == f2[0, 1]


def test_equal_variance_pairs_reduce_to_half():
    # equal areas, equal rays and F_ij = F_ji give equal variances: kappa = 1/2
    inst = W.small_box(3, 1, rays=800, seed=4)
    n = inst.n
    f = inst.f_noisy.copy()
    sym = 0.5 * (f[:, :n] + f[:, :n].T)
    f[:, :n] = sym
    a = np.ones(n)
    g1 = oracle.reciprocity_step(f, a, np.full(n, 800.0), "fracvar")
    g2 = oracle.reciprocity_step(f, a, None, "half")
    assert np.abs(g1 - g2).max() < 1e-16


@pytest.mark.parametrize("mode", ["half", "fracvar"])
def test_invariants_on_noisy_box(mode):
    inst = W.small_box(4, 2, rays=3000, seed=5)
    n = inst.n
    f, info = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, mode, tol=1e-14, max_iter=400)
    assert info["converged"]
    assert (f >= 0).all()
    assert np.abs(f.sum(1) - 1).max() < 1e-14
    eta = inst.area[:, None] * f[:, :n]
    assert np.abs(eta - eta.T).max() / eta.max() < 1e-13
    # zeros of the input (coplanar faces) stay zero
    z = inst.f_noisy[:, :n] == 0
    zz = z & z.T
    assert (f[:, :n][zz] == 0).all()
    # permutation equivariance and area-scale invariance
    perm = np.random.default_rng(0).permutation(n)
    fp = inst.f_noisy[perm][:, np.r_[perm, n]]
    gp, _ = oracle.enforce_vf(fp, inst.area[perm], inst.n_rays[perm], mode, tol=0, max_iter=info["iters"])
    assert np.abs(gp - f[perm][:, np.r_[perm, n]]).max() < 1e-13
    gs, _ = oracle.enforce_vf(inst.f_noisy, 3.7 * inst.area, inst.n_rays, mode, tol=0, max_iter=info["iters"])
    assert np.abs(gs - f).max() < 1e-13


def test_enforcement_reduces_error_against_exact():
    # statistical sanity (Table 6.1's trend), not parity
    inst = W.small_box(6, 3, rays=2000, seed=6)
    f, _ = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-12, max_iter=500)
    assert oracle.mae(f, inst.f_exact) < oracle.mae(inst.f_noisy, inst.f_exact)


def test_closure_step_is_row_normalisation():
    rng = np.random.default_rng(9)
    f = rng.uniform(0, 1, (6, 7))
    g = oracle.closure_step(f, rng.uniform(0.5, 2, 6))
    assert np.abs(g - f / f.sum(1, keepdims=True)).max() < 1e-15
    with pytest.raises(ValueError):
        oracle.closure_step(np.zeros((2, 3)))
