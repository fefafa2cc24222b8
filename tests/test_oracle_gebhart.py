"""Pins for the oracle's open-system Gebhart solve (thesis Sec. 4.2, App. B, Sec. 6.3)."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.golden.loader import load

E2 = load("e2_parallel_plates.txt")
SIGMA = 5.67e-8


def test_parallel_plates_eq_6_11():
    b = oracle.gebhart_ref(E2["F"], E2["eps"], E2["rho"])
    assert np.abs(b - E2["B"]).max() < 1e-6


def _top_plate_temperature(coupling):
    """Radiation-only steady balance of the top plate (faces 1 and 2, one node).

    coupling[i][j] holds the factor multiplying sigma eps_i A (T_i^4 - T_j^4);
    the plate's common emissivity and area cancel.
    """
    tb = E2["boundary_C"][0] + 273.15
    te = E2["boundary_C"][1] + 273.15
    # node temperatures: faces 1,2 top plate (unknown), 3,4 bottom, column 4 space
    c_bottom = coupling[0][2] + coupling[0][3] + coupling[1][2] + coupling[1][3]
    c_space = coupling[0][4] + coupling[1][4]
    t4 = (c_bottom * tb ** 4 + c_space * te ** 4) / (c_bottom + c_space)
    return t4 ** 0.25 - 273.15


def test_table_6_2_top_plate_temperatures():
    f, eps = E2["F"], E2["eps"]
    # view factors: GR_ij = sigma eps_i eps_j A_i F_ij (eq. 3.11), space is black
    cf = [[eps[j] * f[i, j] if j < 4 else f[i, j] for j in range(5)] for i in range(2)]
    t_vf = _top_plate_temperature(cf)
    # REFs: GR_ij = sigma eps_i A_i B_ij (eq. 4.2)
    b = oracle.gebhart_ref(f, eps, E2["rho"])
    t_ref = _top_plate_temperature([[b[i, j] for j in range(5)] for i in range(2)])
    assert abs(t_vf - E2["temperatures_C"][0]) < 0.01
    assert abs(t_ref - E2["temperatures_C"][1]) < 0.01


def test_two_face_closed_form():
    f23, f32 = 0.285913, 0.285927
    rng = np.random.default_rng(3)
    e2, e3, r2, r3 = rng.uniform(0.1, 0.9, 4)
    f = np.array([[0, f23, 1 - f23], [f32, 0, 1 - f32]])
    b = oracle.gebhart_ref(f, [e2, e3], [r2, r3])
    d = 1 - f23 * f32 * r2 * r3
    assert abs(b[0, 1] - e3 * f23 / d) < 1e-16
    assert abs(b[0, 0] - f23 * f32 * r3 * e2 / d) < 1e-16
    assert abs(b[0, 2] - (f[0, 2] + f23 * r3 * f[1, 2]) / d) < 1e-15


def test_rho_zero_limit_is_e():
    inst = W.small_box(4, 2, seed=1)
    eps = inst.eps[0]
    b = oracle.gebhart_ref(inst.f_noisy, eps, np.zeros(inst.n))
    _, e = oracle.form_k_e(inst.f_noisy, eps, np.zeros(inst.n))
    assert np.array_equal(b, e)


def test_reflection_series_brute_force():
    # B = sum_n (F_sq diag rho)^n E converges since ||F diag rho||_inf <= max rho < 1
    inst = W.small_box(3, 1, seed=2)
    f, eps, rho = inst.f_noisy, inst.eps[0], inst.rho[0]
    n = inst.n
    p = f[:, :n] * rho[None, :]
    _, e = oracle.form_k_e(f, eps, rho)
    term = e.copy()
    acc = e.copy()
    for _ in range(2000):
        term = p @ term
        acc += term
        if np.abs(term).max() < 1e-18:
            break
    b = oracle.gebhart_ref(f, eps, rho)
    assert np.abs(acc - b).max() < 1e-14


def test_random_walk_definition_39():
    """Monte-Carlo of Definition 39: fraction of energy leaving i finally absorbed by j."""
    f, eps, rho = E2["F"], np.array([0.3, 0.6, 0.4, 0.7]), np.array([0.7, 0.4, 0.6, 0.3])
    b = oracle.gebhart_ref(f, eps, rho)
    rng = np.random.default_rng(11)
    walks = 200_000
    n = 4
    cdf = np.cumsum(f, axis=1)
    for src in (1, 2):
        cur = np.full(walks, src)
        alive = np.ones(walks, bool)
        hits = np.zeros(n + 1)
        while alive.any():
            idx = np.nonzero(alive)[0]
            u = rng.uniform(size=idx.size)
            tgt = np.minimum((u[:, None] > cdf[cur[idx]]).sum(1), n)
            to_space = tgt == n
            hits[n] += to_space.sum()
            alive[idx[to_space]] = False
            idx2, tgt2 = idx[~to_space], tgt[~to_space]
            absorbed = rng.uniform(size=idx2.size) < eps[tgt2]
            np.add.at(hits, tgt2[absorbed], 1)
            alive[idx2[absorbed]] = False
            cur[idx2[~absorbed]] = tgt2[~absorbed]
        est = hits / walks
        sd = np.sqrt(b[src] * (1 - b[src]) / walks) + 1e-12
        assert (np.abs(est - b[src]) <= 4.5 * sd).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_ref_closure_and_reciprocity(seed):
    inst = W.small_box(4, 2, seed=seed)
    f, _ = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-15, max_iter=600)
    eps, rho = inst.eps[0], inst.rho[0]
    b = oracle.gebhart_ref(f, eps, rho)
    # eq. 4.3 with space: holds when eps + rho = 1 and F is closed
    assert oracle.ref_closure_residual(b) < 1e-13
    # eq. 4.4: holds for any rho once F is reciprocal
    assert oracle.ref_reciprocity_residual(b, eps, inst.area) < 1e-14
    b2 = oracle.gebhart_ref(f, eps, np.random.default_rng(seed).uniform(0, 0.9, inst.n))
    assert oracle.ref_reciprocity_residual(b2, eps, inst.area) < 1e-14


def test_permutation_equivariance():
    inst = W.small_box(3, 2, seed=4)
    n = inst.n
    perm = np.random.default_rng(1).permutation(n)
    b = oracle.gebhart_ref(inst.f_noisy, inst.eps[0], inst.rho[0])
    fp = inst.f_noisy[perm][:, np.r_[perm, n]]
    bp = oracle.gebhart_ref(fp, inst.eps[0][perm], inst.rho[0][perm])
    assert np.abs(bp - b[perm][:, np.r_[perm, n]]).max() < 1e-15
