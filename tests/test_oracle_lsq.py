"""Pins for the oracle's least-squares optimum enforcer (Sec. 3.5.5,
eq. 3.41-3.52; NNR App. A.1, SPVA App. A.2; worked example Sec. 6.2)."""
import numpy as np
import pytest

import oracle
from oracle.lsq import enforce_lsq, restriction_matrix
from synth import workloads as W
from tests.golden.loader import load

E1 = load("e1_discs_enforcer.txt")

# eq. 6.7 and 6.8 as printed (6 decimals)
F4 = np.array([[0.000019, 0.763948, 0.000006, 0.000017, 0.236009],
               [0.190987, 0, 0, 0, 0.809013],
               [0.000006, 0, 0, 0, 0.999994],
               [0.000004, 0, 0, 0, 0.999996]])
F5 = np.array([[0, 0.763969, 0, 0, 0.236031],
               [0.190992, 0, 0, 0, 0.809008],
               [0, 0, 0, 0, 1],
               [0, 0, 0, 0, 1]])


def test_eq_6_8_least_squares_nnr_spva():
    f, info = enforce_lsq(E1["F1_mcrt"], E1["areas"], nnr=True, spva=True)
    assert np.abs(f - F5).max() <= 1e-6
    assert abs(oracle.mae(f, E1["F_analytical"]) - E1["mae_table_6_1"][4]) <= 0.05e-6


def test_eq_6_7_least_squares_nnr():
    """The input is eq. 6.4 printed to 6 decimals, so the result agrees with
    eq. 6.7 to about one unit of its last printed digit."""
    f, info = enforce_lsq(E1["F1_mcrt"], E1["areas"], nnr=True, spva=False)
    assert info["rounds"] > 1  # NNR removed negative coefficients
    assert np.abs(f - F4).max() <= 1.5e-6
    assert abs(oracle.mae(f, E1["F_analytical"]) - E1["mae_table_6_1"][3]) <= 0.2e-6


def _kkt_projection(a, b, x):
    """The same projection from the optimality conditions of
    min |y - x|^2 s.t. A y = b: [I A^T; A 0] [y; l] = [x; b]."""
    keep = np.abs(a).sum(axis=1) > 0
    a, b = a[keep], b[keep]
    m, k = a.shape
    kkt = np.block([[np.eye(k), a.T], [a, np.zeros((m, m))]])
    return np.linalg.solve(kkt, np.concatenate([x, b]))[:k]


def test_plain_projection_matches_the_optimality_conditions():
    inst = W.small_box(3, 1, seed=2)
    n = inst.n
    f, _ = enforce_lsq(inst.f_noisy, inst.area, nnr=False, spva=False)
    a, b = restriction_matrix(n, inst.area)
    y = _kkt_projection(a, b, inst.f_noisy.reshape(-1))
    assert np.abs(f.reshape(-1) - y).max() <= 1e-12


@pytest.mark.parametrize("spva", [False, True])
def test_constraints_sign_and_zeros(spva):
    inst = W.small_box(3, 1, seed=5)
    n = inst.n
    f, info = enforce_lsq(inst.f_noisy, inst.area, nnr=True, spva=spva)
    assert np.abs(f.sum(axis=1) - 1.0).max() <= 1e-12
    eta = inst.area[:, None] * f[:, :n]
    assert np.abs(eta - eta.T).max() <= 1e-12 * eta.max()
    assert f.min() >= 0.0
    if spva:
        assert np.all(f[inst.f_noisy == 0.0] == 0.0)
    # closer to the exact factors than the MCRT input
    assert oracle.mae(f, inst.f_exact) < oracle.mae(inst.f_noisy, inst.f_exact)


def test_exact_factors_are_a_fixed_point():
    inst = W.small_box(3, 1, seed=1)
    f, info = enforce_lsq(inst.f_exact, inst.area, nnr=True, spva=True)
    assert info["rounds"] == 1
    assert np.abs(f - inst.f_exact).max() <= 1e-13


@pytest.mark.parametrize("case", ["e1", "box"])
@pytest.mark.parametrize("spva", [False, True])
def test_nnr_spva_result_is_the_kkt_projection_of_the_reduced_system(case, spva):
    """With NNR (and SPVA) active, the result on the coefficients left free
    is the Euclidean projection of the MCRT input onto the restrictions with
    the removed columns deleted (App. A.1-A.2), computed here from the
    optimality conditions rather than the null-space form of eq. 3.47-3.52;
    the removed coefficients are exactly zero and none is negative."""
    if case == "e1":
        x, omega = E1["F1_mcrt"], E1["areas"]
    else:
        inst = W.small_box(3, 1, seed=11, rays=200)
        x, omega = inst.f_noisy, inst.area
    n = x.shape[0]
    f, info = enforce_lsq(x, omega, nnr=True, spva=spva)
    act = info["active"].reshape(-1)
    if spva:
        assert not act[x.reshape(-1) == 0.0].any()
    a, b = restriction_matrix(n, omega)
    y = _kkt_projection(a[:, act], b, x.reshape(-1)[act])
    assert np.abs(f.reshape(-1)[act] - y).max() <= 1e-12
    assert np.all(f.reshape(-1)[~act] == 0.0)
    assert f.min() >= 0.0
    if case == "e1" and not spva:
        assert info["rounds"] > 1  # NNR removed coefficients that the plain projection made negative
