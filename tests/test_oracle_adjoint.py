"""Pins for the oracle's REF gradients: central finite differences of the solve."""
import numpy as np
import pytest

import oracle
from synth import workloads as W

SIGMA = 5.67e-8


def _objective(b, w):
    return float((w * b).sum())


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    inst = W.small_box(3, 2, seed=seed)
    n = inst.n
    f, eps, rho = inst.f_noisy, inst.eps[0].copy(), inst.rho[0].copy()
    w = np.random.default_rng(seed).uniform(0, 1, (n, n + 1))
    b = oracle.gebhart_ref(f, eps, rho)
    ge, gr, _ = oracle.gebhart_ref_adjoint(f, eps, rho, b, w)
    h = 1e-6
    for k in range(n):
        d = np.zeros(n); d[k] = h
        fd_e = (_objective(oracle.gebhart_ref(f, eps + d, rho), w) - _objective(oracle.gebhart_ref(f, eps - d, rho), w)) / (2 * h)
        fd_r = (_objective(oracle.gebhart_ref(f, eps, rho + d), w) - _objective(oracle.gebhart_ref(f, eps, rho - d), w)) / (2 * h)
        assert abs(fd_e - ge[k]) <= 1e-7 * max(1.0, abs(ge[k]))
        assert abs(fd_r - gr[k]) <= 1e-7 * max(1.0, abs(gr[k]))


def test_two_face_closed_form_derivative():
    # B_23 = eps_3 F_23 / (1 - F_23 F_32 rho_2 rho_3): derivatives by hand
    f23, f32 = 0.3, 0.25
    e2, e3, r2, r3 = 0.4, 0.7, 0.6, 0.3
    f = np.array([[0, f23, 1 - f23], [f32, 0, 1 - f32]])
    b = oracle.gebhart_ref(f, [e2, e3], [r2, r3])
    g = np.zeros((2, 3)); g[0, 1] = 1.0  # J = B_23
    ge, gr, _ = oracle.gebhart_ref_adjoint(f, [e2, e3], [r2, r3], b, g)
    d = 1 - f23 * f32 * r2 * r3
    assert abs(ge[1] - f23 / d) < 1e-15 and abs(ge[0]) < 1e-16
    assert abs(gr[0] - e3 * f23 * f23 * f32 * r3 / d ** 2) < 1e-15
    assert abs(gr[1] - e3 * f23 * f23 * f32 * r2 / d ** 2) < 1e-15


def test_rho_gradient_identity():
    # K^T Lambda = G  =>  rho_k (F^T Lambda)_kj = Lambda_kj - G_kj, so
    # dJ/drho_k = (1/rho_k) sum_j B_kj (Lambda_kj - G_kj)
    inst = W.small_box(4, 2, seed=3)
    n = inst.n
    f, eps, rho = inst.f_noisy, inst.eps[0], inst.rho[0]
    g = np.random.default_rng(2).uniform(-1, 1, (n, n + 1))
    b = oracle.gebhart_ref(f, eps, rho)
    _, gr, lam = oracle.gebhart_ref_adjoint(f, eps, rho, b, g)
    alt = (b * (lam - g)).sum(1) / rho
    assert np.abs(alt - gr).max() < 1e-12 * np.abs(gr).max()
