"""Pins for the oracle's radiation-only steady-state temperatures (Sec. 3.4.4,
eq. 3.12-3.14 with GR from REFs, eq. 4.2; worked example Sec. 6.3, Table 6.2)."""
import numpy as np

import oracle
from oracle.steady import SIGMA, net_radiated_power, steady_temperature
from synth import geometry as geo
from synth import workloads as W
from tests.golden.loader import load

E2 = load("e2_parallel_plates.txt")
K0 = 273.15


def _plates_top_temperature(y_face):
    """Top plate (faces 1, 2) as one node, bottom plate (faces 3, 4) held at
    500 C, environment at 27 C, no heat input (Sec. 6.3)."""
    eps = E2["eps"]
    w = eps * 1.0  # equal plate areas: A cancels
    y, wn = oracle.aggregate_nodes(y_face, w, np.array([0, 0, 1, 1]), 2)
    tb, te = E2["boundary_C"][0] + K0, E2["boundary_C"][1] + K0
    t = steady_temperature(y, wn, np.zeros(2), t_fixed=np.array([0.0, tb]), t_space=te)
    assert t[1] == tb
    return t[0] - K0


def test_table_6_2_with_refs():
    b = oracle.gebhart_ref(E2["F"], E2["eps"], E2["rho"])
    assert abs(_plates_top_temperature(b) - E2["temperatures_C"][1]) < 0.01


def test_table_6_2_with_view_factors():
    """View-factor couplings GR_ij = sigma eps_i eps_j A_i F_ij (eq. 3.11), a
    black environment: in REF form y_ij = eps_j F_ij, y_i,space = F_i,space."""
    f, eps = E2["F"], E2["eps"]
    y = f.copy()
    y[:, :4] *= eps[None, :]
    assert abs(_plates_top_temperature(y) - E2["temperatures_C"][0]) < 0.01


def test_single_plate_closed_form():
    """A face that sees only space: eps A sigma (T^4 - T_s^4) = Q."""
    eps, area, q, ts = 0.7, 2.5, 300.0, 4.0
    y = np.array([[0.0, 1.0]])
    t = steady_temperature(y, np.array([eps * area]), np.array([q]), t_space=ts)
    assert abs(t[0] - (q / (SIGMA * eps * area) + ts ** 4) ** 0.25) <= 1e-12 * t[0]


def _box_refs(seed):
    m = geo.open_box(1.0, 1.0, 0.5, 4, 4, 2)
    f, area = m.exact_vf(), m.areas()
    n = f.shape[0]
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0.2, 0.9, n)
    b = oracle.gebhart_ref(f, eps, 1.0 - eps)
    return b, eps * area, rng


def test_balance_holds_node_by_node():
    """The returned temperatures satisfy the balance as written with explicit
    differences T_i^4 - T_j^4 (independent of the linear form in T^4).  The
    REFs come from noisy view factors, so GR is not symmetric and a
    transposed coupling would show."""
    inst = W.small_box(5, 2, seed=1)
    eps = inst.eps[0]
    b = oracle.gebhart_ref(inst.f_noisy, eps, inst.rho[0])
    w = eps * inst.area
    rng = np.random.default_rng(1)
    n = b.shape[0]
    assert np.abs(w[:, None] * b[:, :n] - (w[:, None] * b[:, :n]).T).max() > 1e-3 * (w[:, None] * b[:, :n]).max()
    q = rng.uniform(0.0, 50.0, (n, 3))
    t_fixed = np.zeros(n)
    t_fixed[rng.choice(n, 5, replace=False)] = rng.uniform(250.0, 350.0, 5)
    t = steady_temperature(b, w, q, t_fixed=t_fixed, t_space=3.0)
    free = t_fixed == 0
    lhs = net_radiated_power(b, w, t, t_space=3.0)
    assert np.abs(lhs[free] - q[free]).max() <= 1e-9 * np.abs(q).max()
    assert np.array_equal(t[~free], np.repeat(t_fixed[~free][:, None], 3, axis=1))


def test_energy_conservation_with_reciprocal_refs():
    """GR_ij = GR_ji: exchanges between nodes cancel in the sum, so the heat
    put into the free nodes plus what the fixed nodes give off equals the
    power radiated to space."""
    b, w, rng = _box_refs(2)
    n = b.shape[0]
    q = rng.uniform(0.0, 80.0, n)
    t_fixed = np.zeros(n)
    t_fixed[:3] = 320.0
    t = steady_temperature(b, w, q, t_fixed=t_fixed, t_space=3.0)
    lhs = net_radiated_power(b, w, t, t_space=3.0)
    to_space = (SIGMA * w * b[:, n] * (t ** 4 - 3.0 ** 4)).sum()
    put_in = q[t_fixed == 0].sum() + lhs[t_fixed > 0].sum()
    assert abs(put_in - to_space) <= 1e-9 * to_space


def test_isothermal_surroundings():
    b, w, _ = _box_refs(3)
    n = b.shape[0]
    t_fixed = np.zeros(n)
    t_fixed[[0, 7]] = 290.0
    t = steady_temperature(b, w, np.zeros(n), t_fixed=t_fixed, t_space=290.0)
    assert np.abs(t - 290.0).max() <= 1e-9 * 290.0


def test_heat_input_raises_temperatures():
    """Physical sign of the balance: more power into one node warms every
    free node (and that node most)."""
    b, w, rng = _box_refs(4)
    n = b.shape[0]
    q = rng.uniform(1.0, 10.0, n)
    t0 = steady_temperature(b, w, q)
    q[5] += 100.0
    t1 = steady_temperature(b, w, q)
    d = t1 - t0
    assert (d > 0).all() and np.argmax(d) == 5


def test_newton_on_t_agrees():
    """Newton's method on the nonlinear residual in T (the paper's route for
    the general network) reaches the same temperatures."""
    b, w, rng = _box_refs(5)
    n = b.shape[0]
    q = rng.uniform(0.0, 40.0, n)
    gr = SIGMA * w[:, None] * b
    t = np.full(n, 300.0)
    for _ in range(50):
        r = net_radiated_power(b, w, t, t_space=3.0) - q
        jac = -gr[:, :n] * 4.0 * t[None, :] ** 3
        jac[np.arange(n), np.arange(n)] += 4.0 * t ** 3 * gr.sum(axis=1)
        step = np.linalg.solve(jac, r)
        t = t - step
        if np.abs(step).max() < 1e-13 * t.max():
            break
    ref = steady_temperature(b, w, q, t_space=3.0)
    assert np.abs(t - ref).max() <= 1e-10 * ref.max()
