"""Pins for the oracle's absorbed heat fluxes (thesis Sec. 4.2.3, eq. 4.6)."""
import numpy as np

import oracle
from synth import geometry as geo
from synth import workloads as W


def _exact_open_box():
    m = geo.open_box(1.0, 1.0, 0.5, 4, 4, 2)
    return m.exact_vf(), m.areas()


def test_reflection_series_from_view_factors():
    """Follow the power physically: the direct power on each face is partly
    absorbed and partly reflected; reflected power travels by the view
    factors to the other faces (or to space), where the same split repeats.
    The absorbed totals of this series must equal eq. 4.6 with the REFs of
    the Gebhart solve (which sums the series in closed form)."""
    f, area = _exact_open_box()
    n = f.shape[0]
    rng = np.random.default_rng(5)
    eps = rng.uniform(0.2, 0.9, n)
    rho = 1.0 - eps
    qd = rng.uniform(0.0, 1400.0, (n, 3))
    b = oracle.gebhart_ref(f, eps, rho)
    qa = oracle.absorbed_flux(b, eps, rho, area, qd)
    absorbed = np.zeros_like(qd)
    arriving = area[:, None] * qd          # power arriving at each face
    for _ in range(400):
        absorbed += eps[:, None] * arriving
        reflected = rho[:, None] * arriving
        arriving = f[:, :n].T @ reflected  # reflected power from j reaching k: F_jk
        if np.abs(arriving).max() < 1e-14 * np.abs(absorbed).max():
            break
    assert np.abs(qa - absorbed).max() <= 1e-10 * np.abs(absorbed).max()


def test_energy_balance_with_closed_refs():
    """eps + rho = 1 and closed REF rows (sum_i B_ji + B_j,space = 1): the
    absorbed power plus the reflected power lost to space is the incident
    power."""
    inst = W.small_box(5, 2, seed=3)
    f, _ = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-15, max_iter=800)
    eps, rho = inst.eps[0], inst.rho[0]
    b = oracle.gebhart_ref(f, eps, rho)
    n = inst.n
    qd = np.random.default_rng(1).uniform(0.0, 1000.0, (n, 4))
    qa = oracle.absorbed_flux(b, eps, rho, inst.area, qd)
    lost = (b[:, n] * inst.area * rho) @ qd
    incident = inst.area @ qd
    assert np.abs(qa.sum(axis=0) + lost - incident).max() <= 1e-11 * incident.max()


def test_non_reflecting_faces_absorb_only_their_direct_flux():
    inst = W.small_box(4, 2, seed=2)
    n = inst.n
    eps = np.random.default_rng(4).uniform(0.1, 1.0, n)
    b = oracle.gebhart_ref(inst.f_noisy, eps, np.zeros(n))
    qd = np.random.default_rng(6).uniform(0.0, 500.0, n)
    qa = oracle.absorbed_flux(b, eps, np.zeros(n), inst.area, qd)
    assert np.array_equal(qa, inst.area * eps * qd)


def test_reciprocal_form():
    """With reciprocal REFs (eps_j A_j B_ji = eps_i A_i B_ij, exact view
    factors) eq. 4.6 equals A_i eps_i [Q_i + sum_j B_ij (rho_j / eps_j) Q_j],
    which tells B from its transpose."""
    f, area = _exact_open_box()
    n = f.shape[0]
    rng = np.random.default_rng(9)
    eps = rng.uniform(0.3, 0.95, n)
    rho = 1.0 - eps
    b = oracle.gebhart_ref(f, eps, rho)
    qd = rng.uniform(0.0, 1.0, n)
    qa = oracle.absorbed_flux(b, eps, rho, area, qd)
    alt = area * eps * (qd + b[:, :n] @ (rho / eps * qd))
    assert np.abs(qa - alt).max() <= 1e-12 * np.abs(qa).max()
