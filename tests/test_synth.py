"""Pins for the synthetic-input layer: closed-form rectangle view factors.

The closed forms are checked against the textbook unit-square values, against
brute-force Gauss-Legendre quadrature of the view-factor integral (thesis
Sec. 2.4.12, eq. 2.68), and against the enclosure relations (eq. 2.70-2.71).
"""
import numpy as np
import pytest

from synth import geometry as geo
from synth import workloads as W


def quad_vf(p0, p1, n1, q0, q1, n2, order=12):
    """Brute-force eq. 2.68 between two planar rectangles.

    p0 + s*p1... : rectangle given by a corner and two edge vectors (each a 3-vector pair).
    """
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    (o1, u1, v1), (o2, u2, v2) = (p0, p1, n1), (q0, q1, n2)
    a1 = np.linalg.norm(np.cross(u1, v1))
    a2 = np.linalg.norm(np.cross(u2, v2))
    nrm1 = np.cross(u1, v1) / a1
    nrm2 = np.cross(u2, v2) / a2
    pts1 = o1 + x[:, None, None] * u1 + x[None, :, None] * v1
    pts2 = o2 + x[:, None, None] * u2 + x[None, :, None] * v2
    w2 = w[:, None] * w[None, :]
    d = pts2[None, None] - pts1[:, :, None, None]
    r2 = (d * d).sum(-1)
    c1 = (d @ nrm1) / np.sqrt(r2)
    c2 = -(d @ nrm2) / np.sqrt(r2)
    k = np.clip(c1, 0, None) * np.clip(c2, 0, None) / (np.pi * r2)
    integ = (k * w2[:, :, None, None] * w2[None, None]).sum()
    return integ * a2  # (1/A1) * A1 * A2 * mean kernel


def test_unit_square_textbook_values():
    # Howell's catalogue: unit squares, unit gap 0.19982; common edge at 90 deg 0.20004
    assert abs(geo.parallel_vf(0, 1, 0, 1, 0, 1, 0, 1, 1.0) - 0.199825) < 1e-6
    assert abs(geo.perpendicular_vf(0, 1, 0, 1, 0, 1, 0, 1) - 0.200044) < 1e-6


def test_parallel_offset_against_quadrature():
    # rect 1: [0,0.5]x[0,0.3] at z=0 facing +z; rect 2: [0.7,1.1]x[-0.2,0.4] at z=0.6 facing -z
    f = geo.parallel_vf(0, 0.5, 0, 0.3, 0.7, 1.1, -0.2, 0.4, 0.6)
    q = quad_vf(np.array([0, 0, 0.]), np.array([0.5, 0, 0]), np.array([0, 0.3, 0]),
                np.array([0.7, -0.2, 0.6]), np.array([0, 0.6, 0]), np.array([0.4, 0, 0]))
    assert abs(f - q) < 1e-7 * max(1.0, abs(f)) + 1e-9


def test_perpendicular_offset_against_quadrature():
    # rect 1 on z=0: x in [0.2,0.6], y in [0.3,0.8] (distance to plane y=0), facing +z
    # rect 2 on y=0: x in [0.5,1.2], z in [0.1,0.9], facing +y
    f = geo.perpendicular_vf(0.2, 0.6, 0.3, 0.8, 0.5, 1.2, 0.1, 0.9)
    q = quad_vf(np.array([0.2, 0.3, 0.]), np.array([0.4, 0, 0]), np.array([0, 0.5, 0]),
                np.array([0.5, 0, 0.1]), np.array([0, 0, 0.8]), np.array([0.7, 0, 0]))
    assert abs(f - q) < 1e-7


def test_closed_cube_closure_and_reciprocity():
    m = geo.open_box(1, 1, 1, 3, 3, 3, open_top=False)
    f = m.exact_vf()
    assert np.abs(f[:, :-1].sum(1) - 1).max() < 1e-13
    a = m.areas()
    s = a[:, None] * f[:, :-1]
    assert np.abs(s - s.T).max() < 1e-15
    # whole-wall values: 4 adjacent walls at 0.20004 plus the opposite one at 0.19982
    m1 = geo.open_box(1, 1, 1, 1, 1, 1, open_top=False)
    f1 = m1.exact_vf()
    assert abs(f1[0, 1] - 0.200044) < 1e-6 and abs(f1[0, 5] - 0.199825) < 1e-6


def test_fast_grid_path_matches_general_path():
    m = geo.open_box(1.0, 0.8, 0.5, 5, 4, 3)
    f = m.exact_vf()
    n = m.n
    off = m.offsets()
    # re-evaluate every wall pair through the general broadcast path
    for a, p in enumerate(m.walls):
        for b, q in enumerate(m.walls):
            if p is q:
                continue
            if p.ax == q.ax:
                if (q.pos - p.pos) * p.sgn <= 0:
                    continue
                a0, a1 = p.axes
                px0, px1 = p.lo_hi(a0); py0, py1 = p.lo_hi(a1)
                qx0, qx1 = q.lo_hi(a0); qy0, qy1 = q.lo_hi(a1)
                ref = geo.parallel_vf(px0[:, None], px1[:, None], py0[:, None], py1[:, None],
                                      qx0[None], qx1[None], qy0[None], qy1[None], abs(q.pos - p.pos))
                assert np.abs(f[off[a]:off[a + 1], off[b]:off[b + 1]] - ref).max() < 1e-14
    assert f.shape == (n, n + 1)


def test_mcrt_noise_rows_close_and_unbiased():
    inst = W.small_box(4, 2, rays=20000, seed=3)
    assert np.abs(inst.f_noisy.sum(1) - 1).max() < 1e-14
    assert (inst.f_noisy >= 0).all()
    # each entry is count / rays, within 6 binomial sd of the exact value
    f, fe = inst.f_noisy, inst.f_exact
    sd = np.sqrt(fe * (1 - fe) / 20000) + 1e-12
    assert (np.abs(f - fe) <= 6 * sd + 1e-12).all()


def test_config_sizes():
    assert W.config1().n == 32
    m = W.geo.open_box(1, 1, 0.75, 64, 64, 48)
    assert m.n == 16384
    assert W.geo.open_box(1, 1, 0.25, 64, 64, 16).n == 8192
    assert W.geo.chimney(24, 19, 32).n == 4096
