"""Seeded synthetic workloads: geometry, MCRT-like noise and optical properties.

This module only *generates inputs*.  It is shared by the tests, the benchmark
and the GPU smoke check so that the HIP path and the CPU oracle are fed the
very same arrays; it contains none of the enforcement, Gebhart or aggregation
arithmetic.

Monte-Carlo noise stands in for the ray tracer: the estimator F_ij = N_ij / N_i
(thesis, Sec. 3.5.1, eq. 3.15) is simulated per emitting face by a multinomial
draw of the face's rays over its N targets plus space, with probabilities equal
to the exact view factors; rows of the noisy matrix therefore close exactly,
as MCRT rows do (Sec. 3.5.4).

Seeds: ``numpy.random.SeedSequence([2511, 4277, config, instance])`` feeding
PCG64, one stream per (config, instance).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import geometry as geo

SIGMA_SB = 5.67e-8  # W m^-2 K^-4, the value the thesis uses (Sec. 2.4)


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2511, 4277, config, instance])))


def mcrt_noise(f_exact: np.ndarray, rays: int, rng: np.random.Generator) -> np.ndarray:
    """Noisy open-system matrix: per-row multinomial counts / rays."""
    p = np.clip(f_exact, 0.0, None)
    p = p / p.sum(axis=1, keepdims=True)
    counts = rng.multinomial(int(rays), p)
    return counts.astype(np.float64) / float(rays)


@dataclasses.dataclass
class Instance:
    """One open N-face model with its noisy and exact view factors."""

    name: str
    f_noisy: np.ndarray          # (N, N+1) float64, last column = space
    f_exact: np.ndarray          # (N, N+1) float64
    area: np.ndarray             # (N,)
    n_rays: np.ndarray           # (N,) rays emitted per face
    eps: List[np.ndarray]        # per band (N,)
    rho: List[np.ndarray]        # per band (N,)
    groups: List[np.ndarray] = dataclasses.field(default_factory=list)  # aggregation levels
    node_temp: Optional[np.ndarray] = None  # per group of the last level, K

    @property
    def n(self) -> int:
        return self.area.shape[0]


def _finish(name, model, rays, rng, eps_lo, eps_hi, bands=1, fixed_eps=None) -> Instance:
    f_exact = model.exact_vf()
    f_noisy = mcrt_noise(f_exact, rays, rng)
    n = model.n
    eps, rho = [], []
    for b in range(bands):
        if fixed_eps is not None:
            e = np.full(n, float(fixed_eps))
        else:
            lo, hi = (eps_lo, eps_hi) if bands == 1 else [(0.05, 0.95), (0.1, 0.9)][b]
            e = rng.uniform(lo, hi, size=n)
        eps.append(e)
        rho.append(1.0 - e)
    return Instance(name, f_noisy, f_exact, model.areas(), np.full(n, float(rays)), eps, rho)


def config1() -> Instance:
    """Two coaxial unit squares 1 m apart, 4x4 cells each (N = 32)."""
    model = geo.square_pair(1.0, 1.0, 4)
    inst = _finish("two_squares_n32", model, 10_000, rng_for(1), 0.8, 0.8, fixed_eps=0.8)
    inst.groups = [geo.block_groups(model, 4)]  # the two whole squares
    return inst


def config2() -> Instance:
    """Open unit cube, five walls of 32x32 cells (N = 5120), 1e5 rays per face."""
    model = geo.open_box(1.0, 1.0, 1.0, 32, 32, 32)
    return _finish("open_cube_n5120", model, 100_000, rng_for(2), 0.1, 0.9)


def _mesh_box(a: float, b: float, target: int):
    lx, ly, lz = 1.0, a, b
    area = lx * ly + 2 * lx * lz + 2 * ly * lz
    h = math.sqrt(area / target)
    nx, ny, nz = (max(1, round(l / h)) for l in (lx, ly, lz))
    return geo.open_box(lx, ly, lz, nx, ny, nz)


def _mesh_plates(kind: int, w: float, gap: float, target: int):
    # each plate is 1 m x w m; target faces split evenly
    h = math.sqrt(2.0 * w / target)
    n1 = max(1, round(1.0 / h))
    nw = max(1, round(w / h))
    if kind == 0:
        hh = 1.0 / n1
        hw = w / nw
        return geo.Model([
            geo.Wall(2, 0.0, +1, 0.0, hh, n1, 0.0, hw, nw, "plate_lo"),
            geo.Wall(2, gap, -1, 0.0, hh, n1, 0.0, hw, nw, "plate_hi"),
        ])
    return geo.plate_pair_perpendicular(1.0, 1.0, w, gap, n1, n1, nw)


def config3_instance(i: int) -> Instance:
    """One instance of the uneven-N batch: open box or plate pair, two bands."""
    rng = rng_for(3, i)
    target = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
    if rng.uniform() < 0.5:
        a, b = rng.uniform(0.5, 2.0, size=2)
        model = _mesh_box(float(a), float(b), target)
        name = f"box_{i}"
    else:
        kind = int(rng.integers(0, 2))
        w = float(rng.uniform(0.5, 2.0))
        gap = float(rng.uniform(0.2, 2.0))
        model = _mesh_plates(kind, w, gap, target)
        name = f"plates{90 * kind}_{i}"
    return _finish(name, model, 10_000, rng, 0.0, 0.0, bands=2)


def config3(count: int = 64) -> List[Instance]:
    return [config3_instance(i) for i in range(count)]


def _rect_block_groups(model: geo.Model, blocks) -> np.ndarray:
    out, base = [], 0
    for w, (b0, b1) in zip(model.walls, blocks):
        if w.n0 % b0 or w.n1 % b1:
            raise ValueError("block does not tile the wall")
        i0, i1 = np.meshgrid(np.arange(w.n0), np.arange(w.n1), indexing="ij")
        g = (i0 // b0) * (w.n1 // b1) + (i1 // b1)
        out.append(base + g.ravel())
        base += (w.n0 // b0) * (w.n1 // b1)
    return np.concatenate(out).astype(np.int32)


def config4() -> Instance:
    """Open unit box plus two 1 m x 2 m vertical panels: N = 4096 -> 64 nodes."""
    model = geo.chimney(24, 19, 32)
    rng = rng_for(4)
    inst = _finish("chimney_n4096", model, 100_000, rng, 0.1, 0.9)
    # walls: 4 x 3 blocks of 6 x 8 faces; panels (19 x 32): 2 blocks of 19 x 16
    blocks = [(6, 8)] * 5 + [(19, 16)] * 2
    inst.groups = [_rect_block_groups(model, blocks)]
    inst.node_temp = rng.uniform(200.0, 350.0, size=64)
    return inst


def _two_level_groups(model: geo.Model, b1: int, b2: int):
    g1 = geo.block_groups(model, b1)
    # faces are b1 x b1 cell blocks; nodes are b2 x b2 face blocks
    face_walls = [geo.Wall(w.ax, w.pos, w.sgn, w.o0, w.h0 * b1, w.n0 // b1,
                           w.o1, w.h1 * b1, w.n1 // b1, w.name) for w in model.walls]
    g2 = geo.block_groups(geo.Model(face_walls), b2)
    return g1, g2


def config5() -> Instance:
    """Open box 1 x 1 x 0.75 m at 1/64 m cells: N = 16384 -> 4096 -> 256."""
    model = geo.open_box(1.0, 1.0, 0.75, 64, 64, 48)
    inst = _finish("open_box_n16384", model, 10_000, rng_for(5), 0.1, 0.9)
    inst.groups = list(_two_level_groups(model, 2, 4))
    return inst


def metric_workload() -> Instance:
    """Open box 1 x 1 x 0.25 m at 1/64 m cells: N = 8192 faces, 1e4 rays.

    Faces group 2 x 2 -> 2048, then 4 x 4 -> 128 nodes.
    """
    model = geo.open_box(1.0, 1.0, 0.25, 64, 64, 16)
    inst = _finish("open_box_n8192", model, 10_000, rng_for(8192), 0.1, 0.9)
    inst.groups = list(_two_level_groups(model, 2, 4))
    return inst


def small_box(n_side: int = 4, depth_cells: int = 2, rays: int = 2000, seed: int = 0,
              bands: int = 1) -> Instance:
    """Small open box for fast parity tests (N = n^2 + 4 n d)."""
    model = geo.open_box(1.0, 1.0, depth_cells / n_side, n_side, n_side, depth_cells)
    rng = rng_for(100, seed)
    return _finish(f"small_box_{model.n}", model, rays, rng, 0.1, 0.9, bands=bands)


def box_with_n(target: int, seed: int = 0, rays: int = 10_000) -> Instance:
    """Open box 1 x 1 x d with n x n base and walls n x m, N = n^2 + 4 n m >= target."""
    n = max(2, int(math.sqrt(target / 2.0)))
    m = max(1, int(round((target - n * n) / (4.0 * n))))
    model = geo.open_box(1.0, 1.0, m / n, n, n, m)
    return _finish(f"box_n{model.n}", model, rays, rng_for(200, seed), 0.1, 0.9)
