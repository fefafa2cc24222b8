"""Axis-aligned rectangular geometry and closed-form view factors.

Synthetic-input layer only: it builds the *exact* view-factor matrices of the
seeded test geometries (open boxes, plate pairs, chimney-like assemblies) from
the classical closed-form expressions for rectangles, and holds none of the
enforcement, Gebhart or aggregation arithmetic.

View factor definition: the double area integral of cos(t_i) cos(t_j) / (pi r^2)
(thesis, Sec. 2.4.12, Def. 34, eq. 2.68).  For axis-aligned rectangles the
integral has closed forms:

* two parallel, directly facing, axis-aligned rectangles separated by ``c``:
  the four-fold corner sum of

      G = 1/(2 pi) [ (y - eta) P atan((y - eta)/P) + (x - xi) Q atan((x - xi)/Q)
                     - c^2/2 ln((x - xi)^2 + (y - eta)^2 + c^2) ],
      P = sqrt((x - xi)^2 + c^2),  Q = sqrt((y - eta)^2 + c^2)

  (Howell's catalogue, configuration C-11; Ehlert & Smith, J. Thermophys.
  Heat Transf. 7(1), 1993);

* two rectangles in perpendicular planes with a common axis ``x``: with ``y``
  the distance of a point of rectangle 1 from the plane of rectangle 2 and
  ``eta`` the distance of a point of rectangle 2 from the plane of rectangle 1,

      G = 1/(2 pi) [ (x - xi) S atan((x - xi)/S)
                     - 1/4 (S^2 - (x - xi)^2) ln((x - xi)^2 + S^2) ],
      S = sqrt(y^2 + eta^2)

  (Howell's catalogue, configuration C-14/C-15; Ehlert & Smith 1993).

In both cases A_1 F_12 = sum over corners (-1)^(i+j+k+l) G(x_i, y_j, xi_k, eta_l).
The expressions are checked against brute-force quadrature of eq. 2.68 and
against the textbook unit-square values in ``tests/test_synth.py``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

_TWO_PI = 2.0 * math.pi


def _xlogx_safe(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a * ln(b) with the continuous limit 0 where b == 0 (a -> 0 there)."""
    out = np.zeros(np.broadcast(a, b).shape)
    mask = b > 0.0
    np.multiply(np.broadcast_to(a, out.shape), np.log(np.where(mask, b, 1.0)), out=out, where=mask)
    return out


def _x_atan_safe(x: np.ndarray, s: np.ndarray) -> np.ndarray:
    """x * s * atan(x / s) with the limit 0 as s -> 0."""
    s_safe = np.where(s > 0.0, s, 1.0)
    return np.where(s > 0.0, x * s * np.arctan(x / s_safe), 0.0)


def _g_parallel(dx, dy, c):
    p = np.sqrt(dx * dx + c * c)
    q = np.sqrt(dy * dy + c * c)
    t = _x_atan_safe(dy, p) + _x_atan_safe(dx, q)
    t = t - 0.5 * c * c * _xlogx_safe(np.ones_like(t), dx * dx + dy * dy + c * c)
    return t / _TWO_PI


def _g_perpendicular(dx, y, eta):
    s2 = y * y + eta * eta
    s = np.sqrt(s2)
    r2 = dx * dx + s2
    t = _x_atan_safe(dx, s) - 0.25 * _xlogx_safe(s2 - dx * dx, r2)
    return t / _TWO_PI


def parallel_vf(x1, x2, y1, y2, xi1, xi2, eta1, eta2, c) -> np.ndarray:
    """F_{1->2} between facing parallel rectangles (broadcasting arrays).

    Rectangle 1: x in [x1, x2], y in [y1, y2] in the plane z = 0.
    Rectangle 2: x in [xi1, xi2], y in [eta1, eta2] in the plane z = c (c > 0).
    """
    xs = (np.asarray(x1, float), np.asarray(x2, float))
    ys = (np.asarray(y1, float), np.asarray(y2, float))
    xis = (np.asarray(xi1, float), np.asarray(xi2, float))
    etas = (np.asarray(eta1, float), np.asarray(eta2, float))
    c = np.asarray(c, float)
    acc = 0.0
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    sign = -1.0 if (i + j + k + l) % 2 else 1.0
                    acc = acc + sign * _g_parallel(xs[i] - xis[k], ys[j] - etas[l], c)
    area = (xs[1] - xs[0]) * (ys[1] - ys[0])
    return acc / area


def perpendicular_vf(x1, x2, y1, y2, xi1, xi2, eta1, eta2) -> np.ndarray:
    """F_{1->2} between rectangles in perpendicular planes sharing the x axis.

    Rectangle 1: x in [x1, x2], distance from the plane of rectangle 2 in [y1, y2].
    Rectangle 2: x in [xi1, xi2], distance from the plane of rectangle 1 in [eta1, eta2].
    Both distances are non-negative (each rectangle lies in front of the other).
    """
    xs = (np.asarray(x1, float), np.asarray(x2, float))
    ys = (np.asarray(y1, float), np.asarray(y2, float))
    xis = (np.asarray(xi1, float), np.asarray(xi2, float))
    etas = (np.asarray(eta1, float), np.asarray(eta2, float))
    acc = 0.0
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    sign = -1.0 if (i + j + k + l) % 2 else 1.0
                    acc = acc + sign * _g_perpendicular(xs[i] - xis[k], ys[j], etas[l])
    area = (xs[1] - xs[0]) * (ys[1] - ys[0])
    return acc / area


@dataclasses.dataclass
class Wall:
    """A uniformly meshed, one-sided, axis-aligned rectangle.

    ``ax`` is the normal axis (0, 1, 2), ``pos`` the plane coordinate and
    ``sgn`` (+1/-1) the direction of the emitting side.  The two in-plane axes
    are taken in increasing order (a0 < a1); cell (i0, i1) spans
    [o0 + i0 h0, o0 + (i0+1) h0] x [o1 + i1 h1, o1 + (i1+1) h1] and has the
    flat index i0 * n1 + i1.
    """

    ax: int
    pos: float
    sgn: int
    o0: float
    h0: float
    n0: int
    o1: float
    h1: float
    n1: int
    name: str = ""

    @property
    def axes(self):
        return tuple(a for a in range(3) if a != self.ax)

    @property
    def n(self) -> int:
        return self.n0 * self.n1

    def cell_area(self) -> float:
        return self.h0 * self.h1

    def lo_hi(self, axis: int):
        """Per-cell [lo, hi] along an in-plane axis, flattened (n,) arrays."""
        a0, a1 = self.axes
        i0, i1 = np.meshgrid(np.arange(self.n0), np.arange(self.n1), indexing="ij")
        if axis == a0:
            lo = self.o0 + i0.ravel() * self.h0
            return lo, lo + self.h0
        if axis == a1:
            lo = self.o1 + i1.ravel() * self.h1
            return lo, lo + self.h1
        raise ValueError("axis is the wall normal")

    def grid_index(self, axis: int) -> np.ndarray:
        a0, a1 = self.axes
        i0, i1 = np.meshgrid(np.arange(self.n0), np.arange(self.n1), indexing="ij")
        return (i0 if axis == a0 else i1).ravel()

    def step(self, axis: int) -> float:
        return self.h0 if axis == self.axes[0] else self.h1

    def count(self, axis: int) -> int:
        return self.n0 if axis == self.axes[0] else self.n1

    def origin(self, axis: int) -> float:
        return self.o0 if axis == self.axes[0] else self.o1

    def extent(self, axis: int):
        return self.origin(axis), self.origin(axis) + self.count(axis) * self.step(axis)


def _same_grid(p: Wall, q: Wall, axis: int) -> bool:
    return math.isclose(p.step(axis), q.step(axis), rel_tol=0, abs_tol=1e-15)


def _block_parallel(p: Wall, q: Wall) -> np.ndarray:
    c = abs(q.pos - p.pos)
    a0, a1 = p.axes
    if _same_grid(p, q, a0) and _same_grid(p, q, a1):
        # F depends only on the integer grid offsets: evaluate once per offset.
        d0 = np.arange(-(q.n0 - 1), p.n0)
        d1 = np.arange(-(q.n1 - 1), p.n1)
        base0 = p.o0 - q.o0
        base1 = p.o1 - q.o1
        x1 = base0 + d0[:, None] * p.h0
        y1 = base1 + d1[None, :] * p.h1
        v = parallel_vf(x1, x1 + p.h0, y1, y1 + p.h1, 0.0, q.h0, 0.0, q.h1, c)
        pi0 = p.grid_index(a0)
        pi1 = p.grid_index(a1)
        qi0 = q.grid_index(a0)
        qi1 = q.grid_index(a1)
        return v[(pi0[:, None] - qi0[None, :]) + (q.n0 - 1), (pi1[:, None] - qi1[None, :]) + (q.n1 - 1)]
    px0, px1 = p.lo_hi(a0)
    py0, py1 = p.lo_hi(a1)
    qx0, qx1 = q.lo_hi(a0)
    qy0, qy1 = q.lo_hi(a1)
    return parallel_vf(px0[:, None], px1[:, None], py0[:, None], py1[:, None],
                       qx0[None, :], qx1[None, :], qy0[None, :], qy1[None, :], c)


def _block_perpendicular(p: Wall, q: Wall) -> np.ndarray:
    a, b = p.ax, q.ax
    cax = 3 - a - b
    # distance of p's cells from q's plane (along b), and of q's cells from p's plane (along a)
    pb0, pb1 = p.lo_hi(b)
    py0 = (pb0 - q.pos) * q.sgn
    py1 = (pb1 - q.pos) * q.sgn
    qa0, qa1 = q.lo_hi(a)
    qz0 = (qa0 - p.pos) * p.sgn
    qz1 = (qa1 - p.pos) * p.sgn
    ylo, yhi = np.minimum(py0, py1), np.maximum(py0, py1)
    zlo, zhi = np.minimum(qz0, qz1), np.maximum(qz0, qz1)
    if ylo.min() < -1e-12 or zlo.min() < -1e-12:
        # a cell behind the other plane: these geometries never need partial visibility
        if yhi.max() <= 1e-12 or zhi.max() <= 1e-12:
            return np.zeros((p.n, q.n))
        raise ValueError(f"walls {p.name}/{q.name} straddle each other's planes")
    ylo = np.maximum(ylo, 0.0)
    zlo = np.maximum(zlo, 0.0)
    if _same_grid(p, q, cax):
        dc = np.arange(-(q.count(cax) - 1), p.count(cax))
        x1 = (p.origin(cax) - q.origin(cax)) + dc * p.step(cax)
        pj = p.grid_index(b)
        qk = q.grid_index(a)
        # unique distance rows / columns
        ny = p.count(b)
        nz = q.count(a)
        yl = np.empty(ny)
        yh = np.empty(ny)
        yl[pj] = ylo
        yh[pj] = yhi
        zl = np.empty(nz)
        zh = np.empty(nz)
        zl[qk] = zlo
        zh[qk] = zhi
        v = perpendicular_vf(x1[:, None, None], x1[:, None, None] + p.step(cax),
                             yl[None, :, None], yh[None, :, None],
                             0.0, q.step(cax), zl[None, None, :], zh[None, None, :])
        pc = p.grid_index(cax)
        qc = q.grid_index(cax)
        return v[(pc[:, None] - qc[None, :]) + (q.count(cax) - 1), pj[:, None], qk[None, :]]
    pc0, pc1 = p.lo_hi(cax)
    qc0, qc1 = q.lo_hi(cax)
    return perpendicular_vf(pc0[:, None], pc1[:, None], ylo[:, None], yhi[:, None],
                            qc0[None, :], qc1[None, :], zlo[None, :], zhi[None, :])


def wall_block(p: Wall, q: Wall) -> np.ndarray:
    """Exact view factors from every cell of ``p`` to every cell of ``q``."""
    if p is q:
        return np.zeros((p.n, q.n))
    if p.ax == q.ax:
        gap = (q.pos - p.pos) * p.sgn
        if gap <= 0.0 or q.sgn != -p.sgn:
            return np.zeros((p.n, q.n))
        # overlapping in-plane extents are required for any exchange; disjoint
        # rectangles still exchange, the formula covers offsets.
        return _block_parallel(p, q)
    # perpendicular: visible iff each lies in the other's front half-space
    return _block_perpendicular(p, q)


@dataclasses.dataclass
class Model:
    """A set of walls whose cells are the faces of an open N-face model."""

    walls: List[Wall]

    @property
    def n(self) -> int:
        return sum(w.n for w in self.walls)

    def offsets(self) -> np.ndarray:
        return np.cumsum([0] + [w.n for w in self.walls])

    def areas(self) -> np.ndarray:
        return np.concatenate([np.full(w.n, w.cell_area()) for w in self.walls])

    def exact_vf(self) -> np.ndarray:
        """Open-system N x (N+1) matrix, last column = view factor to space."""
        n = self.n
        off = self.offsets()
        f = np.zeros((n, n + 1))
        for a, p in enumerate(self.walls):
            for b, q in enumerate(self.walls):
                f[off[a]:off[a + 1], off[b]:off[b + 1]] = wall_block(p, q)
        row = f[:, :n].sum(axis=1)
        if row.max() > 1.0 + 1e-9:
            raise ValueError(f"row sum exceeds 1: {row.max()}")
        f[:, n] = np.clip(1.0 - row, 0.0, None)
        return f


def open_box(lx: float, ly: float, lz: float, nx: int, ny: int, nz: int,
             open_top: bool = True) -> Model:
    """Inward-facing walls of the box [0,lx]x[0,ly]x[0,lz] (top z=lz open).

    Every dimension has one cell size shared by all walls (h = l / n).
    Wall order: base (z=0), x=0, x=lx, y=0, y=ly[, top].
    """
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    walls = [
        Wall(2, 0.0, +1, 0.0, hx, nx, 0.0, hy, ny, "base"),
        Wall(0, 0.0, +1, 0.0, hy, ny, 0.0, hz, nz, "x0"),
        Wall(0, lx, -1, 0.0, hy, ny, 0.0, hz, nz, "x1"),
        Wall(1, 0.0, +1, 0.0, hx, nx, 0.0, hz, nz, "y0"),
        Wall(1, ly, -1, 0.0, hx, nx, 0.0, hz, nz, "y1"),
    ]
    if not open_top:
        walls.append(Wall(2, lz, -1, 0.0, hx, nx, 0.0, hy, ny, "top"))
    return Model(walls)


def square_pair(side: float, gap: float, n: int) -> Model:
    """Two coaxial parallel squares facing each other, each meshed n x n."""
    h = side / n
    return Model([
        Wall(2, 0.0, +1, 0.0, h, n, 0.0, h, n, "bottom"),
        Wall(2, gap, -1, 0.0, h, n, 0.0, h, n, "top"),
    ])


def plate_pair_perpendicular(l1: float, l2: float, width: float, gap: float,
                             n1: int, n2: int, nw: int) -> Model:
    """Plate 1 on z=0 (x in [gap, gap+l1]) and plate 2 on x=0 (z in [gap, gap+l2]).

    Both plates span y in [0, width] and face the quadrant x > 0, z > 0; their
    common axis is y and ``gap`` is each plate's distance from the hinge line.
    """
    hw = width / nw
    return Model([
        Wall(2, 0.0, +1, gap, l1 / n1, n1, 0.0, hw, nw, "plate_z"),
        Wall(0, 0.0, +1, 0.0, hw, nw, gap, l2 / n2, n2, "plate_x"),
    ])


def chimney(box_n: int, panel_nw: int, panel_nh: int, panel_height: float = 2.0) -> Model:
    """Unit open box plus two panels continuing the walls x=0 and x=1 upward.

    The panels (1 m wide along y, ``panel_height`` tall) are hinged on the top
    edges of the two opposite walls and stand vertical; every face lies on
    the boundary of the convex region [0,1]x[0,1]x[0,1+panel_height], so no
    face occludes another.
    """
    box = open_box(1.0, 1.0, 1.0, box_n, box_n, box_n)
    hy = 1.0 / panel_nw
    hz = panel_height / panel_nh
    box.walls.append(Wall(0, 0.0, +1, 0.0, hy, panel_nw, 1.0, hz, panel_nh, "panel_x0"))
    box.walls.append(Wall(0, 1.0, -1, 0.0, hy, panel_nw, 1.0, hz, panel_nh, "panel_x1"))
    return box


def block_groups(model: Model, bs: Sequence[int]) -> np.ndarray:
    """Group id per face: cells of each wall tiled into bs[w] x bs[w] blocks.

    ``bs`` may be one int for all walls.  Group ids are contiguous per wall and
    row-major over blocks inside a wall.
    """
    if isinstance(bs, int):
        bs = [bs] * len(model.walls)
    out = []
    base = 0
    for w, b in zip(model.walls, bs):
        if w.n0 % b or w.n1 % b:
            raise ValueError(f"wall {w.name} ({w.n0}x{w.n1}) not divisible by {b}")
        i0, i1 = np.meshgrid(np.arange(w.n0), np.arange(w.n1), indexing="ij")
        g = (i0 // b) * (w.n1 // b) + (i1 // b)
        out.append(base + g.ravel())
        base += (w.n0 // b) * (w.n1 // b)
    return np.concatenate(out).astype(np.int32)
