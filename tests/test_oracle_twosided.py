"""Pins for the oracle's two-sided multi-node relations (Sec. 5.2.4-5.3,
eq. 5.17, 5.29, 5.33, 5.36; App. C, eq. C.2-C.4)."""
import numpy as np

import oracle
from oracle.twosided import node_emissivity, node_view_factors, view_fractions
from synth import workloads as W
from tests.golden.loader import load

E2 = load("e2_parallel_plates.txt")
PLATES = np.array([0, 0, 1, 1])  # faces 1-2: top plate (two sides), 3-4: bottom plate


def test_parallel_plates_node_view_factors():
    """Sec. 6.3 plates as two-sided nodes: the top plate sees the bottom one
    through one face pair only, so F_top,bottom = F_23 / 2 and the rest goes
    to space (eq. 5.17 with C_n = 2 on the view factors of eq. 6.10)."""
    fn, c = node_view_factors(E2["F"], PLATES, 2)
    assert np.array_equal(c, [2.0, 2.0])
    f = E2["F"]
    assert abs(fn[0, 1] - f[1, 2] / 2) < 1e-15 and fn[0, 0] == 0.0
    assert abs(fn[0, 2] - (f[0, 4] + f[1, 4]) / 2) < 1e-15
    assert abs(fn[1, 0] - f[2, 1] / 2) < 1e-15
    assert np.abs(fn.sum(axis=1) - 1.0).max() < 1e-15  # eq. 5.33


def _two_sided(seed, n_target=120):
    """A noisy box whose faces are paired into two-sided nodes (both faces of
    a node carry the node's area), some nodes left one-sided."""
    inst = W.box_with_n(n_target, seed=seed)
    nf = inst.n
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nf)
    group = np.empty(nf, dtype=np.int64)
    npair = nf // 3
    for k in range(npair):
        group[perm[2 * k]] = group[perm[2 * k + 1]] = k
    rest = perm[2 * npair:]
    group[rest] = npair + np.arange(rest.size)
    g = npair + rest.size
    s_node = rng.uniform(0.5, 2.0, g)
    return inst, group, g, s_node[group]


def test_closure_and_reciprocity_preserved():
    """Eq. 5.33 and 5.36: closed, reciprocal face factors (with equal face
    areas per node) give closed node factors, reciprocal with the node area
    C_n S_n."""
    inst, group, g, s = _two_sided(1)
    f, _ = oracle.enforce_vf(inst.f_noisy, s, inst.n_rays, "fracvar", tol=1e-15, max_iter=2000)
    fn, c = node_view_factors(f, group, g)
    assert np.abs(fn.sum(axis=1) - 1.0).max() < 1e-13
    a_node = c * np.bincount(group, weights=s, minlength=g) / c  # C_n S_n
    gr = a_node[:, None] * fn[:, :g]
    assert np.abs(gr - gr.T).max() < 1e-12 * gr.max()


def test_node_factors_are_the_area_weighted_aggregation():
    inst, group, g, s = _two_sided(2)
    fn, _ = node_view_factors(inst.f_noisy, group, g)
    y, _ = oracle.aggregate_nodes(inst.f_noisy, s, group, g)
    assert np.abs(fn - y).max() < 1e-14


def test_view_fractions_partition_and_rebuild():
    """Eq. 5.29: the fractions of a node pair sum to one over its face
    pairs, and C_n F_ij f^{X->Y} gives back every face factor."""
    inst, group, g, _ = _two_sided(3)
    f = inst.f_noisy
    nf = f.shape[0]
    fr = view_fractions(f, group, g)
    fn, c = node_view_factors(f, group, g)
    cols = np.append(group, g)
    rebuilt = (c[group][:, None] * fn[group][:, cols]) * fr
    assert np.abs(rebuilt - f).max() < 1e-15
    sums = np.zeros((g, g + 1))
    for a in range(nf):
        for b in range(nf + 1):
            sums[group[a], cols[b]] += fr[a, b]
    nz = fn > 0
    assert np.abs(sums[nz] - 1.0).max() < 1e-13 and np.all(sums[~nz] == 0.0)
    # one-sided nodes alone with one-sided nodes: each face pair is the whole pair
    single = np.bincount(group, minlength=g)[group] == 1
    ss = np.ix_(single, np.append(single, True))
    assert np.all((fr[ss] == 1.0) | (f[ss] == 0.0))


def test_node_emissivity_reproduces_the_face_couplings():
    """Eq. C.3: eps_ij C_i S_i B_ij, with B_ij the node REF of eq. 5.17,
    equals the sum over face pairs of eps^X S B^{X->Y}; equal face
    emissivities give that emissivity for every pair; mixed ones stay
    between the two."""
    inst, group, g, s = _two_sided(4)
    rng = np.random.default_rng(4)
    eps = rng.uniform(0.1, 0.9, inst.n)
    b = oracle.gebhart_ref(inst.f_noisy, eps, 1.0 - eps)
    e = node_emissivity(b, eps, s, group, g)
    bn, c = node_view_factors(b, group, g)
    s_node = np.bincount(group, weights=s, minlength=g) / c
    gr_node = e * (c * s_node)[:, None] * bn
    p = np.zeros((inst.n, g))
    p[np.arange(inst.n), group] = 1.0
    gr_face = np.zeros((g, g + 1))
    gr_face[:, :g] = p.T @ ((eps * s)[:, None] * b[:, :inst.n]) @ p
    gr_face[:, g] = p.T @ (eps * s * b[:, inst.n])
    assert np.abs(gr_node - gr_face).max() <= 1e-13 * gr_face.max()
    lo = np.array([eps[group == k].min() for k in range(g)])
    hi = np.array([eps[group == k].max() for k in range(g)])
    assert np.all(e >= lo[:, None] - 1e-15) and np.all(e <= hi[:, None] + 1e-15)
    flat = node_emissivity(b, np.full(inst.n, 0.37), s, group, g)
    assert np.abs(flat - 0.37).max() < 1e-15
