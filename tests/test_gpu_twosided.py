"""GPU parity: two-sided nodes (eq. 5.17 via rad_aggregate_nodes, view
fractions eq. 5.29, node emissivity eq. C.4) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from oracle.twosided import node_emissivity, node_view_factors, view_fractions
from synth import workloads as W
from tests.golden.loader import load
from tests.gpu_util import dev, host, need_gpu, padded, torch

pytestmark = pytest.mark.gpu

# Same quotients of sums taken in different orders: a few ulps.
TOL = 1e-13


def _two_sided(n_target, seed, frac_pairs=3):
    inst = W.box_with_n(n_target, seed=seed)
    nf = inst.n
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nf)
    group = np.empty(nf, dtype=np.int64)
    npair = nf // frac_pairs
    for k in range(npair):
        group[perm[2 * k]] = group[perm[2 * k + 1]] = k
    rest = perm[2 * npair:]
    group[rest] = npair + np.arange(rest.size)
    g = npair + rest.size
    s = rng.uniform(0.5, 2.0, g)[group]
    return inst, group, g, s


def _gi(group):
    return dev(group, torch.int32)


def test_parallel_plates():
    need_gpu()
    import paper_2511_04277_amd as rad
    e2 = load("e2_parallel_plates.txt")
    grp = np.array([0, 0, 1, 1])
    y, _ = rad.aggregate_nodes(dev(e2["F"]), dev(np.ones(4)), _gi(grp), 2)
    fn, _ = node_view_factors(e2["F"], grp, 2)
    assert np.abs(host(y) - fn).max() < 1e-15
    r = host(rad.view_fractions(dev(e2["F"]), _gi(grp), 2))
    assert np.abs(r - view_fractions(e2["F"], grp, 2)).max() <= TOL
    b = oracle.gebhart_ref(e2["F"], e2["eps"], e2["rho"])
    e = host(rad.node_emissivity(dev(b), dev(e2["eps"]), dev(np.ones(4)), _gi(grp), 2))
    assert np.abs(e - 0.5).max() < 1e-15


@pytest.mark.parametrize("pairs", [2, 3])
def test_noisy_box_matches_oracle(pairs):
    need_gpu()
    import paper_2511_04277_amd as rad
    inst, group, g, s = _two_sided(330, seed=pairs, frac_pairs=pairs)
    nf = inst.n
    print(f"[twosided] nf={nf} g={g}", flush=True)
    f = inst.f_noisy
    y, gw = rad.aggregate_nodes(dev(f), dev(s), _gi(group), g)
    fn, c = node_view_factors(f, group, g)
    assert np.abs(host(y) - fn).max() <= TOL
    assert np.abs(host(gw) - np.bincount(group, weights=s, minlength=g)).max() <= 1e-13
    r = host(rad.view_fractions(dev(f), _gi(group), g))
    assert np.abs(r - view_fractions(f, group, g)).max() <= TOL
    rng = np.random.default_rng(pairs)
    eps = rng.uniform(0.1, 0.9, nf)
    b = oracle.gebhart_ref(f, eps, 1.0 - eps)
    e = host(rad.node_emissivity(dev(b), dev(eps), dev(s), _gi(group), g))
    assert np.abs(e - node_emissivity(b, eps, s, group, g)).max() <= TOL


def test_padded_leading_dimensions():
    need_gpu()
    import paper_2511_04277_amd as rad
    inst, group, g, s = _two_sided(200, seed=7)
    nf = inst.n
    f = inst.f_noisy
    out = padded(np.zeros((nf, nf + 1)), nf + 1 + 13)
    r = host(rad.view_fractions(padded(f, nf + 1 + 5), _gi(group), g, out=out))
    assert np.abs(r - view_fractions(f, group, g)).max() <= TOL
    eps = np.random.default_rng(7).uniform(0.1, 0.9, nf)
    b = oracle.gebhart_ref(f, eps, 1.0 - eps)
    eo = padded(np.zeros((g, g + 1)), g + 1 + 3)
    e = host(rad.node_emissivity(padded(b, nf + 1 + 9), dev(eps), dev(s), _gi(group), g, out=eo))
    assert np.abs(e - node_emissivity(b, eps, s, group, g)).max() <= TOL


def test_full_size_8192_faces_4096_two_sided_nodes():
    need_gpu()
    import paper_2511_04277_amd as rad
    nf = 8192
    print(f"[twosided] nf={nf} g={nf // 2}", flush=True)
    inst = W.metric_workload()
    assert inst.n == nf
    rng = np.random.default_rng(11)
    perm = rng.permutation(nf)
    group = np.empty(nf, dtype=np.int64)
    group[perm[0::2]] = np.arange(nf // 2)
    group[perm[1::2]] = np.arange(nf // 2)
    g = nf // 2
    f = inst.f_noisy
    r = host(rad.view_fractions(dev(f), _gi(group), g))
    assert np.abs(r - view_fractions(f, group, g)).max() <= TOL
    del r
    # node emissivity on a REF-like matrix (face REFs at this size come from
    # the GPU solve, which is not an oracle input): eps-weighted rows of F
    eps = inst.eps[0]
    e = host(rad.node_emissivity(dev(f), dev(eps), dev(inst.area), _gi(group), g))
    assert np.abs(e - node_emissivity(f, eps, inst.area, group, g)).max() <= TOL


def test_invalid_groups_and_optics_are_reported():
    need_gpu()
    import paper_2511_04277_amd as rad
    inst, group, g, s = _two_sided(120, seed=9)
    nf = inst.n
    F = dev(inst.f_noisy)
    bad = group.copy()
    bad[4] = g + 3
    with pytest.raises(Exception):
        rad.view_fractions(F, _gi(bad), g)
    empty = group.copy()
    empty[group == g - 1] = 0  # node g-1 left without faces
    with pytest.raises(Exception):
        rad.node_emissivity(F, dev(np.full(nf, 0.5)), dev(s), _gi(empty), g)
    eps = np.full(nf, 0.5)
    eps[3] = 1.5
    with pytest.raises(Exception):
        rad.node_emissivity(F, dev(eps), dev(s), _gi(group), g)
    r = host(rad.view_fractions(F, _gi(group), g))
    assert np.abs(r - view_fractions(inst.f_noisy, group, g)).max() <= TOL
