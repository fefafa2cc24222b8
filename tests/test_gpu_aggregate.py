"""GPU parity: rad_aggregate_nodes against the FP64 oracle (thesis Sec. 5.2.3)."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, padded, torch

pytestmark = pytest.mark.gpu
# Same products and sums as the oracle in a different order: ~1e-16 relative.
TOL = 1e-14


def _agg(x, w, grp, g, ld=None):
    import paper_2511_04277_amd as rad
    xd = padded(x, ld) if ld else dev(x)
    y, gw = rad.aggregate_nodes(xd, dev(w), dev(grp, torch.int32), g)
    return host(y), host(gw)


def test_config1_whole_squares():
    need_gpu()
    inst = W.config1()
    y, gw = _agg(inst.f_exact, inst.area, inst.groups[0], 2)
    ref, rw = oracle.aggregate_nodes(inst.f_exact, inst.area, inst.groups[0], 2)
    assert np.abs(y - ref).max() <= TOL and np.abs(gw - rw).max() <= 1e-15


@pytest.mark.parametrize("g", [1, 5, 37, 300])
def test_random_groups(g):
    need_gpu()
    inst = W.box_with_n(500, seed=g)
    n = inst.n
    rng = np.random.default_rng(g)
    grp = rng.integers(0, g, n).astype(np.int32)
    grp[:g] = rng.permutation(g)
    w = inst.area * rng.uniform(0.1, 1.0, n)
    y, gw = _agg(inst.f_noisy, w, grp, g, ld=n + 3)
    ref, rw = oracle.aggregate_nodes(inst.f_noisy, w, grp, g)
    assert np.abs(y - ref).max() <= TOL
    assert np.abs(gw - rw).max() <= 1e-13


def test_identity_and_errors():
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd._lib import RadError
    inst = W.small_box(4, 2, seed=0)
    n = inst.n
    y, _ = _agg(inst.f_noisy, inst.area, np.arange(n, dtype=np.int32), n)
    assert np.abs(y - inst.f_noisy).max() <= 1e-16
    grp = np.zeros(n, dtype=np.int32)  # group 1 empty
    with pytest.raises(RadError):
        rad.aggregate_nodes(dev(inst.f_noisy), dev(inst.area), dev(grp, torch.int32), 2)


def test_two_level_n16384_sampled():
    """Full-size 16384 -> 4096 -> 256 maps of the large open box on the exact F."""
    need_gpu()
    from synth import geometry as geo
    model = geo.open_box(1.0, 1.0, 0.75, 64, 64, 48)
    g1, g2 = W._two_level_groups(model, 2, 4)
    f = model.exact_vf()
    a = model.areas()
    y1, w1 = _agg(f, a, g1, 4096)
    y2, _ = _agg(y1, w1, g2, 256)
    yd, _ = _agg(f, a, g2[g1], 256)
    ref2, _ = oracle.aggregate_nodes(f, a, g2[g1], 256)
    assert np.abs(yd - ref2).max() <= TOL
    assert np.abs(y2 - yd).max() <= TOL
    # closure preserved at both levels (eq. 5.31-5.33)
    assert np.abs(y1.sum(1) - 1).max() < 1e-13 and np.abs(y2.sum(1) - 1).max() < 1e-13
