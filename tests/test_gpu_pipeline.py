"""GPU parity of the chained radiative pipeline against the chained oracle:
noisy F -> enforcement (Sec. 3.5.5) -> REFs (App. B.2) -> REF-level node
aggregation (eq. 5.6-5.7) and absorbed heat fluxes (eq. 4.6) -> steady node
temperatures (eq. 3.12-3.14, GR from REFs eq. 4.2)."""
import numpy as np
import pytest

import oracle
from oracle.steady import SIGMA
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp64_i8"])
def test_enforce_solve_fluxes_temperatures(precision):
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(1100, seed=12)
    n = inst.n
    print(f"[pipeline] n={n} {precision}", flush=True)
    eps, rho = inst.eps[0], inst.rho[0]
    rng = np.random.default_rng(12)
    qd = rng.uniform(0.0, 1400.0, (n, 4))
    # oracle chain
    f_o, info = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-13, max_iter=400)
    b_o = oracle.gebhart_ref(f_o, eps, rho)
    qa_o = oracle.absorbed_flux(b_o, eps, rho, inst.area, qd)
    g1 = np.arange(n) // 4  # runs of four faces per node
    n1 = int(g1.max()) + 1
    y_o, w_o = oracle.aggregate_nodes(b_o, eps * inst.area, g1, n1)
    q_node = np.zeros((n1, 4))
    np.add.at(q_node, g1, qa_o)
    t_o = oracle.steady_temperature(y_o, w_o, q_node, t_space=3.0)
    # GPU chain, every step on the device
    F = dev(inst.f_noisy)
    st = rad.enforce_vf_(F, dev(inst.area), dev(inst.n_rays), kappa="fracvar", tol=1e-13, max_iter=400)
    B, _, _ = rad.gebhart_ref(F, dev(eps), dev(rho), precision=precision)
    Qa = rad.absorbed_flux(B, dev(eps), dev(rho), dev(inst.area), dev(qd))
    Y, Wn = rad.aggregate_nodes(B, dev(eps * inst.area), dev(g1, torch.int32), n1)
    # node heat input: the faces' absorbed power summed per node (test-side
    # bookkeeping on the device result, as on the oracle side)
    qn = np.zeros((n1, 4))
    np.add.at(qn, g1, host(Qa))
    T, _, sst = rad.steady_temperature(Y, Wn, dev(qn), t_space=3.0, precision=precision)
    t = host(T)
    # every intermediate, element by element: the enforced F (same stopping
    # iteration), the REFs, the node REFs and their weights, the fluxes and
    # the temperatures
    tol_b = 1e-12 if precision == "fp64" else 1e-10
    assert st["iters"] == info["iters"] and st["converged"] == 1
    assert np.abs(host(F) - f_o).max() <= 1e-13
    assert np.abs(host(B) - b_o).max() <= tol_b
    assert np.abs(host(Y) - y_o).max() <= tol_b
    assert np.abs(host(Wn) - w_o).max() <= 1e-15 * np.abs(w_o).max()
    assert np.abs(host(Qa) - qa_o).max() <= 1e-10 * np.abs(qa_o).max()
    assert np.abs(t - t_o).max() <= 1e-10 * t_o.max()
