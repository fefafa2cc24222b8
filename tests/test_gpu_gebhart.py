"""GPU parity: rad_gebhart_ref / rad_ref_check against the FP64 oracle (App. B.2)."""
import numpy as np
import pytest

import oracle
from synth import geometry as geo
from synth import workloads as W
from tests.golden.loader import load
from tests.gpu_util import dev, host, need_gpu, padded, torch

pytestmark = pytest.mark.gpu

# FP64 path: a different but backward-stable elimination order (block LDU, no
# pivoting, K diagonally dominant) -> differences of a few ulps times the
# small condition number of K.  FP32+refinement: the target is 1e-10 abs.
TOL64 = 1e-12
TOL_IR = 1e-10


def _solve(f, eps, rho, precision="fp64", ld=None, ir_tol=1e-13):
    import paper_2511_04277_amd as rad
    fd = padded(f, ld) if ld else dev(f)
    b, fac, st = rad.gebhart_ref(fd, dev(eps), dev(rho), precision=precision, ir_tol=ir_tol, ir_max=6)
    return host(b), fac, st


def test_parallel_plates_eq_6_11():
    need_gpu()
    e2 = load("e2_parallel_plates.txt")
    for prec, tol in (("fp64", TOL64), ("fp32_ir", TOL_IR)):
        b, _, st = _solve(e2["F"], e2["eps"], e2["rho"], prec)
        assert np.abs(b - e2["B"]).max() < 1e-6
        assert np.abs(b - oracle.gebhart_ref(e2["F"], e2["eps"], e2["rho"])).max() <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("n_case", ["c1", "n1", "n128", "n129", "ragged"])
def test_matches_oracle(precision, n_case):
    need_gpu()
    if n_case == "c1":
        inst = W.config1()
    elif n_case == "ragged":
        inst = W.box_with_n(330, seed=3)
    elif n_case == "n1":
        inst = W.Instance("one", np.array([[0.3, 0.7]]), np.array([[0.3, 0.7]]), np.ones(1), np.ones(1),
                          [np.array([0.4])], [np.array([0.6])])
    else:
        n = int(n_case[1:])
        base = W.box_with_n(n + 40, seed=5)
        f = base.f_noisy[:n, list(range(n)) + [base.n]].copy()
        f[:, n] = 1.0 - f[:, :n].sum(1)
        inst = W.Instance(n_case, f, f, base.area[:n], base.n_rays[:n], [base.eps[0][:n]], [base.rho[0][:n]])
    print(f"[gebhart] case={n_case} n={inst.n} precision={precision}", flush=True)
    eps, rho = inst.eps[0], inst.rho[0]
    b, _, st = _solve(inst.f_noisy, eps, rho, precision, ld=inst.n + 5)
    ref = oracle.gebhart_ref(inst.f_noisy, eps, rho)
    assert np.abs(b - ref).max() <= (TOL64 if precision == "fp64" else TOL_IR)
    if precision == "fp32_ir":
        assert st["ir_steps"] >= 1 and st["converged"] == 1


def test_rho_zero_gives_e_exactly():
    need_gpu()
    inst = W.small_box(6, 3, seed=1)
    eps = inst.eps[0]
    b, _, _ = _solve(inst.f_noisy, eps, np.zeros(inst.n))
    _, e = oracle.form_k_e(inst.f_noisy, eps, np.zeros(inst.n))
    assert np.abs(b - e).max() == 0.0


def test_ref_checks_on_enforced_input():
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(400, seed=4)
    f, _ = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=1e-15, max_iter=800)
    eps, rho = inst.eps[0], inst.rho[0]
    bd, _, _ = rad.gebhart_ref(dev(f), dev(eps), dev(rho))
    chk = host(rad.ref_check(bd, dev(eps), dev(inst.area)))
    b = host(bd)
    assert abs(chk[0] - oracle.ref_closure_residual(b)) <= 1e-15
    assert abs(chk[1] - oracle.ref_reciprocity_residual(b, eps, inst.area)) <= 1e-17
    assert chk[0] < 1e-13 and chk[1] < 1e-14


def test_singular_closed_system_is_reported():
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd._lib import RadError
    m = geo.open_box(1, 1, 1, 3, 3, 3, open_top=False)  # closed: F_space = 0
    f = m.exact_vf()
    f[:, -1] = 0.0
    n = m.n
    with pytest.raises(RadError) as e:
        rad.gebhart_ref(dev(f), dev(np.zeros(n)), dev(np.ones(n)))  # rho = 1: K 1 = 0
    assert e.value.code == -4


def test_invalid_optical_properties():
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd._lib import RadError
    inst = W.small_box(3, 1, seed=0)
    rho = inst.rho[0].copy()
    rho[2] = 1.5
    with pytest.raises(RadError) as e:
        rad.gebhart_ref(dev(inst.f_noisy), dev(inst.eps[0]), dev(rho))
    assert e.value.code == -2


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "fp64_i8"])
def test_full_size_open_cube_n5120(precision):
    """The 5120-face open cube: enforced on the GPU, then solved; element-wise vs the oracle."""
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.config2()
    print(f"[gebhart] open cube n={inst.n} precision={precision}", flush=True)
    fd = dev(inst.f_noisy)
    rad.enforce_vf_(fd, dev(inst.area), dev(inst.n_rays), tol=0.0, max_iter=30)
    f = host(fd)
    eps, rho = inst.eps[0], inst.rho[0]
    bd, _, st = rad.gebhart_ref(fd, dev(eps), dev(rho), precision=precision, ir_tol=1e-13, ir_max=6)
    ref = oracle.gebhart_ref(f, eps, rho)
    err = np.abs(host(bd) - ref).max()
    print(f"[gebhart] n=5120 {precision} max|dB|={err:.3e} stats={st}", flush=True)
    assert err <= {"fp64": TOL64, "fp32_ir": TOL_IR, "fp64_i8": TOL_IR}[precision]


def test_tuning_knobs_leave_results_bitwise_unchanged():
    """Tile shape, look-ahead and the side update's chunking reorder launches
    only: B and the adjoint's gradients must be identical under every
    setting."""
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd import _lib as L
    inst = W.box_with_n(2300, seed=8)
    fd, eps, rho = dev(inst.f_noisy), dev(inst.eps[0]), dev(inst.rho[0])
    g = dev(np.random.default_rng(3).standard_normal((inst.n, inst.n + 1)))
    saved = L.tuning()
    outs = []
    try:
        for tile, look, chunk in ((0, 1, 0), (4096, 1, 0), (1 << 30, 0, 0), (256, 0, 0), (4096, 1, 512), (0, 1, 100)):
            L.apply_tuning({"small_tile_below_f64": tile, "small_tile_below_f32": tile, "lookahead": look,
                            "side_chunk_tiles": chunk})
            for prec in ("fp64", "fp32_ir", "fp64_i8"):
                b, fac, _ = rad.gebhart_ref(fd, eps, rho, precision=prec, ir_tol=1e-13, ir_max=3)
                ge, gr, _, _ = rad.gebhart_ref_adjoint(fac, fd, rho, b, g)
                outs.append((tile, look, prec, b.clone(), ge.clone(), gr.clone()))
    finally:
        L.apply_tuning(saved)
    for prec in ("fp64", "fp32_ir", "fp64_i8"):
        ref = [o for o in outs if o[2] == prec]
        for o in ref[1:]:
            assert torch.equal(o[3], ref[0][3]) and torch.equal(o[4], ref[0][4]) and torch.equal(o[5], ref[0][5]), o[:3]
