"""GPU parity: rad_gebhart_ref_adjoint and the autograd Function against the oracle."""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu
SIGMA = 5.67e-8


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("case", ["small", "ragged"])
def test_adjoint_matches_oracle(precision, case):
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.small_box(5, 2, seed=7) if case == "small" else W.box_with_n(300, seed=8)
    n = inst.n
    f, eps, rho = inst.f_noisy, inst.eps[0], inst.rho[0].copy()
    rho[3] = 1e-4  # exercises the direct small-rho form
    g = np.random.default_rng(1).uniform(-1, 1, (n, n + 1))
    print(f"[adjoint] case={case} n={n} precision={precision}", flush=True)
    fd, rd = dev(f), dev(rho)
    bd, fac, _ = rad.gebhart_ref(fd, dev(eps), rd, precision=precision, ir_tol=1e-13)
    ge, gr, lam, st = rad.gebhart_ref_adjoint(fac, fd, rd, bd, dev(g), want_lambda=True, ir_tol=1e-13)
    b = oracle.gebhart_ref(f, eps, rho)
    rge, rgr, rlam = oracle.gebhart_ref_adjoint(f, eps, rho, b, g)
    tol = 1e-11 if precision == "fp64" else 1e-9
    assert _rel(host(lam), rlam) <= tol
    assert _rel(host(ge), rge) <= tol
    assert _rel(host(gr), rgr) <= tol


def test_autograd_function_and_finite_differences():
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.small_box(4, 2, seed=9)
    n = inst.n
    f = dev(inst.f_noisy)
    w = dev(np.random.default_rng(3).uniform(0, 1, (n, n + 1)))
    eps = dev(inst.eps[0]).requires_grad_(True)
    rho = dev(inst.rho[0]).requires_grad_(True)
    b = rad.GebhartREF.apply(f, eps, rho)
    (w * b).sum().backward()
    rge, rgr, _ = oracle.gebhart_ref_adjoint(inst.f_noisy, inst.eps[0], inst.rho[0],
                                              oracle.gebhart_ref(inst.f_noisy, inst.eps[0], inst.rho[0]),
                                              host(w))
    assert _rel(host(eps.grad), rge) < 1e-11 and _rel(host(rho.grad), rgr) < 1e-11
    # central differences through the GPU forward
    h = 1e-6
    wn = host(w)
    for k in (0, n // 2, n - 1):
        for which in ("eps", "rho"):
            e0, r0 = inst.eps[0].copy(), inst.rho[0].copy()
            vals = []
            for sgn in (1, -1):
                e, r = e0.copy(), r0.copy()
                (e if which == "eps" else r)[k] += sgn * h
                bb, _, _ = rad.gebhart_ref(f, dev(e), dev(r))
                vals.append((wn * host(bb)).sum())
            fdv = (vals[0] - vals[1]) / (2 * h)
            ad = host(eps.grad if which == "eps" else rho.grad)[k]
            assert abs(fdv - ad) <= 1e-7 * max(1.0, abs(ad))


def _net_loss_objective(b, eps, area, t_face, t_space=3.0):
    """J = sigma sum_i eps_i A_i [sum_j B_ij (T_i^4 - T_j^4) + B_i,sp (T_i^4 - T_sp^4)]."""
    t4 = t_face ** 4
    n = b.shape[0]
    diff = np.empty((n, n + 1))
    diff[:, :n] = t4[:, None] - t4[None, :]
    diff[:, n] = t4 - t_space ** 4
    coef = SIGMA * eps * area
    return float((coef[:, None] * b * diff).sum()), coef[:, None] * diff


def test_chimney_assembly_n4096_gradient():
    """The 4096-face chimney with 64 node temperatures: adjoint vs oracle and vs FD."""
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.config4()
    n = inst.n
    print(f"[adjoint] chimney n={n}", flush=True)
    fd = dev(inst.f_noisy)
    rad.enforce_vf_(fd, dev(inst.area), dev(inst.n_rays), tol=0.0, max_iter=20)
    f = host(fd)
    eps, rho = inst.eps[0], inst.rho[0]
    t_face = inst.node_temp[inst.groups[0]]
    b = oracle.gebhart_ref(f, eps, rho)
    j0, g = _net_loss_objective(b, eps, inst.area, t_face)
    rge, rgr, _ = oracle.gebhart_ref_adjoint(f, eps, rho, b, g)
    bd, fac, _ = rad.gebhart_ref(fd, dev(eps), dev(rho))
    ge, gr, _, _ = rad.gebhart_ref_adjoint(fac, fd, dev(rho), bd, dev(g))
    assert _rel(host(ge), rge) < 1e-10 and _rel(host(gr), rgr) < 1e-10
    # the same gradients through the int8-emulated solve and transposed solve
    b8, fac8, _ = rad.gebhart_ref(fd, dev(eps), dev(rho), precision="fp64_i8")
    ge8, gr8, _, _ = rad.gebhart_ref_adjoint(fac8, fd, dev(rho), b8, dev(g))
    print(f"[adjoint] chimney fp64_i8 rel err eps={_rel(host(ge8), rge):.2e} rho={_rel(host(gr8), rgr):.2e}",
          flush=True)
    assert _rel(host(ge8), rge) < 1e-10 and _rel(host(gr8), rgr) < 1e-10
    # central differences of J (through B only) on seeded faces, h = 1e-6
    rng = np.random.default_rng(44)
    h = 1e-6
    for k in rng.choice(n, 4, replace=False):
        for which in ("eps", "rho"):
            vals = []
            for sgn in (1, -1):
                e, r = eps.copy(), rho.copy()
                (e if which == "eps" else r)[k] += sgn * h
                bb, _, _ = rad.gebhart_ref(fd, dev(e), dev(r))
                vals.append(float((g * host(bb)).sum()))
            fdv = (vals[0] - vals[1]) / (2 * h)
            ad = (host(ge) if which == "eps" else host(gr))[k]
            # FD of this 16.8M-term J at h = 1e-6 carries ~1e-7 absolute roundoff
            # (solve and sum rounding / 2h); the oracle comparison above is the tight check
            scale = np.abs(host(ge if which == "eps" else gr)).max()
            assert abs(fdv - ad) <= 1e-6 * abs(ad) + 2e-6 * scale


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "fp64_i8"])
def test_non_finite_gradient_is_reported(precision):
    """A NaN in dJ/dB is raised by the adjoint (RAD_ENONFINITE) in every
    precision, also through the autograd Function's backward; an
    out-of-range rho is raised by the Function's forward."""
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd._lib import RadError
    inst = W.small_box(3, 1, seed=4)
    n = inst.n
    fd, ed, rd = dev(inst.f_noisy), dev(inst.eps[0]), dev(inst.rho[0])
    print(f"[adjoint] non-finite G n={n} precision={precision}", flush=True)
    bd, fac, _ = rad.gebhart_ref(fd, ed, rd, precision=precision, ir_tol=1e-13)
    g = np.ones((n, n + 1))
    g[1, 2] = np.nan
    with pytest.raises(RadError) as e:
        rad.gebhart_ref_adjoint(fac, fd, rd, bd, dev(g), ir_tol=1e-13)
    assert e.value.code == -2
    eps = ed.clone().requires_grad_(True)
    rho = rd.clone().requires_grad_(True)
    b = rad.GebhartREF.apply(fd, eps, rho, precision)
    with pytest.raises(RadError):
        (dev(g) * b).sum().backward()
    bad = inst.rho[0].copy()
    bad[0] = 1.5
    with pytest.raises(RadError) as e:
        rad.GebhartREF.apply(fd, ed, dev(bad).requires_grad_(True), precision)
    assert e.value.code == -2
