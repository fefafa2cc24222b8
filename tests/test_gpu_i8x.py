"""GPU parity of RAD_PREC_FP64_I8 (FP64 solves whose panel-width products are
exact int8 digit products, FP64 accumulation) against the FP64 oracle.

The emulated products only run where a panel has rows or columns beyond it,
so the cases have n > 1024 (two to four 1024-wide panels, ragged tails).
Each dropped digit pair and operand tail is below 2^-49 of the row and
column maxima per unit of K; summed over the panel updates and both
substitutions that leaves about 1e-12 on B at these sizes (FP64: 3e-15).
The bound used here, 1e-11 absolute on B and relative on the adjoint, is ten
times inside the 1e-10 target; a row sum of n + 1 such errors (closure) is
held to 1e-10.
"""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, padded, torch

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.mark.parametrize("n", [1025, 1100, 2049, 2300, 3000])
def test_solve_matches_oracle(n):
    """Ragged sizes, including one row past a 1024 panel (a 1-row trailing
    update, padded to one 64-row tile) and one past two panels."""
    need_gpu()
    import paper_2511_04277_amd as rad
    if n in (1025, 2049):  # exact sizes: cut a larger box down to n faces, rows re-closed
        base = W.box_with_n(n + 160, seed=n)
        assert base.n > n
        f = base.f_noisy[:n, list(range(n)) + [base.n]].copy()
        f[:, n] = 1.0 - f[:, :n].sum(1)
        inst = W.Instance(f"n{n}", f, f, base.area[:n], base.n_rays[:n], [base.eps[0][:n]], [base.rho[0][:n]])
    else:
        inst = W.box_with_n(n, seed=n)
    eps, rho = inst.eps[0], inst.rho[0]
    print(f"[i8x] solve n={inst.n}", flush=True)
    bd, _, st = rad.gebhart_ref(dev(inst.f_noisy), dev(eps), dev(rho), precision="fp64_i8")
    ref = oracle.gebhart_ref(inst.f_noisy, eps, rho)
    err = np.abs(host(bd) - ref).max()
    print(f"[i8x] n={inst.n} max|dB|={err:.3e} stats={st}", flush=True)
    assert err <= TOL


def test_padded_leading_dimension():
    """F with ld = n + 7: the emulated products read the factors and
    right-hand sides through the solver's own padded buffers either way."""
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(1500, seed=44)
    eps, rho = inst.eps[0], inst.rho[0]
    fd = padded(inst.f_noisy, inst.n + 7)
    print(f"[i8x] padded ld n={inst.n}", flush=True)
    bd, _, _ = rad.gebhart_ref(fd, dev(eps), dev(rho), precision="fp64_i8")
    err = np.abs(host(bd) - oracle.gebhart_ref(inst.f_noisy, eps, rho)).max()
    assert err <= TOL


def test_invalid_optical_properties():
    need_gpu()
    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd._lib import RadError
    inst = W.box_with_n(1100, seed=45)
    rho = inst.rho[0].copy()
    rho[17] = 1.5
    with pytest.raises(RadError) as e:
        rad.gebhart_ref(dev(inst.f_noisy), dev(inst.eps[0]), dev(rho), precision="fp64_i8")
    assert e.value.code == -2


def test_rho_zero_gives_e_exactly():
    """rho = 0: L = I, so every emulated update adds exact zeros."""
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(2100, seed=5)
    eps = inst.eps[0]
    bd, _, _ = rad.gebhart_ref(dev(inst.f_noisy), dev(eps), dev(np.zeros(inst.n)), precision="fp64_i8")
    _, e = oracle.form_k_e(inst.f_noisy, eps, np.zeros(inst.n))
    assert np.abs(host(bd) - e).max() == 0.0


def test_adjoint_matches_oracle():
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(2300, seed=31)
    n = inst.n
    f, eps, rho = inst.f_noisy, inst.eps[0], inst.rho[0].copy()
    rho[7] = 1e-4  # the direct small-rho form
    g = np.random.default_rng(2).uniform(-1, 1, (n, n + 1))
    print(f"[i8x] adjoint n={n}", flush=True)
    fd, rd = dev(f), dev(rho)
    bd, fac, _ = rad.gebhart_ref(fd, dev(eps), rd, precision="fp64_i8")
    ge, gr, lam, _ = rad.gebhart_ref_adjoint(fac, fd, rd, bd, dev(g), want_lambda=True)
    b = oracle.gebhart_ref(f, eps, rho)
    rge, rgr, rlam = oracle.gebhart_ref_adjoint(f, eps, rho, b, g)

    def rel(a, r):
        return np.abs(a - r).max() / np.abs(r).max()
    print(f"[i8x] adjoint rel err lambda={rel(host(lam), rlam):.2e} eps={rel(host(ge), rge):.2e} "
          f"rho={rel(host(gr), rgr):.2e}", flush=True)
    assert rel(host(lam), rlam) <= TOL and rel(host(ge), rge) <= TOL and rel(host(gr), rgr) <= TOL


def test_ref_checks_and_fp64_agreement():
    """On an enforced F the emulated B keeps closure and reciprocity at
    rounding level and agrees with the FP64 path's B."""
    need_gpu()
    import paper_2511_04277_amd as rad
    inst = W.box_with_n(2200, seed=12)
    fd, area = dev(inst.f_noisy), dev(inst.area)
    rad.enforce_vf_(fd, area, dev(inst.n_rays), tol=1e-14, max_iter=200)
    eps, rho = dev(inst.eps[0]), dev(inst.rho[0])
    b64, _, _ = rad.gebhart_ref(fd, eps, rho, precision="fp64")
    b8, _, _ = rad.gebhart_ref(fd, eps, rho, precision="fp64_i8")
    chk = host(rad.ref_check(b8, eps, area))
    d = torch.max(torch.abs(b8 - b64)).item()
    print(f"[i8x] closure={chk[0]:.2e} reciprocity={chk[1]:.2e} max|B_i8 - B_64|={d:.2e}", flush=True)
    assert d <= TOL and chk[0] < 1e-10 and chk[1] < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_block_sparse_plate_pairs_match_oracle(kind):
    """Two plates (parallel or perpendicular) of about 1150 faces each: the
    faces of one plate see each other with zero view factor, so whole 64 x 64
    blocks of K, of its factors and of the right-hand sides are zero and the
    emulated products skip those tiles (zero row or column exponents), next
    to full tiles and tiles cut by the 1024-wide panels.  B against the
    oracle, and against the FP64 path on the same input."""
    need_gpu()
    import paper_2511_04277_amd as rad
    model = W._mesh_plates(kind, 1.0, 0.6, 2300)
    inst = W._finish(f"plates{kind}", model, 10_000, W.rng_for(300, kind), 0.1, 0.9)
    n = inst.n
    eps, rho = inst.eps[0], inst.rho[0]
    f = inst.f_noisy
    assert n > 2048 and np.all(f[: n // 4, : n // 4] == 0.0)  # a coplanar block
    print(f"[i8x] plates kind={kind} n={n}", flush=True)
    bi, _, _ = rad.gebhart_ref(dev(f), dev(eps), dev(rho), precision="fp64_i8")
    bf, _, _ = rad.gebhart_ref(dev(f), dev(eps), dev(rho), precision="fp64")
    ref = oracle.gebhart_ref(f, eps, rho)
    bi, bf = host(bi), host(bf)
    assert np.abs(bi - ref).max() <= TOL
    assert np.abs(bi - bf).max() <= TOL
