"""GPU parity: rad_absorbed_flux against the FP64 oracle (thesis Sec. 4.2.3, eq. 4.6)."""
import ctypes

import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, padded, torch

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _tol(n):
    """Elementwise relative bound for non-negative data: each side sums n + 1
    non-negative products in FP64 (in different orders), so each is within
    gamma_(n+2) of the exact value; the two differ by at most twice that."""
    return 2.0 * (n + 2) * U / (1.0 - (n + 2) * U)


def _inputs(n, m, seed, b=None):
    rng = np.random.default_rng(seed)
    if b is None:
        # REF-like rows: non-negative, each row summing to about one
        b = rng.uniform(0.0, 2.0 / (n + 1), (n, n + 1))
    eps = rng.uniform(0.05, 0.95, n)
    rho = 1.0 - eps
    area = rng.uniform(0.5, 2.0, n)
    qd = rng.uniform(0.0, 1400.0, (n, m)) if m else rng.uniform(0.0, 1400.0, n)
    return b, eps, rho, area, qd


def _gpu(b, eps, rho, area, qd, ldb=None, ldq=None, lda=None):
    import paper_2511_04277_amd as rad
    B = padded(b, ldb) if ldb else dev(b)
    if qd.ndim == 2 and ldq:
        Q = padded(qd, ldq)
    else:
        Q = dev(qd)
    out = padded(np.zeros(qd.shape), lda) if lda else None
    r = rad.absorbed_flux(B, dev(eps), dev(rho), dev(area), Q, out=out)
    return host(r)


def _check(g, ref, n):
    assert g.shape == ref.shape
    scale = np.maximum(np.abs(ref), 1e-300)
    assert (np.abs(g - ref) / scale).max() <= _tol(n)


@pytest.mark.parametrize("m", [1, 3, 16])
@pytest.mark.parametrize("n", [7, 330, 2300])
def test_matches_oracle(n, m):
    need_gpu()
    print(f"[ahf] n={n} m={m}", flush=True)
    b, eps, rho, area, qd = _inputs(n, m, seed=n * 31 + m)
    _check(_gpu(b, eps, rho, area, qd), oracle.absorbed_flux(b, eps, rho, area, qd), n)


def test_vector_load_case():
    need_gpu()
    b, eps, rho, area, qd = _inputs(513, 0, seed=2)
    g = _gpu(b, eps, rho, area, qd)
    assert g.ndim == 1
    _check(g, oracle.absorbed_flux(b, eps, rho, area, qd), 513)


def test_refs_from_the_gebhart_solve():
    """B from the oracle's Gebhart solve on a ragged box (physical REFs)."""
    need_gpu()
    inst = W.box_with_n(330, seed=4)
    eps, rho = inst.eps[0], inst.rho[0]
    b = oracle.gebhart_ref(inst.f_noisy, eps, rho)
    area = inst.area
    qd = np.random.default_rng(9).uniform(0.0, 1400.0, (inst.n, 5))
    _check(_gpu(b, eps, rho, area, qd), oracle.absorbed_flux(b, eps, rho, area, qd), inst.n)


def test_padded_leading_dimensions():
    need_gpu()
    n, m = 1100, 5
    b, eps, rho, area, qd = _inputs(n, m, seed=7)
    g = _gpu(b, eps, rho, area, qd, ldb=n + 1 + 29, ldq=m + 3, lda=m + 11)
    _check(g, oracle.absorbed_flux(b, eps, rho, area, qd), n)


def test_black_faces_absorb_only_direct_flux():
    """rho = 0: nothing is reflected, Qa = A eps Qd exactly (same product order)."""
    need_gpu()
    n, m = 900, 4
    b, eps, _, area, qd = _inputs(n, m, seed=3)
    rho = np.zeros(n)
    g = _gpu(b, eps, rho, area, qd)
    assert np.array_equal(g, oracle.absorbed_flux(b, eps, rho, area, qd))


def test_full_size_open_box_8192():
    """N = 8192 (the Gebhart workload's size), 16 load cases, every output."""
    need_gpu()
    n, m = 8192, 16
    print(f"[ahf] n={n} m={m}", flush=True)
    b, eps, rho, area, qd = _inputs(n, m, seed=11)
    _check(_gpu(b, eps, rho, area, qd), oracle.absorbed_flux(b, eps, rho, area, qd), n)


def test_bitwise_reproducible():
    need_gpu()
    import paper_2511_04277_amd as rad
    b, eps, rho, area, qd = _inputs(2049, 8, seed=5)
    args = [dev(x) for x in (b, eps, rho, area, qd)]
    r1 = host(rad.absorbed_flux(*args))
    r2 = host(rad.absorbed_flux(*args))
    assert np.array_equal(r1, r2)


def test_invalid_arguments_are_rejected():
    need_gpu()
    from paper_2511_04277_amd import _lib as L
    lib = L.lib()
    n, m = 64, 2
    b, eps, rho, area, qd = _inputs(n, m, seed=1)
    B, E, R, A, Q = (dev(x) for x in (b, eps, rho, area, qd))
    out = torch.empty((n, m), dtype=torch.float64, device="cuda")
    ws = lib.rad_absorbed_flux_workspace_bytes(n, m)
    work = torch.empty(ws, dtype=torch.uint8, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    base = dict(B=p(B), n=n, ldb=n + 1, eps=p(E), rho=p(R), area=p(A), Qd=p(Q), m=m, ldq=m, Qa=p(out), lda=m,
                work=p(work), wb=ws)

    def call(**kw):
        a = dict(base, **kw)
        return lib.rad_absorbed_flux(a["B"], a["n"], a["ldb"], a["eps"], a["rho"], a["area"], a["Qd"], a["m"],
                                     a["ldq"], a["Qa"], a["lda"], a["work"], a["wb"], None)

    assert call() == 0
    torch.cuda.synchronize()
    assert lib.rad_absorbed_flux_workspace_bytes(n, 17) == 0
    assert call(m=17) != 0
    assert call(m=0) != 0
    assert call(ldb=n) != 0
    assert call(lda=m - 1) != 0
    assert call(wb=ws - 8) != 0
    assert call(eps=None) != 0
    torch.cuda.synchronize()
    _check(host(out), oracle.absorbed_flux(b, eps, rho, area, qd), n)
