"""PyTorch-facing wrappers of the C ABI (include/rad.h).

Torch supplies device memory and the current HIP stream; every step of the
computation runs in librad's HIP kernels.  Matrices are float64 CUDA tensors
of shape (N, N+1) whose rows may be padded (``stride(0) >= N+1``,
``stride(1) == 1``).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _lib as L

_KAPPA = {"fracvar": L.RAD_KAPPA_FRACVAR, "half": L.RAD_KAPPA_HALF}
_PREC = {"fp64": L.RAD_PREC_FP64, "fp32_ir": L.RAD_PREC_FP32_IR, "fp64_i8": L.RAD_PREC_FP64_I8}


def _vp(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _mat(t: torch.Tensor, name: str, rows: Optional[int] = None, cols: Optional[int] = None) -> int:
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
        raise ValueError(f"{name}: expected a 2-D float64 CUDA tensor with unit column stride")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name}: expected {rows} rows, got {t.shape[0]}")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name}: expected {cols} columns, got {t.shape[1]}")
    return t.stride(0) if t.shape[0] > 1 else max(t.stride(0), t.shape[1])


def _vec(t: Optional[torch.Tensor], name: str, n: int, dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.dim() == 1 and t.shape[0] == n and t.is_contiguous()):
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA vector of length {n}")
    return t


class _Workspace:
    """Per-device, per-stream scratch buffers, grown on demand and reused
    across calls (calls on different streams may run concurrently, so they
    never share one)."""

    def __init__(self):
        self._bufs = {}

    def get(self, device: torch.device, key: str, nbytes: int) -> torch.Tensor:
        k = (device.index, torch.cuda.current_stream(device).cuda_stream, key)
        buf = self._bufs.get(k)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
            self._bufs[k] = buf
        return buf


WORKSPACE = _Workspace()


def enforce_vf_(F: torch.Tensor, area: torch.Tensor, n_rays: Optional[torch.Tensor] = None,
                kappa: str = "fracvar", tol: float = 0.0, max_iter: int = 100,
                want_stats: bool = True) -> dict:
    """In-place iterative closure + reciprocity enforcement (Sec. 3.5.5)."""
    n = F.shape[0]
    ld = _mat(F, "F", n, n + 1)
    _vec(area, "area", n)
    _vec(n_rays, "n_rays", n)
    lib = L.lib()
    wb = lib.rad_enforce_workspace_bytes(n)
    work = WORKSPACE.get(F.device, "enforce", wb)
    st = L.RadStats()
    code = lib.rad_enforce_vf(_vp(F), n, ld, _vp(area), _vp(n_rays), _KAPPA[kappa], float(tol),
                              int(max_iter), _vp(work), work.numel(),
                              ctypes.byref(st) if want_stats else None, _stream(F.device))
    L.check(code, "rad_enforce_vf")
    out = st.as_dict() if want_stats else {}
    out["status"] = code
    return out


def aggregate_nodes(X: torch.Tensor, weight: torch.Tensor, group: torch.Tensor, g: int,
                    out: Optional[torch.Tensor] = None, validate: bool = True) -> Tuple[torch.Tensor, torch.Tensor]:
    """Y_GH = sum_{i in G, j in H} w_i X_ij / W_G (eq. 5.6-5.7); returns (Y, W)."""
    n = X.shape[0]
    ldx = _mat(X, "X", n, n + 1)
    _vec(weight, "weight", n)
    _vec(group, "group", n, torch.int32)
    if out is None:
        out = torch.empty((g, g + 1), dtype=torch.float64, device=X.device)
    ldy = _mat(out, "Y", g, g + 1)
    gw = torch.empty(g, dtype=torch.float64, device=X.device)
    lib = L.lib()
    wb = lib.rad_aggregate_workspace_bytes(n, g)
    work = WORKSPACE.get(X.device, "aggregate", wb)
    st = L.RadStats()
    code = lib.rad_aggregate_nodes(_vp(X), n, ldx, _vp(weight), _vp(group), int(g), _vp(out), ldy,
                                   _vp(gw), _vp(work), work.numel(),
                                   ctypes.byref(st) if validate else None, _stream(X.device))
    L.check(code, "rad_aggregate_nodes")
    return out, gw


def absorbed_flux(B: torch.Tensor, eps: torch.Tensor, rho: torch.Tensor, area: torch.Tensor, Qd: torch.Tensor,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Absorbed heat fluxes (eq. 4.6): Qa = diag(A eps) Qd + B_sq^T diag(A rho) Qd.

    Qd: direct heat flux per unit area, n values or n x m load cases (m <= 16);
    returns the absorbed power with the same shape.
    """
    n = B.shape[0]
    ldb = _mat(B, "B", n, n + 1)
    for v, nm in ((eps, "eps"), (rho, "rho"), (area, "area")):
        _vec(v, nm, n)
    vec = Qd.dim() == 1
    q = Qd.unsqueeze(1) if vec else Qd
    m = q.shape[1]
    ldq = _mat(q, "Qd", n, m)
    if out is None:
        out = torch.empty((n, m), dtype=torch.float64, device=B.device)
    o = out.unsqueeze(1) if out.dim() == 1 else out
    lda = _mat(o, "Qa", n, m)
    lib = L.lib()
    work = WORKSPACE.get(B.device, "ahf", lib.rad_absorbed_flux_workspace_bytes(n, m))
    code = lib.rad_absorbed_flux(_vp(B), n, ldb, _vp(eps), _vp(rho), _vp(area), _vp(q), m, ldq, _vp(o), lda,
                                 _vp(work), work.numel(), _stream(B.device))
    L.check(code, "rad_absorbed_flux")
    return out[:, 0] if (vec and out.dim() == 2) else out


def enforce_lsq(F: torch.Tensor, area: torch.Tensor, nnr: bool = True, spva: bool = True, max_rounds: int = 50,
                precision: str = "fp64", factors: Optional["Factors"] = None, out: Optional[torch.Tensor] = None):
    """Least-squares optimum closure + reciprocity enforcement (eq. 3.41-3.52) with
    NNR / SPVA (App. A).  Returns (F_hat, factors, stats); F is not modified."""
    n = F.shape[0]
    ldf = _mat(F, "F", n, n + 1)
    _vec(area, "area", n)
    if out is None:
        out = torch.empty((n, n + 1), dtype=torch.float64, device=F.device)
    ldo = _mat(out, "Fout", n, n + 1)
    if factors is None or factors.n != n or factors.precision != precision:
        factors = Factors(n, precision, F.device)
    lib = L.lib()
    p = _PREC[precision]
    work = WORKSPACE.get(F.device, "lsq", lib.rad_enforce_lsq_workspace_bytes(n, p))
    st = L.RadStats()
    flags = (L.RAD_LSQ_NNR if nnr else 0) | (L.RAD_LSQ_SPVA if spva else 0)
    code = lib.rad_enforce_lsq(_vp(F), n, ldf, _vp(area), _vp(out), ldo, flags, int(max_rounds), p,
                               _vp(factors.buf), factors.buf.numel(), _vp(work), work.numel(), ctypes.byref(st),
                               _stream(F.device))
    L.check(code, "rad_enforce_lsq")
    stats = st.as_dict()
    stats["status"] = code
    return out, factors, stats


def view_fractions(F: torch.Tensor, group: torch.Tensor, g: int, out: Optional[torch.Tensor] = None,
                   validate: bool = True) -> torch.Tensor:
    """View fractions of two-sided nodes (eq. 5.29): each face pair's share of its node pair's total."""
    nf = F.shape[0]
    ldf = _mat(F, "F", nf, nf + 1)
    _vec(group, "group", nf, torch.int32)
    if out is None:
        out = torch.empty((nf, nf + 1), dtype=torch.float64, device=F.device)
    ldr = _mat(out, "R", nf, nf + 1)
    lib = L.lib()
    work = WORKSPACE.get(F.device, "vfrac", lib.rad_view_fractions_workspace_bytes(nf, g))
    st = L.RadStats()
    code = lib.rad_view_fractions(_vp(F), nf, ldf, _vp(group), g, _vp(out), ldr, _vp(work), work.numel(),
                                  ctypes.byref(st) if validate else None, _stream(F.device))
    L.check(code, "rad_view_fractions")
    return out


def node_emissivity(B: torch.Tensor, eps: torch.Tensor, area: torch.Tensor, group: torch.Tensor, g: int,
                    out: Optional[torch.Tensor] = None, validate: bool = True) -> torch.Tensor:
    """Pair-dependent emissivity of two-sided nodes (App. C, eq. C.4), g x (g+1)."""
    nf = B.shape[0]
    ldb = _mat(B, "B", nf, nf + 1)
    _vec(eps, "eps", nf)
    _vec(area, "area", nf)
    _vec(group, "group", nf, torch.int32)
    if out is None:
        out = torch.empty((g, g + 1), dtype=torch.float64, device=B.device)
    lde = _mat(out, "E", g, g + 1)
    lib = L.lib()
    work = WORKSPACE.get(B.device, "nodeeps", lib.rad_node_emissivity_workspace_bytes(nf, g))
    st = L.RadStats()
    code = lib.rad_node_emissivity(_vp(B), nf, ldb, _vp(eps), _vp(area), _vp(group), g, _vp(out), lde, _vp(work),
                                   work.numel(), ctypes.byref(st) if validate else None, _stream(B.device))
    L.check(code, "rad_node_emissivity")
    return out


SIGMA = 5.670374419e-8  # Stefan-Boltzmann constant, W m^-2 K^-4


def steady_temperature(Y: torch.Tensor, weight: torch.Tensor, Q: torch.Tensor,
                       t_fixed: Optional[torch.Tensor] = None, t_space: float = 3.0, sigma: float = SIGMA,
                       precision: str = "fp64", factors: Optional["Factors"] = None,
                       out: Optional[torch.Tensor] = None, want_stats: bool = True):
    """Radiation-only steady node temperatures (eq. 3.12-3.14, GR = sigma w Y, eq. 4.2).

    Y: n x (n+1) REFs (face or node level); weight: eps A per node; Q: heat
    input in W, n values or n x m load cases; t_fixed: n values, > 0 holds a
    node at that temperature, 0 leaves it free.  Returns (T, factors, stats)
    with T shaped like Q.
    """
    n = Y.shape[0]
    ldy = _mat(Y, "Y", n, n + 1)
    _vec(weight, "weight", n)
    _vec(t_fixed, "t_fixed", n)
    vec = Q.dim() == 1
    q = Q.unsqueeze(1) if vec else Q
    m = q.shape[1]
    ldq = _mat(q, "Q", n, m)
    if out is None:
        out = torch.empty((n, m), dtype=torch.float64, device=Y.device)
    o = out.unsqueeze(1) if out.dim() == 1 else out
    ldt = _mat(o, "T", n, m)
    if factors is None or factors.n != n or factors.precision != precision:
        factors = Factors(n, precision, Y.device)
    lib = L.lib()
    p = _PREC[precision]
    work = WORKSPACE.get(Y.device, "steady", lib.rad_steady_temperature_workspace_bytes(n, p))
    st = L.RadStats()
    code = lib.rad_steady_temperature(_vp(Y), n, ldy, _vp(weight), _vp(q), m, ldq,
                                      _vp(t_fixed), float(t_space), float(sigma),
                                      _vp(o), ldt, p, _vp(factors.buf), factors.buf.numel(), _vp(work),
                                      work.numel(), ctypes.byref(st) if want_stats else None, _stream(Y.device))
    L.check(code, "rad_steady_temperature")
    stats = st.as_dict() if want_stats else {}
    stats["status"] = code
    return (out[:, 0] if (vec and out.dim() == 2) else out), factors, stats


class Factors:
    """Device buffer holding a factorization of K (reused by the adjoint)."""

    def __init__(self, n: int, precision: str, device: torch.device):
        self.n = n
        self.precision = precision
        nbytes = L.lib().rad_gebhart_factor_bytes(n, _PREC[precision])
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)


def gebhart_ref(F: torch.Tensor, eps: torch.Tensor, rho: torch.Tensor, precision: str = "fp64",
                ir_tol: float = 1e-12, ir_max: int = 4, out: Optional[torch.Tensor] = None,
                factors: Optional[Factors] = None, want_stats: bool = True):
    """B = K^{-1} E (App. B.2, eq. B.8-B.11).  Returns (B, factors, stats)."""
    n = F.shape[0]
    ldf = _mat(F, "F", n, n + 1)
    _vec(eps, "eps", n)
    _vec(rho, "rho", n)
    if out is None:
        out = torch.empty((n, n + 1), dtype=torch.float64, device=F.device)
    ldb = _mat(out, "B", n, n + 1)
    if factors is None or factors.n != n or factors.precision != precision:
        factors = Factors(n, precision, F.device)
    lib = L.lib()
    p = _PREC[precision]
    work = WORKSPACE.get(F.device, "gebhart", lib.rad_gebhart_workspace_bytes(n, p))
    st = L.RadStats()
    code = lib.rad_gebhart_ref(_vp(F), n, ldf, _vp(eps), _vp(rho), _vp(out), ldb, p, float(ir_tol),
                               int(ir_max), _vp(factors.buf), factors.buf.numel(), _vp(work), work.numel(),
                               ctypes.byref(st) if want_stats else None, _stream(F.device))
    L.check(code, "rad_gebhart_ref")
    stats = st.as_dict() if want_stats else {}
    stats["status"] = code
    return out, factors, stats


def ref_check(B: torch.Tensor, eps: torch.Tensor, area: torch.Tensor) -> torch.Tensor:
    """[closure residual, reciprocity residual] of a REF matrix (eq. 4.3-4.4)."""
    n = B.shape[0]
    ldb = _mat(B, "B", n, n + 1)
    _vec(eps, "eps", n)
    _vec(area, "area", n)
    out = torch.empty(2, dtype=torch.float64, device=B.device)
    lib = L.lib()
    work = WORKSPACE.get(B.device, "refcheck", lib.rad_ref_check_workspace_bytes(n))
    code = lib.rad_ref_check(_vp(B), n, ldb, _vp(eps), _vp(area), _vp(out), _vp(work), work.numel(),
                             _stream(B.device))
    L.check(code, "rad_ref_check")
    return out


def gebhart_ref_adjoint(factors: Factors, F: torch.Tensor, rho: torch.Tensor, B: torch.Tensor,
                        G: torch.Tensor, want_lambda: bool = False, ir_tol: float = 1e-12,
                        ir_max: int = 4, want_stats: bool = True):
    """Returns (grad_eps, grad_rho, Lambda or None, stats) for G = dJ/dB."""
    n = F.shape[0]
    ldf = _mat(F, "F", n, n + 1)
    ldb = _mat(B, "B", n, n + 1)
    ldg = _mat(G, "G", n, n + 1)
    _vec(rho, "rho", n)
    ge = torch.empty(n, dtype=torch.float64, device=F.device)
    gr = torch.empty(n, dtype=torch.float64, device=F.device)
    lam = torch.empty((n, n + 1), dtype=torch.float64, device=F.device) if want_lambda else None
    ldl = lam.stride(0) if lam is not None else n + 1
    lib = L.lib()
    p = _PREC[factors.precision]
    work = WORKSPACE.get(F.device, "adjoint", lib.rad_adjoint_workspace_bytes(n, p))
    st = L.RadStats()
    code = lib.rad_gebhart_ref_adjoint(_vp(factors.buf), factors.buf.numel(), p, _vp(F), n, ldf, _vp(rho),
                                       _vp(B), ldb, _vp(G), ldg, _vp(ge), _vp(gr), _vp(lam), ldl,
                                       float(ir_tol), int(ir_max), _vp(work), work.numel(),
                                       ctypes.byref(st) if want_stats else None, _stream(F.device))
    L.check(code, "rad_gebhart_ref_adjoint")
    stats = st.as_dict() if want_stats else {}
    stats["status"] = code
    return ge, gr, lam, stats


class GebhartREF(torch.autograd.Function):
    """B = K(F, rho)^{-1} E(F, eps) with a hand-written adjoint backward.

    forward(F, eps, rho, precision) -> B;  backward gives (None, dJ/d eps,
    dJ/d rho, None) from the transposed solve that reuses the forward's factors.
    F is treated as a constant.
    """

    @staticmethod
    def forward(ctx, F, eps, rho, precision="fp64"):
        # statistics requested: the call waits for its kernels and raises on a
        # device-detected error (out-of-range eps / rho, non-finite F, singular K)
        B, factors, _ = gebhart_ref(F.detach(), eps.detach(), rho.detach(), precision=precision,
                                    want_stats=True)
        ctx.factors = factors
        ctx.save_for_backward(F, rho, B)
        return B

    @staticmethod
    def backward(ctx, G):
        F, rho, B = ctx.saved_tensors
        ge, gr, _, _ = gebhart_ref_adjoint(ctx.factors, F.detach(), rho.detach(), B,
                                           G.contiguous(), want_stats=True)
        return None, ge, gr, None


class Batch:
    """Many open models enforced and solved together (rad_batch_*, include/rad.h).

    ``models`` is a list of dicts with keys ``F`` ((n, n+1) float64 CUDA
    tensor, enforced in place), ``area``, ``n_rays`` (optional for
    kappa="half"), ``eps`` and ``rho`` (lists of one or two band vectors).
    The REF matrices land in ``self.B[i][band]``.  ``run`` only enqueues
    kernels on the current stream, so it may be captured in a CUDA graph.
    """

    def __init__(self, models, precision: str = "fp32_ir", kappa: str = "fracvar"):
        if not models:
            raise ValueError("empty batch")
        self.device = models[0]["F"].device
        self._keep = []
        self.B = []
        arr = (L.RadInstance * len(models))()
        for k, m in enumerate(models):
            F = m["F"]
            n = F.shape[0]
            ldf = _mat(F, f"models[{k}].F", n, n + 1)
            area = _vec(m["area"], "area", n)
            nr = _vec(m.get("n_rays"), "n_rays", n)
            eps, rho = list(m["eps"]), list(m["rho"])
            if not 1 <= len(eps) <= 2 or len(rho) != len(eps):
                raise ValueError(f"models[{k}]: one or two bands of eps and rho expected")
            bs = [torch.empty((n, n + 1), dtype=torch.float64, device=self.device) for _ in eps]
            s = arr[k]
            s.F, s.n, s.ldf = F.data_ptr(), n, ldf
            s.area = area.data_ptr()
            s.n_rays = nr.data_ptr() if nr is not None else None
            s.bands = len(eps)
            for b in range(len(eps)):
                s.eps[b] = _vec(eps[b], "eps", n).data_ptr()
                s.rho[b] = _vec(rho[b], "rho", n).data_ptr()
                s.B[b] = bs[b].data_ptr()
                s.ldb[b] = bs[b].stride(0)
            self._keep += [F, area, nr, *eps, *rho]
            self.B.append(bs)
        self.count = len(models)
        lib = L.lib()
        plan = ctypes.c_void_p()
        wb = ctypes.c_size_t()
        L.check(lib.rad_batch_plan_create(arr, len(models), _PREC[precision], _KAPPA[kappa], ctypes.byref(plan),
                                          ctypes.byref(wb)), "rad_batch_plan_create")
        self._plan = plan
        self.work = torch.empty(max(int(wb.value), 256), dtype=torch.uint8, device=self.device)
        L.check(lib.rad_batch_prepare(self._plan, _vp(self.work), self.work.numel(), _stream(self.device)),
                "rad_batch_prepare")

    def run(self, enforce_iters: int = 0, enforce_tol: float = 0.0, ir_steps: int = 1) -> None:
        L.check(L.lib().rad_batch_run(self._plan, _vp(self.work), float(enforce_tol), int(enforce_iters),
                                      int(ir_steps), _stream(self.device)), "rad_batch_run")

    def stats(self):
        out = (L.RadStats * self.count)()
        code = L.lib().rad_batch_stats(self._plan, _vp(self.work), out, _stream(self.device))
        L.check(code, "rad_batch_stats")
        return [s.as_dict() for s in out]

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan:
            L.lib().rad_batch_plan_destroy(plan)
            self._plan = None
