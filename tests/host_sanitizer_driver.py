"""Drives the host-side code of librad through its C ABI, for the sanitized
build (AddressSanitizer + UBSan on the host code; see build.py).

Run by tests/test_host_sanitizers.py in a child process that preloads the
sanitizer runtime and points RAD_LIBRARY at the sanitized library.  Every call
here is rejected by the library's host-side checks before any HIP call (the
device pointers are fake, never dereferenced), so the script needs no GPU and
does nothing to one: argument validation of every entry point, the workspace
and factor layouts over a range of sizes, the batch planner on many instance
sets, the tuning and profiling knobs, and the error strings.

It loads the binding module by path so that torch is not imported.  Exit
status 0 means every call returned what it should; a sanitizer report makes
the process fail on its own.
"""
from __future__ import annotations

import ctypes
import importlib.util
import math
import pathlib
import random
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]
_spec = importlib.util.spec_from_file_location("rad_host_lib", ROOT / "paper_2511_04277_amd" / "_lib.py")
L = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(L)

FAKE = 1 << 20  # a 256-byte aligned address that no call below dereferences
failures: list[str] = []


def expect(label: str, code: int, want, fragment: str = "") -> None:
    msg = (L.lib().rad_last_error() or b"").decode()
    ok = (code == want) if isinstance(want, int) else want(code)
    if not ok or (fragment and fragment not in msg):
        failures.append(f"{label}: code {code}, message {msg!r}")


def neg(code: int) -> bool:
    return code < 0


def mutate(base: dict, **kw) -> list:
    d = dict(base)
    d.update(kw)
    return list(d.values())


def sizes():
    return [1, 2, 31, 63, 64, 65, 127, 128, 129, 1000, 1023, 1024, 1025, 4097, 8192, 16384, 65535]


def check_queries(lib) -> None:
    precs = (L.RAD_PREC_FP64, L.RAD_PREC_FP32_IR, L.RAD_PREC_FP64_I8)
    one_arg = ["rad_enforce_workspace_bytes", "rad_ref_check_workspace_bytes"]
    by_prec = ["rad_gebhart_factor_bytes", "rad_gebhart_workspace_bytes", "rad_adjoint_workspace_bytes",
               "rad_enforce_lsq_workspace_bytes", "rad_steady_temperature_workspace_bytes"]
    two_arg = ["rad_aggregate_workspace_bytes", "rad_view_fractions_workspace_bytes",
               "rad_node_emissivity_workspace_bytes", "rad_absorbed_flux_workspace_bytes"]
    for name in one_arg:
        f = getattr(lib, name)
        prev = 0
        for n in sizes():
            b = f(n)
            if b < prev or b == 0:
                failures.append(f"{name}({n}) = {b} after {prev}")
            prev = b
        for n in (0, -1):
            f(n)
    for name in by_prec:
        f = getattr(lib, name)
        for p in precs:
            prev = 0
            for n in sizes():
                b = f(n, p)
                if b < prev:
                    failures.append(f"{name}({n}, {p}) = {b} after {prev}")
                prev = b
            f(0, p)
            f(-5, p)
        f(100, 77)
    for name in two_arg:
        f = getattr(lib, name)
        for n in sizes():
            for g in (1, 2, max(1, n // 4), n):
                f(n, g)
        f(0, 0)
        f(10, -1)


def check_enforce(lib) -> None:
    n = 1000
    need = lib.rad_enforce_workspace_bytes(n)
    base = dict(F=FAKE, n=n, ldf=n + 1, area=FAKE, n_rays=FAKE, kappa=L.RAD_KAPPA_FRACVAR, tol=0.0, max_iter=5,
                work=FAKE, work_bytes=need - 1, stats=None, stream=None)
    f = lib.rad_enforce_vf
    expect("enforce: short workspace", f(*mutate(base)), L.RAD_EWORKSPACE, "workspace")
    expect("enforce: misaligned", f(*mutate(base, work=FAKE + 8, work_bytes=need)), L.RAD_EWORKSPACE, "aligned")
    expect("enforce: n = 0", f(*mutate(base, n=0)), L.RAD_EINVAL, "n out of range")
    expect("enforce: n too big", f(*mutate(base, n=(1 << 20) + 1, ldf=(1 << 20) + 2)), L.RAD_EINVAL, "n out")
    expect("enforce: ldf", f(*mutate(base, ldf=n)), L.RAD_EINVAL, "ldf")
    expect("enforce: F", f(*mutate(base, F=None)), L.RAD_EINVAL, "NULL")
    expect("enforce: area", f(*mutate(base, area=None)), L.RAD_EINVAL, "NULL")
    expect("enforce: kappa", f(*mutate(base, kappa=9)), L.RAD_EINVAL, "kappa")
    expect("enforce: n_rays", f(*mutate(base, n_rays=None)), L.RAD_EINVAL, "n_rays")
    expect("enforce: max_iter", f(*mutate(base, max_iter=0)), L.RAD_EINVAL, "max_iter")
    expect("enforce: tol", f(*mutate(base, tol=-1.0)), L.RAD_EINVAL, "tol")
    expect("enforce: tol nan", f(*mutate(base, tol=math.nan)), L.RAD_EINVAL, "tol")
    g = lib.rad_enforce_vf_noalloc
    nb = dict(base)
    del nb["work"], nb["work_bytes"]
    expect("noalloc: n too big for scratch", g(*mutate(nb, n=20000, ldf=20001)), L.RAD_EWORKSPACE, "needs")
    expect("noalloc: kappa", g(*mutate(nb, kappa=3)), L.RAD_EINVAL, "kappa")
    expect("noalloc: ldf", g(*mutate(nb, ldf=5)), L.RAD_EINVAL, "ldf")


def check_gebhart(lib) -> None:
    n = 1000
    for p in (L.RAD_PREC_FP64, L.RAD_PREC_FP32_IR, L.RAD_PREC_FP64_I8):
        fb = lib.rad_gebhart_factor_bytes(n, p)
        wb = lib.rad_gebhart_workspace_bytes(n, p)
        base = dict(F=FAKE, n=n, ldf=n + 1, eps=FAKE, rho=FAKE, B=FAKE, ldb=n + 1, precision=p, ir_tol=0.0, ir_max=0,
                    factors=FAKE, fbytes=fb, work=FAKE, wbytes=wb - 1, stats=None, stream=None)
        f = lib.rad_gebhart_ref
        tag = f"gebhart[{p}]"
        expect(tag + ": short workspace", f(*mutate(base)), L.RAD_EWORKSPACE)
        expect(tag + ": short factors", f(*mutate(base, fbytes=fb - 1, wbytes=wb)), neg)
        expect(tag + ": n", f(*mutate(base, n=0)), L.RAD_EINVAL, "n out of range")
        expect(tag + ": ldb", f(*mutate(base, ldb=n)), L.RAD_EINVAL, "ld")
        expect(tag + ": B", f(*mutate(base, B=None)), L.RAD_EINVAL, "NULL")
        expect(tag + ": precision", f(*mutate(base, precision=17)), L.RAD_EINVAL, "precision")
        expect(tag + ": ir_max", f(*mutate(base, ir_max=-1)), L.RAD_EINVAL, "ir_max")
        # adjoint
        aw = lib.rad_adjoint_workspace_bytes(n, p)
        abase = dict(factors=FAKE, fbytes=fb, precision=p, F=FAKE, n=n, ldf=n + 1, rho=FAKE, B=FAKE, ldb=n + 1,
                     G=FAKE, ldg=n + 1, grad_eps=FAKE, grad_rho=FAKE, Lam=None, ldl=0, ir_tol=0.0, ir_max=0,
                     work=FAKE, wbytes=aw - 1, stats=None, stream=None)
        a = lib.rad_gebhart_ref_adjoint
        tag = f"adjoint[{p}]"
        expect(tag + ": short workspace", a(*mutate(abase)), L.RAD_EWORKSPACE)
        expect(tag + ": short factors", a(*mutate(abase, fbytes=fb - 8, wbytes=aw)), L.RAD_EWORKSPACE)
        expect(tag + ": ldg", a(*mutate(abase, ldg=3)), L.RAD_EINVAL)
        expect(tag + ": Lambda ld", a(*mutate(abase, Lam=FAKE, ldl=n)), L.RAD_EINVAL)
        expect(tag + ": grad", a(*mutate(abase, grad_rho=None)), L.RAD_EINVAL, "NULL")
        expect(tag + ": precision", a(*mutate(abase, precision=-3)), L.RAD_EINVAL, "precision")
    # REF checks
    rw = lib.rad_ref_check_workspace_bytes(n)
    rbase = dict(B=FAKE, n=n, ldb=n + 1, eps=FAKE, area=FAKE, out=FAKE, work=FAKE, wbytes=rw - 1, stream=None)
    r = lib.rad_ref_check
    expect("ref_check: short workspace", r(*mutate(rbase)), neg)
    expect("ref_check: ldb", r(*mutate(rbase, ldb=n)), L.RAD_EINVAL)
    expect("ref_check: out", r(*mutate(rbase, out=None)), L.RAD_EINVAL, "NULL")


def check_next_rows(lib) -> None:
    n, g = 1000, 100
    # aggregation
    aw = lib.rad_aggregate_workspace_bytes(n, g)
    base = dict(X=FAKE, n=n, ldx=n + 1, weight=FAKE, group=FAKE, g=g, Y=FAKE, ldy=g + 1, gw=None, work=FAKE,
                wbytes=aw - 1, stats=None, stream=None)
    f = lib.rad_aggregate_nodes
    expect("aggregate: short workspace", f(*mutate(base)), L.RAD_EWORKSPACE)
    expect("aggregate: g > n", f(*mutate(base, g=n + 1, ldy=n + 2)), L.RAD_EINVAL, "g must")
    expect("aggregate: ldy", f(*mutate(base, ldy=g)), L.RAD_EINVAL, "ld")
    expect("aggregate: group", f(*mutate(base, group=None)), L.RAD_EINVAL, "NULL")
    # view fractions, node emissivity
    vw = lib.rad_view_fractions_workspace_bytes(n, g)
    vbase = dict(F=FAKE, nf=n, ldf=n + 1, group=FAKE, g=g, R=FAKE, ldr=n + 1, work=FAKE, wbytes=vw - 1, stats=None,
                 stream=None)
    v = lib.rad_view_fractions
    expect("view_fractions: short workspace", v(*mutate(vbase)), L.RAD_EWORKSPACE)
    expect("view_fractions: g", v(*mutate(vbase, g=0)), L.RAD_EINVAL, "g must")
    expect("view_fractions: ldr", v(*mutate(vbase, ldr=n)), L.RAD_EINVAL, "ld")
    ew = lib.rad_node_emissivity_workspace_bytes(n, g)
    ebase = dict(B=FAKE, nf=n, ldb=n + 1, eps=FAKE, area=FAKE, group=FAKE, g=g, E=FAKE, lde=g + 1, work=FAKE,
                 wbytes=ew - 1, stats=None, stream=None)
    e = lib.rad_node_emissivity
    expect("node_emissivity: short workspace", e(*mutate(ebase)), L.RAD_EWORKSPACE)
    expect("node_emissivity: lde", e(*mutate(ebase, lde=g)), L.RAD_EINVAL, "ld")
    expect("node_emissivity: eps", e(*mutate(ebase, eps=None)), L.RAD_EINVAL, "NULL")
    # absorbed fluxes
    for m in (1, 7, 16):
        hw = lib.rad_absorbed_flux_workspace_bytes(n, m)
        hbase = dict(B=FAKE, n=n, ldb=n + 1, eps=FAKE, rho=FAKE, area=FAKE, Qd=FAKE, m=m, ldq=m, Qa=FAKE, lda=m,
                     work=FAKE, wbytes=hw - 1, stream=None)
        h = lib.rad_absorbed_flux
        expect(f"ahf[{m}]: short workspace", h(*mutate(hbase)), neg)
        expect(f"ahf[{m}]: m", h(*mutate(hbase, m=17, ldq=17, lda=17)), L.RAD_EINVAL, "m outside")
        expect(f"ahf[{m}]: ldq", h(*mutate(hbase, ldq=m - 1)), L.RAD_EINVAL, "leading")
    # steady temperatures and the least-squares enforcer
    for p in (L.RAD_PREC_FP64, L.RAD_PREC_FP64_I8):
        fb = lib.rad_gebhart_factor_bytes(n, p)
        sw = lib.rad_steady_temperature_workspace_bytes(n, p)
        sbase = dict(Y=FAKE, n=n, ldy=n + 1, weight=FAKE, Q=FAKE, m=4, ldq=4, fixed=None, t_space=3.0,
                     sigma=5.670374419e-8, T=FAKE, ldt=4, precision=p, factors=FAKE, fbytes=fb, work=FAKE,
                     wbytes=sw - 1, stats=None, stream=None)
        s = lib.rad_steady_temperature
        expect(f"steady[{p}]: short workspace", s(*mutate(sbase)), L.RAD_EWORKSPACE)
        expect(f"steady[{p}]: m", s(*mutate(sbase, m=65, ldq=65, ldt=65)), L.RAD_EINVAL)
        expect(f"steady[{p}]: sigma", s(*mutate(sbase, sigma=0.0)), L.RAD_EINVAL)
        expect(f"steady[{p}]: fp32", s(*mutate(sbase, precision=L.RAD_PREC_FP32_IR)), L.RAD_EINVAL)
        lw = lib.rad_enforce_lsq_workspace_bytes(n, p)
        lbase = dict(F=FAKE, n=n, ldf=n + 1, omega=FAKE, Fout=FAKE + 4096, ldo=n + 1, flags=3, max_rounds=4,
                     precision=p, factors=FAKE, fbytes=fb, work=FAKE, wbytes=lw - 1, stats=None, stream=None)
        q = lib.rad_enforce_lsq
        expect(f"lsq[{p}]: short workspace", q(*mutate(lbase)), L.RAD_EWORKSPACE)
        expect(f"lsq[{p}]: same buffer", q(*mutate(lbase, Fout=FAKE)), L.RAD_EINVAL, "same buffer")
        expect(f"lsq[{p}]: flags", q(*mutate(lbase, flags=8)), L.RAD_EINVAL)
        expect(f"lsq[{p}]: n", q(*mutate(lbase, n=70000, ldf=70001, ldo=70001)), L.RAD_EINVAL, "n out")


def _inst(n, bands, fracvar=True, ldf=None):
    s = L.RadInstance()
    s.F = FAKE
    s.n = n
    s.ldf = ldf if ldf is not None else n + 1 + (n % 3)
    s.area = FAKE
    s.n_rays = FAKE if fracvar else None
    s.bands = bands
    for b in range(min(bands, 2)):
        s.eps[b] = FAKE
        s.rho[b] = FAKE
        s.B[b] = FAKE
        s.ldb[b] = n + 1
    return s


def check_batch(lib) -> None:
    rng = random.Random(2511)
    create = lib.rad_batch_plan_create
    for trial in range(40):
        count = rng.choice([1, 2, 3, 7, 16, 40])
        insts = [_inst(int(math.exp(rng.uniform(0.0, math.log(5000)))), rng.choice([1, 2])) for _ in range(count)]
        for p in (L.RAD_PREC_FP64, L.RAD_PREC_FP32_IR, L.RAD_PREC_FP64_I8):
            for kappa in (L.RAD_KAPPA_FRACVAR, L.RAD_KAPPA_HALF):
                arr = (L.RadInstance * count)(*insts)
                plan = ctypes.c_void_p()
                wb = ctypes.c_size_t()
                code = create(arr, count, p, kappa, ctypes.byref(plan), ctypes.byref(wb))
                expect(f"batch create trial {trial}", code, L.RAD_OK)
                if code != L.RAD_OK:
                    continue
                need = sum(s.bands * lib.rad_gebhart_factor_bytes(s.n, p) for s in insts)
                if wb.value <= need:
                    failures.append(f"batch workspace {wb.value} <= factor bytes {need}")
                expect("batch prepare short", lib.rad_batch_prepare(plan, FAKE, wb.value - 1, None), L.RAD_EWORKSPACE)
                expect("batch prepare misaligned", lib.rad_batch_prepare(plan, FAKE + 16, wb.value, None),
                       L.RAD_EWORKSPACE)
                expect("batch run unprepared", lib.rad_batch_run(plan, FAKE, 0.0, 1, 0, None), L.RAD_EINVAL,
                       "prepared")
                expect("batch stats NULL", lib.rad_batch_stats(plan, FAKE, None, None), L.RAD_EINVAL)
                lib.rad_batch_plan_destroy(plan)
    bad = [
        ([_inst(100, 1, ldf=50)], "ldf"),
        ([_inst(100, 3)], "bands"),
        ([_inst(100, 1, fracvar=False)], "n_rays"),
        ([_inst(0, 1)], ""),
    ]
    for insts, frag in bad:
        arr = (L.RadInstance * len(insts))(*insts)
        plan = ctypes.c_void_p()
        wb = ctypes.c_size_t()
        expect(f"batch rejects ({frag})", create(arr, len(insts), L.RAD_PREC_FP64, L.RAD_KAPPA_FRACVAR,
                                                 ctypes.byref(plan), ctypes.byref(wb)), L.RAD_EINVAL, frag)
        if plan.value:
            failures.append("a rejected plan was returned")
    one = (L.RadInstance * 1)(_inst(10, 1))
    plan = ctypes.c_void_p()
    wb = ctypes.c_size_t()
    expect("batch count 0", create(one, 0, 0, 0, ctypes.byref(plan), ctypes.byref(wb)), L.RAD_EINVAL)
    expect("batch precision", create(one, 1, 9, 0, ctypes.byref(plan), ctypes.byref(wb)), L.RAD_EINVAL)
    expect("batch kappa", create(one, 1, 0, 9, ctypes.byref(plan), ctypes.byref(wb)), L.RAD_EINVAL)
    expect("batch NULL outputs", create(one, 1, 0, 0, None, None), L.RAD_EINVAL)
    lib.rad_batch_plan_destroy(None)


def check_knobs(lib) -> None:
    t = L.RadTuning()
    expect("tuning get", lib.rad_tuning_get(ctypes.byref(t)), L.RAD_OK)
    saved = L.RadTuning(t.small_tile_below_f64, t.small_tile_below_f32, t.lookahead, t.side_chunk_tiles)
    expect("tuning set", lib.rad_tuning_set(ctypes.byref(L.RadTuning(0, 1 << 30, 0, 384))), L.RAD_OK)
    expect("tuning set invalid", lib.rad_tuning_set(ctypes.byref(L.RadTuning(-1, 0, 1, 0))), L.RAD_EINVAL)
    expect("tuning NULL", lib.rad_tuning_set(None), L.RAD_EINVAL)
    expect("tuning restore", lib.rad_tuning_set(ctypes.byref(saved)), L.RAD_OK)
    expect("profile kinds", lib.rad_profile_kinds(0xFFFFFFFF), L.RAD_OK)
    expect("profile off", lib.rad_profile_enable(0), lambda c: c >= 0)
    out = (L.RadKernelProfile * 16)()
    expect("profile read", lib.rad_profile_read(out, 16), lambda c: c >= 0)
    expect("profile read NULL", lib.rad_profile_read(None, 4), L.RAD_EINVAL)
    for code in range(-12, 4):
        if not lib.rad_status_string(code):
            failures.append(f"no status string for {code}")
    if lib.rad_version() <= 0:
        failures.append("rad_version")


def main() -> int:
    lib = L.lib()
    for step in (check_queries, check_enforce, check_gebhart, check_next_rows, check_batch, check_knobs):
        step(lib)
        print(f"{step.__name__}: done", flush=True)
    for f in failures:
        print("FAIL", f)
    return 1 if failures else 0


if __name__ == "__main__":
    sys.exit(main())
