"""GPU: the allocation-free enforcement entry point (rad_enforce_vf_noalloc)
against rad_enforce_vf, called through the C ABI (the module is named to be
collected last): two calls in a row, the
second on a smaller input, each bitwise equal to the workspace entry point
(same kernels, same order of operations), in fixed-iteration and tolerance
mode; a size beyond the built-in scratch is refused before any device work."""
import ctypes

import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu


def _workspace_call(lib, L, F, inst, mode, tol, iters):
    n = inst.n
    wb = lib.rad_enforce_workspace_bytes(n)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    area, nr = dev(inst.area), dev(inst.n_rays)
    st = L.RadStats()
    code = lib.rad_enforce_vf(ctypes.c_void_p(F.data_ptr()), n, F.stride(0), ctypes.c_void_p(area.data_ptr()),
                              ctypes.c_void_p(nr.data_ptr()), mode, tol, iters, ctypes.c_void_p(work.data_ptr()),
                              work.numel(), ctypes.byref(st), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, st


def _noalloc_call(lib, L, F, inst, mode, tol, iters, stats=True):
    n = inst.n
    area, nr = dev(inst.area), dev(inst.n_rays)
    st = L.RadStats()
    code = lib.rad_enforce_vf_noalloc(ctypes.c_void_p(F.data_ptr()), n, F.stride(0),
                                      ctypes.c_void_p(area.data_ptr()), ctypes.c_void_p(nr.data_ptr()), mode, tol,
                                      iters, ctypes.byref(st) if stats else None,
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return code, st


@pytest.mark.parametrize("mode, tol, iters", [(0, 0.0, 12), (0, 1e-12, 400), (1, 0.0, 9)])
def test_noalloc_matches_workspace_entry_point(mode, tol, iters):
    need_gpu()
    from paper_2511_04277_amd import _lib as L
    lib = L.lib()
    # a large input first, then a smaller one: the second call must not see
    # anything the first left in the shared scratch
    for inst in (W.box_with_n(2300, seed=21, rays=5000), W.small_box(5, 2, seed=22)):
        n = inst.n
        print(f"[noalloc] n={n} mode={mode} tol={tol} iters={iters}", flush=True)
        f_ref = dev(inst.f_noisy)
        code_ref, st_ref = _workspace_call(lib, L, f_ref, inst, mode, tol, iters)
        f_new = dev(inst.f_noisy)
        code_new, st_new = _noalloc_call(lib, L, f_new, inst, mode, tol, iters)
        assert code_ref == code_new == 0
        assert torch.equal(f_ref, f_new)
        assert st_new.iters == st_ref.iters and st_new.converged == st_ref.converged
        assert st_new.closure_defect == st_ref.closure_defect and st_new.recip_err == st_ref.recip_err
    # statistics off (no host synchronisation): same result once the stream is drained
    inst = W.small_box(4, 2, seed=23)
    f_ref = dev(inst.f_noisy)
    _workspace_call(lib, L, f_ref, inst, mode, 0.0, 7)
    f_new = dev(inst.f_noisy)
    code, _ = _noalloc_call(lib, L, f_new, inst, mode, 0.0, 7, stats=False)
    assert code == 0 and torch.equal(f_ref, f_new)


def test_noalloc_refuses_sizes_beyond_its_scratch():
    need_gpu()
    from paper_2511_04277_amd import _lib as L
    lib = L.lib()
    n = 20000
    assert lib.rad_enforce_workspace_bytes(n) > L.RAD_ENFORCE_NOALLOC_BYTES
    assert lib.rad_enforce_workspace_bytes(16384) <= L.RAD_ENFORCE_NOALLOC_BYTES
    # only the pointers' non-NULL-ness matters: the size check comes before any device work
    code = lib.rad_enforce_vf_noalloc(ctypes.c_void_p(256), n, n + 1, ctypes.c_void_p(256), None, 1, 0.0, 1, None,
                                      None)
    assert code == L.RAD_EWORKSPACE
    assert b"scratch" in lib.rad_last_error()
