"""CPU checks of the batch planner: rad_batch_plan_create does host work only."""
import ctypes

from paper_2511_04277_amd import _lib


def _inst(n, bands=2, ldf=None, fake=4096):
    s = _lib.RadInstance()
    s.F = fake
    s.n = n
    s.ldf = ldf if ldf is not None else n + 1
    s.area = fake
    s.n_rays = fake
    s.bands = bands
    for b in range(min(bands, 2)):
        s.eps[b] = fake
        s.rho[b] = fake
        s.B[b] = fake
        s.ldb[b] = n + 1
    return s


def _create(insts, precision=_lib.RAD_PREC_FP32_IR, kappa=_lib.RAD_KAPPA_FRACVAR):
    arr = (_lib.RadInstance * len(insts))(*insts)
    plan = ctypes.c_void_p()
    wb = ctypes.c_size_t()
    code = _lib.lib().rad_batch_plan_create(arr, len(insts), precision, kappa, ctypes.byref(plan), ctypes.byref(wb))
    return code, plan, wb.value


def test_plan_sizes_cover_every_problem():
    lib = _lib.lib()
    ns = [300, 129, 1000, 64, 2100]
    sizes = {}
    for prec in (_lib.RAD_PREC_FP64, _lib.RAD_PREC_FP32_IR, _lib.RAD_PREC_FP64_I8):
        code, plan, wb = _create([_inst(n, bands=1 + (k % 2)) for k, n in enumerate(ns)], prec)
        assert code == _lib.RAD_OK
        # at least the factor buffers of every (instance, band) problem
        need = sum((1 + (k % 2)) * lib.rad_gebhart_factor_bytes(n, prec) for k, n in enumerate(ns))
        assert wb > need
        sizes[prec] = wb
        lib.rad_batch_plan_destroy(plan)
    # the int8-emulated mode adds digit buffers for the problems past one
    # 1024-wide panel (n = 2100 here: 7 digits of a 2176 x 1024 and a
    # (2176 + 2101) x 1024 operand), nothing else
    digits = 7 * 1024 * (2176 + (2176 + 2101 + 63) // 64 * 64)
    assert sizes[_lib.RAD_PREC_FP64_I8] >= sizes[_lib.RAD_PREC_FP64] + digits


def test_plan_rejects_bad_instances():
    lib = _lib.lib()
    code, plan, _ = _create([_inst(100, ldf=50)])
    assert code == _lib.RAD_EINVAL and not plan.value
    assert b"ldf" in lib.rad_last_error()
    code, _, _ = _create([_inst(100, bands=3)])
    assert code == _lib.RAD_EINVAL and b"bands" in lib.rad_last_error()
    bad = _inst(100)
    bad.n_rays = None
    code, _, _ = _create([bad])
    assert code == _lib.RAD_EINVAL and b"n_rays" in lib.rad_last_error()
    code, plan, _ = _create([bad], kappa=_lib.RAD_KAPPA_HALF)
    assert code == _lib.RAD_OK
    lib.rad_batch_plan_destroy(plan)


def test_run_rejects_unprepared_workspace():
    lib = _lib.lib()
    code, plan, wb = _create([_inst(64)])
    assert code == _lib.RAD_OK
    code = lib.rad_batch_run(plan, ctypes.c_void_p(1 << 20), 0.0, 1, 1, None)
    assert code == _lib.RAD_EINVAL and b"prepared" in lib.rad_last_error()
    code = lib.rad_batch_prepare(plan, ctypes.c_void_p(1 << 20), wb - 256, None)
    assert code == _lib.RAD_EWORKSPACE
    lib.rad_batch_plan_destroy(plan)
