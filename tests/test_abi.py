"""CPU checks of the C ABI: the library loads and exports what include/rad.h declares."""
import pathlib
import re

from paper_2511_04277_amd import _lib

ROOT = pathlib.Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "rad.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rad_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_symbols()
    assert decl, "no declarations found"
    assert sorted(_lib.SIGNATURES) == decl


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_workspace_queries():
    lib = _lib.lib()
    assert lib.rad_status_string(-4).decode() == "singular pivot block"
    assert lib.rad_enforce_workspace_bytes(0) == 0
    assert lib.rad_enforce_workspace_bytes(1000) > 8 * 1000
    assert lib.rad_aggregate_workspace_bytes(1000, 10) >= 4 * 1000


def test_host_side_argument_errors_need_no_gpu():
    # argument validation happens before any device call
    lib = _lib.lib()
    code = lib.rad_enforce_vf(None, 10, 11, None, None, 0, 0.0, 1, None, 0, None, None)
    assert code == _lib.RAD_EINVAL
    assert b"NULL" in lib.rad_last_error()
    code = lib.rad_enforce_vf(_lib.ctypes.c_void_p(256), 10, 5, _lib.ctypes.c_void_p(256), None, 1, 0.0, 1,
                              None, 0, None, None)
    assert code == _lib.RAD_EINVAL and b"ldf" in lib.rad_last_error()


def test_tuning_roundtrip_and_validation():
    lib = _lib.lib()
    saved = _lib.tuning()
    try:
        _lib.apply_tuning({"small_tile_below_f64": 300, "small_tile_below_f32": 7, "lookahead": 0,
                           "side_chunk_tiles": 512})
        assert _lib.tuning() == {"small_tile_below_f64": 300, "small_tile_below_f32": 7, "lookahead": 0,
                                 "side_chunk_tiles": 512}
        bad = _lib.RadTuning(-1, 0, 1, 0)
        assert lib.rad_tuning_set(_lib.ctypes.byref(bad)) == _lib.RAD_EINVAL
        bad = _lib.RadTuning(0, 0, 2, 0)
        assert lib.rad_tuning_set(_lib.ctypes.byref(bad)) == _lib.RAD_EINVAL
        bad = _lib.RadTuning(0, 0, 1, -3)
        assert lib.rad_tuning_set(_lib.ctypes.byref(bad)) == _lib.RAD_EINVAL
        assert _lib.tuning()["small_tile_below_f64"] == 300  # unchanged by a rejected call
    finally:
        _lib.apply_tuning(saved)


def test_precision_size_queries():
    lib = _lib.lib()
    n = 4000
    f64 = lib.rad_gebhart_factor_bytes(n, _lib.RAD_PREC_FP64)
    # the int8-emulated mode keeps FP64 factors and adds the digit buffers
    assert lib.rad_gebhart_factor_bytes(n, _lib.RAD_PREC_FP64_I8) == f64
    w64 = lib.rad_gebhart_workspace_bytes(n, _lib.RAD_PREC_FP64)
    assert lib.rad_gebhart_workspace_bytes(n, _lib.RAD_PREC_FP64_I8) > w64 + 7 * 4096 * 1024
    assert lib.rad_adjoint_workspace_bytes(n, _lib.RAD_PREC_FP64_I8) > lib.rad_adjoint_workspace_bytes(
        n, _lib.RAD_PREC_FP64)
    for q in (lib.rad_gebhart_factor_bytes, lib.rad_gebhart_workspace_bytes, lib.rad_adjoint_workspace_bytes):
        assert q(n, 3) == 0 and q(0, _lib.RAD_PREC_FP64_I8) == 0


def test_calls_are_marked_as_roctx_ranges():
    # every compute entry point opens a named roctx range (marker traces)
    import subprocess
    syms = subprocess.run(["nm", "-D", "--undefined-only", str(_lib.LIB_PATH)], capture_output=True, text=True,
                          check=True).stdout
    assert "roctxRangePushA" in syms and "roctxRangePop" in syms
    src = "\n".join(p.read_text() for p in sorted((ROOT / "paper_2511_04277_amd" / "csrc").glob("*.hip")))
    for name in ("rad_enforce_vf", "rad_enforce_vf_noalloc", "rad_gebhart_ref", "rad_gebhart_ref_adjoint",
                 "rad_ref_check", "rad_aggregate_nodes", "rad_absorbed_flux", "rad_enforce_lsq", "rad_view_fractions",
                 "rad_node_emissivity", "rad_steady_temperature", "rad_batch_prepare", "rad_batch_run"):
        assert f'ApiRange range("{name}")' in src, name
