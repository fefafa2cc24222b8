"""The host code of librad under AddressSanitizer and UBSan (CPU only).

build.build_host_sanitized() compiles the library with both sanitizers on the
host side; tests/host_sanitizer_driver.py then runs every entry point's
argument checks, the workspace and factor layouts over many sizes, the batch
planner on many instance sets and the runtime knobs in a child process that
preloads the sanitizer runtime.  No call reaches the GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

from paper_2511_04277_amd import build

ROOT = build.ROOT


@pytest.fixture(scope="module")
def sanitized():
    if not shutil.which(build.HIPCC) and not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.build_host_sanitized()
    return lib, build.sanitizer_runtime()


def test_sanitized_library_is_instrumented(sanitized):
    lib, _ = sanitized
    syms = subprocess.run(["nm", "-D", "--undefined-only", str(lib)], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in syms
    assert "__ubsan_handle" in syms


def test_host_code_is_clean_under_asan_and_ubsan(sanitized):
    lib, runtime = sanitized
    env = dict(os.environ)
    env.update(LD_PRELOAD=str(runtime), RAD_LIBRARY=str(lib), RAD_NO_TUNING="1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(ROOT / "tests" / "host_sanitizer_driver.py")], capture_output=True,
                       text=True, env=env, cwd=str(ROOT), timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "check_batch: done" in r.stdout and "check_knobs: done" in r.stdout
