"""Build librad.so (the gfx950 HIP library behind include/rad.h) in-tree.

    python -m paper_2511_04277_amd.build

compiles every ``csrc/*.hip`` and ``csrc/*.cpp`` with hipcc for gfx950 into
``paper_2511_04277_amd/librad.so``.  Object files go to ``_build/``.

``build_host_sanitized()`` builds a second copy whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer instrumentation (device code
is compiled as usual, without it) into ``_build/host_sanitize/librad.so``;
the CPU tests load it with the sanitizer runtime preloaded and drive the
host-side logic (argument checks, workspace layouts, the batch planner).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import shutil
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = ROOT / "_build"
LIB = PKG / "librad.so"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = os.environ.get("RAD_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # keep MFMA accumulators in VGPRs (no per-iteration AGPR copies)
          "-mllvm", "-amdgpu-mfma-vgpr-form",
          "-Wno-unused-result", "-I", str(ROOT / "include")]
# roctx ranges around the C-ABI calls (marker traces)
LINK = ["-L", str(pathlib.Path(HIPCC).resolve().parent.parent / "lib"), "-lrocprofiler-sdk-roctx"]


def _compile(src: pathlib.Path) -> pathlib.Path:
    obj = BUILD / (src.name + ".o")
    cmd = [HIPCC, *COMMON, "-c", str(src), "-o", str(obj)]
    if src.suffix == ".cpp":
        cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-I", str(ROOT / "include"), "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> pathlib.Path:
    BUILD.mkdir(exist_ok=True)
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs), *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


SANITIZE_DIR = BUILD / "host_sanitize"
SANITIZE_LIB = SANITIZE_DIR / "librad.so"
# each -fsanitize= goes to the host compilation only
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _sources() -> list[pathlib.Path]:
    return sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.cpp"))


def sanitizer_runtime() -> pathlib.Path:
    """The clang AddressSanitizer runtime (it also carries the UBSan handlers)
    that a process loading the sanitized library must preload."""
    clang = pathlib.Path(HIPCC).resolve().parent.parent / "lib" / "llvm" / "lib" / "clang"
    found = sorted(clang.glob("*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        found = sorted(pathlib.Path("/opt/rocm/lib/llvm/lib/clang").glob("*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under the ROCm clang")
    return found[-1]


def build_host_sanitized(verbose: bool = False) -> pathlib.Path:
    """Sanitized host build (see the module docstring); rebuilt only when a
    source or header is newer than the library.  The shared library leaves the
    sanitizer symbols to the preloaded runtime."""
    SANITIZE_DIR.mkdir(parents=True, exist_ok=True)
    inputs = _sources() + sorted(CSRC.glob("*.h")) + sorted((ROOT / "include").glob("*.h"))
    if SANITIZE_LIB.exists() and SANITIZE_LIB.stat().st_mtime >= max(p.stat().st_mtime for p in inputs):
        return SANITIZE_LIB

    def one(src: pathlib.Path) -> pathlib.Path:
        obj = SANITIZE_DIR / (src.name + ".o")
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", *SANITIZE_HOST, "-Wno-unused-result",
               "-I", str(ROOT / "include"), "-c", str(src), "-o", str(obj)]
        if src.suffix == ".hip":
            cmd[5:5] = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    tmp = SANITIZE_LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs), *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SANITIZE_LIB)
    if verbose:
        print(f"built {SANITIZE_LIB}")
    return SANITIZE_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
