"""Helpers for the GPU parity tests (inputs on the device, results back on the host)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2511_04277_amd import _lib
    _lib.lib()  # raises if the HIP library is missing: no silent fallback


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def padded(a, ld):
    """Device copy of a 2-D array stored with leading dimension ld >= cols."""
    rows, cols = a.shape
    buf = torch.full((rows, ld), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :cols] = dev(a)
    return buf[:, :cols]


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
