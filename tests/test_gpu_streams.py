"""GPU: independent pipelines on separate streams.

Two enforce -> solve -> adjoint pipelines issued on two streams at once
(their own buffers, the binding's per-stream workspaces, the library's shared
side stream for the look-ahead) must give bit for bit what each gives alone,
in FP64, in FP32 with refinement and with int8-emulated products.
"""
import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_util import dev, need_gpu, torch

pytestmark = pytest.mark.gpu


def _pipeline(rad, f0, area, nrays, eps, rho, g, precision):
    f = f0.clone()
    rad.enforce_vf_(f, area, nrays, tol=1e-13, max_iter=60, want_stats=False)
    b, fac, _ = rad.gebhart_ref(f, eps, rho, precision=precision, ir_tol=0.0, ir_max=2, want_stats=False)
    ge, gr, _, _ = rad.gebhart_ref_adjoint(fac, f, rho, b, g, ir_tol=0.0, ir_max=2, want_stats=False)
    return f, b, ge, gr


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "fp64_i8"])
def test_two_streams_match_sequential(precision):
    need_gpu()
    import paper_2511_04277_amd as rad
    insts = [W.box_with_n(2300, seed=21), W.box_with_n(1500, seed=22)]
    args = []
    for inst in insts:
        g = dev(np.random.default_rng(inst.n).uniform(-1, 1, (inst.n, inst.n + 1)))
        args.append((dev(inst.f_noisy), dev(inst.area), dev(inst.n_rays), dev(inst.eps[0]), dev(inst.rho[0]), g))
    print(f"[streams] precision={precision} n={[i.n for i in insts]}", flush=True)
    ref = [_pipeline(rad, *a, precision) for a in args]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]
    for rep in range(2):
        for s in streams:
            s.wait_stream(torch.cuda.current_stream())
        for k in (0, 1):
            with torch.cuda.stream(streams[k]):
                out[k] = _pipeline(rad, *args[k], precision)
        for s in streams:
            torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for k in (0, 1):
            for a, b in zip(out[k], ref[k]):
                assert torch.equal(a, b), (rep, k)
