"""GPU parity: the batched pipeline (rad_batch_*) of many uneven-N models x bands.

Checked three ways: against the FP64 oracle (Sec. 3.5.5 enforcement, App. B.2
solve), bit for bit against the single-model entry points (same kernels, same
arithmetic order), and across replays of a captured CUDA graph.
"""
import numpy as np
import pytest

import oracle
from synth import workloads as W
from tests.gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_IR = 1e-10
ITERS = 6


def _instances():
    # uneven sizes: below one 64-tile, ragged tails, one spanning three
    # 1024-wide panels; two bands each except the small one-band box
    out = [W.config3_instance(i) for i in (0, 3, 2, 9)]
    out.append(W.small_box(4, 2, seed=7))
    return out


def _models(insts):
    models, f0 = [], []
    for inst in insts:
        F = dev(inst.f_noisy)
        f0.append(F.clone())
        models.append({"F": F, "area": dev(inst.area), "n_rays": dev(inst.n_rays),
                       "eps": [dev(e) for e in inst.eps], "rho": [dev(r) for r in inst.rho]})
    return models, f0


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "fp64_i8"])
def test_batch_matches_oracle(precision):
    need_gpu()
    import paper_2511_04277_amd as rad
    insts = _instances()
    models, _ = _models(insts)
    print(f"[batch] oracle parity, precision={precision}, n={[i.n for i in insts]}", flush=True)
    batch = rad.Batch(models, precision=precision)
    batch.run(enforce_iters=ITERS, ir_steps=2)
    stats = batch.stats()
    tol = TOL64 if precision == "fp64" else TOL_IR  # fp32_ir: two refinement steps; fp64_i8: digit products
    for k, inst in enumerate(insts):
        f_ref, info = oracle.enforce_vf(inst.f_noisy, inst.area, inst.n_rays, "fracvar", tol=0.0, max_iter=ITERS)
        f_gpu = host(models[k]["F"])
        assert np.abs(f_gpu - f_ref).max() <= 1e-13, inst.name
        assert stats[k]["iters"] == ITERS and stats[k]["device_status"] == 0
        assert abs(stats[k]["closure_defect"] - info["closure_defect"]) <= 1e-12
        for b in range(len(inst.eps)):
            b_ref = oracle.gebhart_ref(f_gpu, inst.eps[b], inst.rho[b])
            err = np.abs(host(batch.B[k][b]) - b_ref).max()
            assert err <= tol, (inst.name, b, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "fp64_i8"])
def test_batch_equals_single_model_path(precision):
    need_gpu()
    import paper_2511_04277_amd as rad
    insts = _instances()
    models, f0 = _models(insts)
    print(f"[batch] single-path equality, precision={precision}", flush=True)
    batch = rad.Batch(models, precision=precision)
    batch.run(enforce_iters=ITERS, ir_steps=2)
    torch.cuda.synchronize()
    for k, m in enumerate(models):
        F = f0[k].clone()
        rad.enforce_vf_(F, m["area"], m["n_rays"], tol=0.0, max_iter=ITERS)
        assert torch.equal(F, m["F"]), insts[k].name
        for b in range(len(m["eps"])):
            B, _, _ = rad.gebhart_ref(F, m["eps"][b], m["rho"][b], precision=precision, ir_tol=0.0, ir_max=2)
            assert torch.equal(B, batch.B[k][b]), (insts[k].name, b)


def test_batch_tolerance_stops_each_instance():
    need_gpu()
    import paper_2511_04277_amd as rad
    insts = _instances()
    models, f0 = _models(insts)
    batch = rad.Batch(models, precision="fp64")
    batch.run(enforce_iters=300, enforce_tol=1e-10, ir_steps=0)
    stats = batch.stats()
    for k, m in enumerate(models):
        F = f0[k].clone()
        st = rad.enforce_vf_(F, m["area"], m["n_rays"], tol=1e-10, max_iter=300)
        assert stats[k]["converged"] == 1 and stats[k]["closure_defect"] <= 1e-10
        assert stats[k]["iters"] == st["iters"], insts[k].name
        assert torch.equal(F, m["F"])


@pytest.mark.parametrize("precision", ["fp32_ir", "fp64_i8"])
def test_batch_graph_replays_match_eager(precision):
    need_gpu()
    import paper_2511_04277_amd as rad
    insts = _instances()
    models, f0 = _models(insts)
    batch = rad.Batch(models, precision=precision)

    def step():
        for k, m in enumerate(models):
            m["F"].copy_(f0[k])
        batch.run(enforce_iters=ITERS, ir_steps=2)

    step()
    torch.cuda.synchronize()
    eager_b = [[b.clone() for b in bs] for bs in batch.B]
    eager_f = [m["F"].clone() for m in models]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        for bs in batch.B:  # clobber the outputs between replays with eager work
            for b in bs:
                b.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"[batch] graph replay {rep}", flush=True)
        for k in range(len(models)):
            assert torch.equal(models[k]["F"], eager_f[k])
            for b in range(len(eager_b[k])):
                assert torch.equal(batch.B[k][b], eager_b[k][b]), (rep, k, b)
