"""Autotuner of the library's runtime knobs (rad_tuning_set, include/rad.h).

    python -m paper_2511_04277_amd.autotune [--sizes 2048,8192] [--reps 3]

For each precision it times the Gebhart REF solve (FP64, and FP32 with one
refinement step) on synthetic open systems of the given sizes under every
candidate of

  * small_tile_below: GEMMs with fewer 128 x 128 output tiles than this run
    with 64 x 64 tiles (0 = never, a huge value = always);
  * lookahead: split each trailing update over two streams (0 / 1);
  * side_chunk_tiles: with look-ahead, the second stream's update in row
    chunks of at most this many 128 x 128 tiles (0 = one launch), tried
    with the best of the two knobs above;

keeps the fastest (summed over the sizes) and writes the table to
``paper_2511_04277_amd/tuning.json``, which the binding applies when the
library is loaded.  The knobs never change results beyond bitwise-identical
reordering of launches, so tuning needs no accuracy check; one is still made
against the untuned run as a guard.
"""
from __future__ import annotations

import argparse
import ctypes
import itertools
import json
import pathlib
import sys
import time

TUNING_PATH = pathlib.Path(__file__).resolve().parent / "tuning.json"
TILE_CANDIDATES = [0, 256, 1024, 4096, 1 << 30]
CHUNK_CANDIDATES = [256, 384, 512, 768, 1024, 2048]


def _system(n: int, seed: int, device):
    """A random open system with closed rows (the solve's cost does not
    depend on the values): F >= 0 with rows summing to 1 over N+1 columns,
    eps ~ U[0.1, 0.9], rho = 1 - eps."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    f = torch.rand((n, n + 1), generator=g, dtype=torch.float64)
    f /= f.sum(dim=1, keepdim=True)
    eps = 0.1 + 0.8 * torch.rand(n, generator=g, dtype=torch.float64)
    return f.to(device), eps.to(device), (1.0 - eps).to(device)


def _time_solve(rad, F, eps, rho, precision, reps, factors):
    import torch
    kw = {"precision": precision, "ir_tol": 1.0, "ir_max": 1} if precision == "fp32_ir" else {
        "precision": precision}
    B, factors, _ = rad.gebhart_ref(F, eps, rho, factors=factors, want_stats=False, **kw)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B, factors, _ = rad.gebhart_ref(F, eps, rho, out=B, factors=factors, want_stats=False, **kw)
        e1.record()
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1))
    t.sort()
    return t[len(t) // 2], B, factors


def tune(sizes, reps: int, out_path: pathlib.Path = TUNING_PATH, log=print) -> dict:
    import torch

    import paper_2511_04277_amd as rad
    from paper_2511_04277_amd import _lib as L

    assert torch.cuda.is_available(), "autotuning needs a ROCm device"
    lib = L.lib()
    dev = torch.device("cuda:0")
    systems = {n: _system(n, 2511 + n, dev) for n in sizes}
    best = {}
    table = []
    for precision in ("fp64", "fp32_ir"):
        ref = {}
        results = []

        def measure(tile, look, chunk):
            tun = L.RadTuning(tile, tile, look, chunk)
            L.check(lib.rad_tuning_set(ctypes.byref(tun)), "rad_tuning_set")
            total = 0.0
            per = {}
            for n, (F, eps, rho) in systems.items():
                ms, B, _ = _time_solve(rad, F, eps, rho, precision, reps, None)
                if n not in ref:
                    ref[n] = B.clone()
                elif not torch.equal(B, ref[n]):
                    raise RuntimeError(f"tuning changed the result (n={n}, tile={tile}, lookahead={look}, "
                                       f"side_chunk_tiles={chunk})")
                per[n] = ms
                total += ms
            results.append((total, tile, look, chunk, per))
            table.append({"precision": precision, "small_tile_below": tile, "lookahead": look,
                          "side_chunk_tiles": chunk, "ms": {str(k): round(v, 3) for k, v in per.items()}})
            log(f"[autotune] {precision} small_tile_below={tile} lookahead={look} side_chunk_tiles={chunk}: "
                + ", ".join(f"n={k} {v:.2f} ms" for k, v in per.items()))

        for tile, look in itertools.product(TILE_CANDIDATES, (1, 0)):
            measure(tile, look, 0)
        _, tile, look, _, _ = min(results, key=lambda r: r[0])
        if look:
            for chunk in CHUNK_CANDIDATES:
                measure(tile, 1, chunk)
        total, tile, look, chunk, _ = min(results, key=lambda r: r[0])
        best[precision] = {"small_tile_below": tile, "lookahead": look, "side_chunk_tiles": chunk,
                           "total_ms": round(total, 3)}
        log(f"[autotune] {precision}: best small_tile_below={tile} lookahead={look} side_chunk_tiles={chunk} "
            f"({total:.2f} ms)")
    # one look-ahead setting serves both precisions: the FP64 choice
    chosen = {"small_tile_below_f64": best["fp64"]["small_tile_below"],
              "small_tile_below_f32": best["fp32_ir"]["small_tile_below"],
              "lookahead": best["fp64"]["lookahead"], "side_chunk_tiles": best["fp64"]["side_chunk_tiles"]}
    doc = {"device": torch.cuda.get_device_name(0), "sizes": list(sizes), "reps": reps,
           "chosen": chosen, "best": best, "measurements": table}
    out_path.write_text(json.dumps(doc, indent=1) + "\n")
    L.apply_tuning(chosen)
    log(f"[autotune] wrote {out_path}: {chosen}")
    return doc


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", default="2048,8192", help="comma list of N")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=str(TUNING_PATH))
    args = ap.parse_args()
    t0 = time.time()
    tune([int(x) for x in args.sizes.split(",") if x], args.reps, pathlib.Path(args.out))
    print(f"[autotune] done in {time.time() - t0:.1f}s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
