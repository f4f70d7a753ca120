"""Tile-shape autotuner for the factorisation on the current GPU.

For each precision and each size in the sweep it times chol_factor on a
synthetic squared-exponential GP matrix for every (tile, panel width) pair
and records the fastest; the result is a table of rows
[n_max, tile, panel_width] per precision, read by the serving loop
(``serve.TuningTable``).  Timing uses HIP events around the call on the
current stream, best of ``reps`` after one warm-up.

    python -m paper_2605_13209_amd.autotune --out paper_2605_13209_amd/tuning/mi355x_gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

SIZES = (256, 512, 1024, 2048, 4096, 8192, 16384)
TILES = (64, 128)
WIDTHS = (1, 2, 4, 8)


def _problem(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, (n, 8)))


def time_factor(P, torch, A, precision: str, tile: int, width: int, reps: int) -> float:
    n = A.shape[0]
    ws = torch.empty(P.chol_factor_bytes(n, precision, tile), dtype=torch.uint8, device=A.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for r in range(reps + 1):
        e0.record()
        F = P.chol_factor(A, precision, tile, workspace=ws, sync=False, panel_width=width)
        e1.record()
        e1.synchronize()
        if F.info() != 0:
            raise RuntimeError(f"factorisation failed at n={n}")
        if r > 0:
            best = min(best, e0.elapsed_time(e1))
    return best


def sweep(sizes=SIZES, precisions=("fp64", "fp32"), tiles=TILES, widths=WIDTHS, reps: int = 3):
    import torch
    from . import _native as P
    torch.cuda.set_device(0)
    table, meas = {}, []
    for prec in precisions:
        rows = []
        for n in sizes:
            Xd = torch.from_numpy(_problem(n)).cuda()
            A = P.gp_assemble(Xd, 1.0, 1.0, 0.1, full=False)
            best = None
            for tile in tiles:
                for w in widths:
                    if tile == 64 and n > 4096:
                        continue  # the 64-tile update has no matrix-core path
                    ms = time_factor(P, torch, A, prec, tile, w, reps)
                    meas.append({"precision": prec, "n": n, "tile": tile, "panel_width": w, "ms": ms})
                    if best is None or ms < best[0]:
                        best = (ms, tile, w)
            rows.append([n, best[1], best[2]])
            print(f"{prec} n={n}: tile={best[1]} panel_width={best[2]} {best[0]:.3f} ms", flush=True)
            del A, Xd
            torch.cuda.empty_cache()
        table[prec] = rows
    return table, meas


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning",
                                                  "mi355x_gfx950.json"))
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sizes", type=int, nargs="*", default=list(SIZES))
    args = ap.parse_args()
    t0 = time.time()
    table, meas = sweep(tuple(args.sizes), reps=args.reps)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump({"arch": "gfx950", "generator": "paper_2605_13209_amd.autotune",
                   "input": "SE kernel d=8 ls=1 var=1 noise=0.1 seed 0", "table": table,
                   "measurements_ms": meas, "sweep_seconds": round(time.time() - t0, 1)}, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
