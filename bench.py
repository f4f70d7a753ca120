#!/usr/bin/env python3
"""Benchmark of the GP Cholesky solver path on one MI355X.

Default workload (headline_n65536): FP64 against mixed precision at
n = 65536, SE kernel d = 8, lengthscale 1, variance 1, noise 0.1, seed 0,
one right-hand side, A (FP64, lower triangle of a 34 GB column-major array)
and b resident in HBM before timing starts.  One "step":
  chol_factor (FP64, tile 128) -> chol_refine_solve (solve with the factor,
  certify ||x - x*|| / ||x|| <= 1e-10 from the FP64 residual), then
  chol_factor (FP32 MFMA trailing updates, FP64 diagonal blocks) ->
  chol_refine_solve (iterative refinement to the same certificate).
``value`` is n^3/3 over the FP64 factorisation time (GFLOP/s); the line also
carries both times to a certified solution, their ratio, the FP32 factor
preconditioning CG instead of IR, and (unless --no-sub) shorter runs of the
other configurations: n = 1024 latency (100 steps), n = 32768 FP64 with 1 and
16 right-hand sides, n = 131072 FP16-scaled with 8 right-hand sides, and the
Poisson serving stream (30 s of arrivals, 50 requests checked against the
oracle).

Other workloads (``--workload``) print their own line:
  fp64_n32768, fp64_n1024, fp64_n65536   FP64 factor + solves;
  mixed_n65536  FP64 vs FP32-factor + IR / PCG (older form of the headline);
  cg_n65536     the paper's CG against the Cholesky solver on the same
                system (eps 1e-6), value = n^3/3 over the CG time to solution;
  mixed_fp16_n131072, serve  (see bench_fp16, bench_serve).

The roofline object is measured live: every launch of the bulk
trailing-triangle update (the dominant kernel, update_f64_kernel<0> or
update_f32_kernel<0>) is bracketed by HIP events on the stream it runs on,
and its algorithmic flop count is summed (chol_profile_read with profile
mode 2).  The smaller panel-band launches of the same update, which run on
the lookahead stream concurrently with it, are not part of the figure.
cpu_baseline times the CPU oracle (assembly + Cholesky + solve) on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Bytes moved between L2 and the memory fabric per launch of the bulk
# (whole-trailing-triangle) update, from two rocprofv3 --pmc runs (FETCH_SIZE,
# WRITE_SIZE) over one run of the workload, each scaled by what the same
# counter reads for a plain 1 GiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).
# Keyed by (operand precision, n); valid only for the kernel source they were
# measured on, otherwise reported as null.  Algorithmic bytes per launch: each
# C tile read and written once, each panel tile read once, averaged over the
# launches of one factorisation (panel width 8; width 32 for FP16).
TRAFFIC_RECORDS = {
    ("f64", 65536): {"update_hip_sha256_16": "8c934b5e35c6ab2e", "bytes_per_launch": 3.283e10,
                     "algorithmic_bytes_per_launch": 1.131e10,
                     "source": "profiles/update_f64_kernel_traffic_n65536.md"},
    ("f64", 32768): {"update_hip_sha256_16": "8c934b5e35c6ab2e", "bytes_per_launch": 7.901e9,
                     "algorithmic_bytes_per_launch": 2.790e9,
                     "source": "profiles/update_f64_kernel_traffic_n32768.md"},
    ("f32", 65536): {"update_hip_sha256_16": "8c934b5e35c6ab2e", "bytes_per_launch": 1.708e10,
                     "algorithmic_bytes_per_launch": 5.65e9,
                     "source": "profiles/update_f32_kernel_traffic_n65536.md"},
    ("f16", 131072): {"update_hip_sha256_16": "8c934b5e35c6ab2e", "bytes_per_launch": 6.997e10,
                      "algorithmic_bytes_per_launch": 2.170e10,
                      "source": "profiles/update_f16_wide_kernel_traffic_n131072.md"},
}


# The same for the CG tile product (symv_tiles_kernel<128>) at n = 65536:
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 per launch.
CG_TRAFFIC = {"cg_hip_sha256_16": "6793051c70b70a14", "n": 65536, "bytes_per_launch": 17.49e9,
              "source": "profiles/symv_tiles_kernel_cg_n65536.md"}

METRIC = "Cholesky GFLOP/s (n^3/3) + time-to-1e-10 solve, FP64 vs mixed; p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
FP16_PEAK_TFLOPS = 2500.0  # MI355X dense FP16 matrix peak
HP = (1.0, 1.0, 0.1)      # lengthscale, variance, noise


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def cpu_baseline(n: int, hp=HP, k: int = 1):
    """Oracle pipeline (assembly + Cholesky-Crout + forward/back substitution) on the host."""
    import gp_inputs
    import oracle
    X, B = gp_inputs.gp_problem(n, d=8, k=k, seed=0)
    oracle.build()
    t0 = time.perf_counter()
    A = oracle.gp_assemble(X, *hp)
    L, info = oracle.cholesky(A)
    oracle.solve(L, B)
    dt = time.perf_counter() - t0
    assert info == 0
    return {"value": round(n ** 3 / 3 / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle gp_assemble + Cholesky-Crout + solve (k={k}) at n={n}, SE d=8, "
                      f"ls={hp[0]:g} var={hp[1]:g} noise={hp[2]:g}, seed 0: {dt:.2f} s; GFLOP/s = n^3/3 / time"}


def _headline_problem(n):
    """SE kernel d=8, lengthscale 1, variance 1, noise 0.1, seed 0; A (lower) and b resident in HBM."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    X_np, B_np = gp_inputs.gp_problem(n, d=8, k=1, seed=0)
    Xd = torch.from_numpy(X_np).cuda()
    Bd = P.to_colmajor(torch.from_numpy(B_np))
    A = P.colmajor_empty(n, n)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.gp_assemble(Xd, *HP, full=False, out=A)
    e1.record()
    e1.synchronize()
    return Xd, Bd, A, e0.elapsed_time(e1)


def _update_roofline(kms, kl, kfl, peak, dtype, n, kernel):
    if not (kl > 0 and kms > 0):
        return None
    ach = kfl / (kms * 1e-3) / 1e12
    tr = measured_traffic(n, dtype)
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "traffic": tr,
            "traffic_unit": "bytes per launch between L2 and the memory fabric (calibrated counters)",
            "algorithmic_bytes_per_launch": TRAFFIC_RECORDS[(dtype, n)]["algorithmic_bytes_per_launch"] if tr else None,
            "kernel": kernel, "launches": kl, "avg_launch_us": round(kms * 1e3 / kl, 2),
            "avg_launch_gflop": round(kfl / kl / 1e9, 4)}


def bench_headline(args):
    """FP64 against mixed precision at n = 65536 (the headline configuration).

    One step = (FP64 chol_factor -> chol_refine_solve, which solves with the
    factor and certifies ||x - x*|| / ||x|| <= 1e-10 from the FP64 residual)
    then (FP32 chol_factor -> chol_refine_solve by iterative refinement to the
    same certificate), on the same resident A and b.  value = n^3/3 over the
    FP64 factorisation time (HIP events on the caller stream, which the
    lookahead stream joins); the times to a certified solution are host wall
    times around each leg (each leg ends with the refinement's own stream
    synchronisation).  The roofline is the FP64 bulk update
    update_f64_kernel<0>, timed live per launch (profile mode 2)."""
    import torch
    import paper_2605_13209_amd as P
    n = args.n or 65536
    tile = 128
    steps, warmup = args.steps, args.warmup
    Xd, Bd, A, t_asm = _headline_problem(n)
    ws64 = torch.empty(P.chol_factor_bytes(n, "fp64", tile), dtype=torch.uint8, device="cuda")
    ws32 = torch.empty(P.chol_factor_bytes(n, "fp32", tile), dtype=torch.uint8, device="cuda")
    wsr = torch.empty(P.chol_refine_bytes(n, 1, "pcg"), dtype=torch.uint8, device="cuda")
    x64, x32 = P.colmajor_empty(n, 1), P.colmajor_empty(n, 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    lam = HP[2]
    acc = {"f64": [0.0, 0, 0.0], "f32": [0.0, 0, 0.0]}

    def leg(prec, ws, out, e0, e1, method="ir"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        F = P.chol_factor(A, prec, tile, workspace=ws, sync=False)
        e1.record()
        r = P.chol_refine_solve(F, Bd, A=A, noise=lam, tol=1e-10, method=method, out=out, workspace=wsr,
                                max_iter=30)
        t1 = time.perf_counter()
        if F.info() != 0 or not r.converged:
            raise RuntimeError(f"{prec} leg failed: info={F.info()} converged={r.converged} iters={r.iters}")
        return (t1 - t0) * 1e3, e0.elapsed_time(e1), r

    rec = {k: [] for k in ("step", "tts64", "fac64", "tts32", "fac32", "it64", "it32", "ce64", "ce32", "fb")}
    prof = not args.no_profile
    for i in range(warmup + steps):
        timed = i >= warmup
        if timed and prof:
            P.chol_profile_reset()
            P.set_option("profile", 2)
        t0 = time.perf_counter()
        tts64, f64, r64 = leg("fp64", ws64, x64, ev[0], ev[1])
        if timed and prof:
            kms, kl, kfl = P.chol_profile_read()
            acc["f64"] = [acc["f64"][0] + kms, acc["f64"][1] + kl, acc["f64"][2] + kfl]
            P.chol_profile_reset()
        tts32, f32, r32 = leg("fp32", ws32, x32, ev[2], ev[3])
        if timed and prof:
            kms, kl, kfl = P.chol_profile_read()
            acc["f32"] = [acc["f32"][0] + kms, acc["f32"][1] + kl, acc["f32"][2] + kfl]
            P.chol_profile_reset()
            P.set_option("profile", 0)
        if timed:
            rec["step"].append((time.perf_counter() - t0) * 1e3)
            rec["tts64"].append(tts64)
            rec["fac64"].append(f64)
            rec["tts32"].append(tts32)
            rec["fac32"].append(f32)
            rec["it64"].append(r64.iters)
            rec["it32"].append(r32.iters)
            rec["ce64"].append(r64.cert)
            rec["ce32"].append(r32.cert)
            rec["fb"].append(r64.fallback_used | r32.fallback_used)
    P.set_option("profile", 0)
    # the FP32 factor with the paper's other solver preconditioned by it (two runs, not in the step)
    pcg = []
    for _ in range(2):
        pcg.append(leg("fp32", ws32, x32, ev[2], ev[3], method="pcg"))
    flops = n ** 3 / 3
    m = lambda k: float(np.mean(rec[k]))
    tts64, tts32 = m("tts64"), m("tts32")
    value = flops / (m("fac64") * 1e-3) / 1e9
    out = {"metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(m("step"), 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"fp64_vs_mixed_cholesky_solve_n{n}", "n": n, "tile": tile, "rhs": 1,
                      "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1", "seed": 0, "tol": 1e-10,
                      "panel_width": P.get_option("panel_width"), "lookahead": P.get_option("lookahead"),
                      "value_is": "n^3/3 / FP64 factorisation time",
                      "step_is": "FP64 factor + certified solve, then FP32 factor + IR to the same certificate"},
           "roofline": _update_roofline(*acc["f64"], FP64_PEAK_TFLOPS, "f64", n,
                                        "update_f64_kernel<0> (Step-3 update of the trailing triangle)"),
           "fp64": {"factor_ms": round(m("fac64"), 2), "factor_gflops": round(value, 1),
                    "factor_frac_fp64_peak": round(value / (FP64_PEAK_TFLOPS * 1e3), 4),
                    "factor_p50_ms": round(percentile(rec["fac64"], 50), 2),
                    "factor_p99_ms": round(percentile(rec["fac64"], 99), 2),
                    "time_to_solution_ms": round(tts64, 2), "tts_p50_ms": round(percentile(rec["tts64"], 50), 2),
                    "tts_p99_ms": round(percentile(rec["tts64"], 99), 2),
                    "corrections": int(max(rec["it64"])), "cert": float(max(rec["ce64"]))},
           "fp32_ir": {"factor_ms": round(m("fac32"), 2),
                       "factor_gflops": round(flops / (m("fac32") * 1e-3) / 1e9, 1),
                       "time_to_solution_ms": round(tts32, 2), "tts_p50_ms": round(percentile(rec["tts32"], 50), 2),
                       "tts_p99_ms": round(percentile(rec["tts32"], 99), 2),
                       "corrections": int(max(rec["it32"])), "cert": float(max(rec["ce32"])),
                       "roofline": _update_roofline(*acc["f32"], FP32_PEAK_TFLOPS, "f32", n,
                                                    "update_f32_kernel<0> (Step-3 update of the trailing triangle)")},
           "fp32_pcg": {"time_to_solution_ms": round(float(np.mean([p[0] for p in pcg])), 2),
                        "iterations": int(max(p[2].iters for p in pcg)), "cert": float(max(p[2].cert for p in pcg))},
           "speedup_mixed_vs_fp64": round(tts64 / tts32, 3),
           "fallbacks": int(max(rec["fb"])),
           "assemble_ms": round(t_asm, 3),
           "certificate": "||b - A x||_2 / (noise ||x||_2) <= tol / 2 bounds ||x - x*|| / ||x|| "
                          "(lambda_min(A) >= noise)"}
    del ws64, ws32, wsr, A
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline_n65536",
                    choices=["headline_n65536", "fp64_n32768", "fp64_n1024", "fp64_n65536", "mixed_n65536",
                             "mixed_fp16_n131072", "serve", "cg_n65536", "hetero", "cg_hetero"])
    ap.add_argument("--shares", default="1.0,0.999,0.997,0.995,0.99,0.98,0.95,0.9",
                    help="hetero: GPU shares of the Step-3 tiles to sweep")
    ap.add_argument("--no-sub", action="store_true",
                    help="headline: skip the other configurations' summaries (n = 1024, 32768, 131072, serving)")
    ap.add_argument("--duration", type=float, default=30.0, help="serve: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: mean arrivals per second")
    ap.add_argument("--workers", type=int, default=8, help="serve: concurrent requests")
    ap.add_argument("--oracle-sample", type=int, default=50, help="serve: requests checked against the oracle")
    ap.add_argument("--serve-executor", default="batched", choices=["batched", "streams"],
                    help="serve: continuous batching of the factorisations (one graph-captured column step "
                         "for all active requests) or one stream and launch chain per request")
    ap.add_argument("--n", type=int, default=0, help="override the order")
    ap.add_argument("--tile", type=int, default=128)
    ap.add_argument("--panel-width", type=int, default=0)
    ap.add_argument("--lookahead", type=int, default=-1)
    ap.add_argument("--super-tile", type=int, default=0)
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="order of the CPU oracle sample (0: 12288 for Cholesky, 10240 for CG)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--cg-max-iter", type=int, default=0,
                    help="cg_n65536: cap the CG iterations (profiling runs; 0 = run to eps)")
    ap.add_argument("--no-cholesky", action="store_true", help="cg_n65536: skip the Cholesky comparison")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="before the workload, one plain device copy of this many GiB (outside the "
                         "timed region): the known-size kernel that calibrates byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)

    import torch
    import paper_2605_13209_amd as P

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_gib > 0:
        src = torch.ones(int(args.copy_probe_gib * (1 << 27)), dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.panel_width:
        P.set_option("panel_width", args.panel_width)
    if args.lookahead >= 0:
        P.set_option("lookahead", args.lookahead)
    if args.super_tile:
        P.set_option("super_tile", args.super_tile)

    wl = args.workload
    if wl == "serve":
        out = bench_serve(args)
    elif wl == "mixed_fp16_n131072":
        out = bench_fp16(args)
    elif wl == "cg_n65536":
        out = bench_cg(args)
    elif wl == "hetero":
        out = bench_hetero(args)
    elif wl == "cg_hetero":
        out = bench_cg_hetero(args)
    elif wl == "headline_n65536":
        out = bench_headline(args)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.cpu_n or 12288)
        if not args.no_sub:
            out["other_configs"] = other_configs(args)
    else:
        out = bench_chol(args)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.cpu_n or 12288)
    print(json.dumps(out), flush=True)


def other_configs(args):
    """Shorter runs of the other configurations, one summary each (same
    format as their own bench lines); a failure is reported, not raised."""
    import copy
    import torch
    res = {}
    for name, fn, kw in (("fp64_n1024", bench_chol, {"workload": "fp64_n1024", "n": 0}),
                         ("fp64_n32768", bench_chol, {"workload": "fp64_n32768", "n": 0, "steps": 3, "warmup": 1}),
                         ("mixed_fp16_n131072", bench_fp16, {"n": 0, "steps": 3, "warmup": 1}),
                         ("serve", bench_serve, {"n": 0})):
        a = copy.copy(args)
        a.steps, a.warmup = 10, 2
        for k, v in kw.items():
            setattr(a, k, v)
        print(f"bench: {name}", file=sys.stderr, flush=True)
        try:
            r = fn(a)
            if name == "fp64_n1024" and not args.no_cpu_baseline:
                r["cpu_baseline"] = cpu_baseline(1024)
            if name == "fp64_n32768" and not args.no_cpu_baseline:
                r["cpu_baseline"] = "the headline's cpu_baseline (same matrix family, Cholesky + solve)"
        except Exception as e:  # noqa: BLE001 - reported in the line
            r = {"error": f"{type(e).__name__}: {e}"}
        for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            r.pop(k, None)
        res[name] = r
        torch.cuda.empty_cache()
    return res


def bench_chol(args):
    """FP64 factorisation + solves: fp64_n32768 (k = 1 and 16), fp64_n1024
    (the latency case, k = 1, 100 steps), fp64_n65536, mixed_n65536 (the
    older FP64 vs FP32 + IR / PCG line)."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    wl = args.workload
    n = args.n or {"fp64_n32768": 32768, "fp64_n1024": 1024, "fp64_n65536": 65536, "mixed_n65536": 65536}[wl]
    tile = args.tile
    steps, warmup = args.steps, args.warmup
    if wl == "fp64_n1024" and steps == 10:
        steps, warmup = 100, 5

    X_np, B_np = gp_inputs.gp_problem(n, d=8, k=16, seed=0)
    Xd = torch.from_numpy(X_np).cuda()
    B16_src = P.to_colmajor(torch.from_numpy(B_np))
    B1_src = B16_src[:, :1]
    A = P.colmajor_empty(n, n)
    extra = {}
    prof_mode = 2

    if wl.startswith("fp64"):
        ws = torch.empty(P.chol_factor_bytes(n, "fp64", tile), dtype=torch.uint8, device="cuda")
        b1 = P.colmajor_empty(n, 1)
        b16 = P.colmajor_empty(n, 16)
        with_16 = wl != "fp64_n65536"
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]

        def step():
            ev[0].record()
            P.gp_assemble(Xd, *HP, full=False, out=A)
            ev[1].record()
            F = P.chol_factor(A, "fp64", tile, workspace=ws, sync=False)
            ev[2].record()
            b1.copy_(B1_src)
            P.chol_solve(F, b1)
            ev[3].record()
            if with_16:
                b16.copy_(B16_src)
                P.chol_solve(F, b16)
            ev[4].record()
            return F

        for _ in range(warmup):
            F = step()
        torch.cuda.synchronize()
        if warmup and F.info() != 0:
            raise RuntimeError(f"factorisation failed, info={F.info()}")
        P.chol_profile_reset()
        if not args.no_profile:
            # small orders are one panel (no whole-triangle launches): time every update launch
            prof_mode = 1 if n < 192 * tile else 2
            P.set_option("profile", prof_mode)
        t_step, t_asm, t_fac, t_s1, t_s16 = [], [], [], [], []
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        for _ in range(steps):
            F = step()
            ev[4].synchronize()
            t_asm.append(ev[0].elapsed_time(ev[1]))
            t_fac.append(ev[1].elapsed_time(ev[2]))
            t_s1.append(ev[2].elapsed_time(ev[3]))
            t_s16.append(ev[3].elapsed_time(ev[4]))
            t_step.append(ev[0].elapsed_time(ev[4]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        P.set_option("profile", 0)
        info = F.info()
        if info != 0:
            raise RuntimeError(f"factorisation failed, info={info}")
        # certificate of the k=1 solve: ||b - A x|| / (noise ||x||) bounds the relative error
        R = P.chol_residual(A, b1, B1_src)
        cert = float(torch.linalg.norm(R) / (HP[2] * torch.linalg.norm(b1)))
        flops = n ** 3 / 3
        ms_step = float(np.mean(t_step))
        value = flops / (ms_step * 1e-3) / 1e9
        extra.update({
            "factor_gflops": round(flops / (np.mean(t_fac) * 1e-3) / 1e9, 1),
            "factor_frac_fp64_peak": round(flops / (np.mean(t_fac) * 1e-3) / (FP64_PEAK_TFLOPS * 1e12), 4),
            "ms": {"assemble": round(float(np.mean(t_asm)), 3), "factor": round(float(np.mean(t_fac)), 3),
                   "solve_k1": round(float(np.mean(t_s1)), 3),
                   "solve_k16": round(float(np.mean(t_s16)), 3) if with_16 else None},
            "p50_ms": round(percentile(t_step, 50), 3), "p99_ms": round(percentile(t_step, 99), 3),
            "factor_p50_ms": round(percentile(t_fac, 50), 3), "factor_p99_ms": round(percentile(t_fac, 99), 3),
            "solve_cert_k1": cert, "wall_s": round(wall, 3),
            "solve_k1_gbps": round(chol_bytes(n, tile, 8) * 2 / (np.mean(t_s1) * 1e-3) / 1e9, 1),
        })
        launch = "direct"
        if wl == "fp64_n1024":
            # the latency case again with the factorisation replayed from a captured HIP
            # graph (option graph; capture needs a stream other than the legacy default one)
            gstream = torch.cuda.Stream()
            P.set_option("graph", 1)
            try:
                with torch.cuda.stream(gstream):
                    for _ in range(warmup):
                        F = step()
                    gstream.synchronize()
                    g_step, g_fac = [], []
                    for _ in range(steps):
                        F = step()
                        ev[4].synchronize()
                        g_fac.append(ev[1].elapsed_time(ev[2]))
                        g_step.append(ev[0].elapsed_time(ev[4]))
                    gstream.synchronize()
                    info = F.info()
                    Rg = P.chol_residual(A, b1, B1_src)
                    gstream.synchronize()
            finally:
                P.set_option("graph", 0)
            if info != 0:
                raise RuntimeError(f"graph-replayed factorisation failed, info={info}")
            g_cert = float(torch.linalg.norm(Rg) / (HP[2] * torch.linalg.norm(b1)))
            extra["direct_launches"] = {"ms_per_step": round(ms_step, 3), "p50_ms": extra["p50_ms"],
                                        "p99_ms": extra["p99_ms"], "factor_ms": extra["ms"]["factor"]}
            extra["graph"] = {"ms_per_step": round(float(np.mean(g_step)), 3),
                              "p50_ms": round(percentile(g_step, 50), 3),
                              "p99_ms": round(percentile(g_step, 99), 3),
                              "factor_ms": round(float(np.mean(g_fac)), 3),
                              "factor_p50_ms": round(percentile(g_fac, 50), 3),
                              "solve_cert_k1": g_cert}
            if float(np.mean(g_step)) < ms_step:  # the line reports the faster launch mode
                launch = "hip_graph"
                ms_step = float(np.mean(g_step))
                value = flops / (ms_step * 1e-3) / 1e9
                extra.update({"p50_ms": extra["graph"]["p50_ms"], "p99_ms": extra["graph"]["p99_ms"],
                              "factor_p50_ms": extra["graph"]["factor_p50_ms"],
                              "factor_gflops": round(flops / (np.mean(g_fac) * 1e-3) / 1e9, 1),
                              "factor_frac_fp64_peak": round(flops / (np.mean(g_fac) * 1e-3)
                                                             / (FP64_PEAK_TFLOPS * 1e12), 4)})
                extra["ms"]["factor"] = extra["graph"]["factor_ms"]
        dtype = "f64"
        peak = FP64_PEAK_TFLOPS
        config = {"workload": f"fp64_cholesky_solve_n{n}", "n": n, "tile": tile,
                  "panel_width": P.get_option("panel_width"), "lookahead": P.get_option("lookahead"),
                  "rhs": [1, 16] if with_16 else [1], "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1",
                  "seed": 0, "precision": "fp64", "launch": launch}
    else:  # mixed_n65536: time to a certified 1e-10 solution, FP64 vs FP32 + IR / PCG
        P.gp_assemble(Xd, *HP, full=False, out=A)
        res = {}
        b = P.colmajor_empty(n, 1)
        for prec, method in (("fp64", "ir"), ("fp32", "ir"), ("fp32", "pcg")):
            ws = torch.empty(P.chol_factor_bytes(n, prec, tile), dtype=torch.uint8, device="cuda")
            ts, tf, it, ce = [], [], [], []
            for rep in range(warmup + steps):
                torch.cuda.synchronize()
                if rep == warmup and not args.no_profile and prec == "fp32" and method == "ir":
                    P.chol_profile_reset()
                    P.set_option("profile", 2)
                t0 = time.perf_counter()
                F = P.chol_factor(A, prec, tile, workspace=ws, sync=False)
                torch.cuda.synchronize()
                tm = time.perf_counter()
                r = P.chol_refine_solve(F, B1_src, A=A, noise=HP[2], tol=1e-10, method=method, out=b)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                if rep >= warmup:
                    ts.append((t1 - t0) * 1e3)
                    tf.append((tm - t0) * 1e3)
                    it.append(r.iters)
                    ce.append(r.cert)
                del F
            if prec == "fp32" and method == "ir":
                P.set_option("profile", 0)
            res[f"{prec}_{method}"] = {"time_to_solution_ms": round(float(np.mean(ts)), 2),
                                       "factor_ms": round(float(np.mean(tf)), 2),
                                       "iters": int(max(it)), "cert": float(max(ce)),
                                       "p50_ms": round(percentile(ts, 50), 2), "p99_ms": round(percentile(ts, 99), 2)}
            del ws
            torch.cuda.empty_cache()
        flops = n ** 3 / 3
        best_mixed = min(res["fp32_ir"]["time_to_solution_ms"], res["fp32_pcg"]["time_to_solution_ms"])
        ms_step = best_mixed
        value = flops / (best_mixed * 1e-3) / 1e9  # n^3/3 over the whole time to a certified solution
        extra.update({"solutions": res,
                      "speedup_mixed_vs_fp64": round(res["fp64_ir"]["time_to_solution_ms"] / best_mixed, 3)})
        dtype = "f32"
        peak = FP32_PEAK_TFLOPS
        config = {"workload": f"mixed_fp32_ir_n{n}", "n": n, "tile": tile, "rhs": [1],
                  "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1", "seed": 0, "tol": 1e-10}

    kms, kl, kfl = P.chol_profile_read()
    kernel = (("update_f64_kernel" if dtype == "f64" else "update_f32_kernel")
              + ("<0> (Step-3 update of the trailing triangle)" if prof_mode == 2 else " (every Step-3 update launch)"))
    roofline = _update_roofline(kms, kl, kfl, peak, dtype, n, kernel)
    out = {"metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
           "roofline": roofline}
    out.update(extra)
    return out


def bench_hetero(args):
    """The paper's heterogeneous CPU + GPU Cholesky against the GPU alone:
    SE kernel d=8, lengthscale 1, variance 1, noise 0.1, seed 0, FP64, tile
    128, A resident in HBM.  For each GPU share of the Step-3 tiles in
    --shares, chol_factor_hetero is timed (wall time of the synchronous call,
    host <-> device copies of the CPU's rows included); the GPU-alone line is
    chol_factor with its tuned schedule (panel width 8, lookahead).  value =
    n^3/3 over the best heterogeneous time."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    n = args.n or 32768
    steps = args.steps if args.steps != 10 else 2
    X_np, B_np = gp_inputs.gp_problem(n, d=8, k=1, seed=0)
    Xd = torch.from_numpy(X_np).cuda()
    Bd = P.to_colmajor(torch.from_numpy(B_np))
    A = P.colmajor_empty(n, n)
    P.gp_assemble(Xd, *HP, full=False, out=A)
    ws = torch.empty(P.chol_factor_bytes(n, "fp64", 128), dtype=torch.uint8, device="cuda")
    host_ws = torch.empty(P.chol_hetero_host_bytes(n), dtype=torch.uint8, pin_memory=True)
    flops = n ** 3 / 3

    def timed(fn):
        ts = []
        for r in range(1 + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            if r >= 1:
                ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.mean(ts)), res

    t_gpu, F = timed(lambda: P.chol_factor(A, "fp64", 128, workspace=ws))
    curve = []
    for share in [float(v) for v in args.shares.split(",")]:
        t, (F, rep) = timed(lambda: P.chol_factor_hetero(A, share, workspace=ws, host_ws=host_ws))
        b = P.colmajor_empty(n, 1)
        b.copy_(Bd)
        P.chol_solve(F, b)
        R = P.chol_residual(A, b, Bd)
        cert = float(torch.linalg.norm(R) / (HP[2] * torch.linalg.norm(b)))
        curve.append({"gpu_share": share, "ms": round(t, 2), "gflops": round(flops / (t * 1e-3) / 1e9, 1),
                      "gpu_share_tiles": round(rep["gpu_share_tiles"], 5),
                      "border_shifts": rep["border_shifts"], "handover_column": rep["handover_column"],
                      "ms_cpu": round(rep["ms_cpu"], 1), "ms_wait_gpu": round(rep["ms_wait_gpu"], 1),
                      "gb_h2d": round(rep["bytes_h2d"] / 1e9, 3), "gb_d2h": round(rep["bytes_d2h"] / 1e9, 3),
                      "cpu_threads": rep["cpu_threads"], "solve_cert": cert})
        print(f"bench: hetero n={n} share={share} {t:.1f} ms", file=sys.stderr, flush=True)
    best = min(curve, key=lambda c: c["ms"])
    out = {"metric": METRIC, "value": best["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": steps,
           "warmup": 1, "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"hetero_cpu_gpu_cholesky_n{n}", "n": n, "tile": 128, "panel_width": 8,
                      "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1", "seed": 0,
                      "value_is": "n^3/3 / best heterogeneous factorisation time (copies included)"},
           "roofline": None,
           "gpu_only": {"ms": round(t_gpu, 2), "gflops": round(flops / (t_gpu * 1e-3) / 1e9, 1),
                        "schedule": "chol_factor: panel width 8, lookahead"},
           "best_share": best["gpu_share"],
           "hetero_gain_vs_gpu_only": round((t_gpu - best["ms"]) / t_gpu, 4),
           "curve": curve}
    del host_ws
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n or 12288)
    return out


def bench_cg_hetero(args):
    """The paper's heterogeneous CG against the GPU alone (its CG workload:
    eps = 1e-6, recomputation every 50 iterations, no iteration cap): SE
    kernel d=8, lengthscale 1, variance 1, noise 0.1, n = 65536, one
    right-hand side, A resident in HBM.  For each GPU share of the stored
    tiles in --shares, cg_solve_hetero is timed (packing and the copies of
    the CPU's tiles included, as cg_solve packs too); the GPU-alone line is
    cg_solve.  value = n^3/3 over the best heterogeneous time (the unit of
    the Cholesky lines)."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    n = args.n or 65536
    eps, recompute = 1e-6, 50
    steps = args.steps if args.steps != 10 else 2
    X, B = gp_inputs.gp_problem(n, d=8, k=1, seed=0)
    Xd = torch.from_numpy(X).cuda()
    Bd = P.to_colmajor(torch.from_numpy(B))
    A = P.colmajor_empty(n, n)
    P.gp_assemble(Xd, *HP, full=False, out=A)
    shares = [float(v) for v in (args.shares if args.shares != "1.0,0.999,0.997,0.995,0.99,0.98,0.95,0.9"
                                 else "1.0,0.995,0.99,0.98,0.97,0.95").split(",")]
    ws = torch.empty(max(P.cg_workspace_bytes(n, 1, 128), P.lib().cg_hetero_workspace_bytes(n)),
                     dtype=torch.uint8, device="cuda")
    host_ws = torch.empty(max(P.lib().cg_hetero_host_bytes(n, s) for s in shares), dtype=torch.uint8,
                          pin_memory=True)
    Xs = P.colmajor_empty(n, 1)

    def timed(fn):
        ts, res = [], None
        for r in range(1 + steps):
            Xs.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            if r >= 1:
                ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.mean(ts)), res

    t_gpu, g = timed(lambda: P.cg_solve(A, Bd, X=Xs, eps=eps, max_iter=100000, recompute=recompute, tile=128,
                                        workspace=ws))
    curve = []
    for share in shares:
        t, (x, it, rr, conv, rep) = timed(lambda: P.cg_solve_hetero(A, Bd[:, 0], share, X=Xs[:, 0], eps=eps,
                                                                    max_iter=100000, recompute=recompute,
                                                                    workspace=ws, host_ws=host_ws))
        R = P.chol_residual(A, Xs, Bd)
        curve.append({"gpu_share": share, "ms": round(t, 2), "iterations": it, "converged": conv,
                      "ms_per_iteration": round(t / max(it, 1), 4),
                      "gpu_share_tiles": round(rep["gpu_share_tiles"], 5), "gpu_rows": rep["gpu_rows"],
                      "ms_cpu": round(rep["ms_cpu"], 1), "ms_wait_gpu": round(rep["ms_wait_gpu"], 1),
                      "gb_h2d": round(rep["bytes_h2d"] / 1e9, 3), "gb_d2h": round(rep["bytes_d2h"] / 1e9, 3),
                      "relres_true": float(torch.linalg.norm(R) / torch.linalg.norm(Bd)),
                      "cpu_threads": rep["cpu_threads"]})
        print(f"bench: cg hetero n={n} share={share} {t:.1f} ms, {it} iterations", file=sys.stderr, flush=True)
    best = min(curve, key=lambda c: c["ms"])
    out = {"metric": METRIC, "value": round(n ** 3 / 3 / (best["ms"] * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
           "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": best["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"hetero_cpu_gpu_cg_n{n}", "n": n, "tile": 128, "rhs": 1, "eps": eps,
                      "recompute": recompute, "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1", "seed": 0,
                      "value_is": "n^3/3 / best heterogeneous CG time to solution"},
           "roofline": None,
           "gpu_only": {"ms": round(t_gpu, 2), "iterations": int(g.iters[0]),
                        "ms_per_iteration": round(t_gpu / max(g.iters[0], 1), 4)},
           "best_share": best["gpu_share"], "hetero_gain_vs_gpu_only": round((t_gpu - best["ms"]) / t_gpu, 4),
           "curve": curve}
    del host_ws
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_cg(args.cpu_n or 10240, eps)
    return out


def cpu_baseline_cg(n: int, eps: float):
    """The oracle's CG (assembled A, long-double products) on the host."""
    import gp_inputs
    import oracle
    X, B = gp_inputs.gp_problem(n, d=8, k=1, seed=0)
    oracle.build()
    t0 = time.perf_counter()
    A = oracle.gp_assemble(X, *HP)
    x, it, rr, stopped = oracle.cg(A, B, eps=eps, max_iter=100000, recompute=50)
    dt = time.perf_counter() - t0
    assert stopped == 0
    return {"value": round(n ** 3 / 3 / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle gp_assemble + CG (eps {eps:g}, recompute 50) at n={n}, SE d=8, ls=1 var=1 "
                      f"noise=0.1, seed 0: {int(it[0])} iterations, {dt:.2f} s; "
                      f"GFLOP/s-equivalent = n^3/3 / time"}


def bench_cg(args):
    """The paper's CG against its Cholesky solver on the same system (its
    CG/Cholesky comparison: eps = 1e-6, no iteration cap, the Cholesky time
    including the forward and back substitution): SE kernel d=8, lengthscale 1,
    variance 1, noise 0.1, n = 65536, one right-hand side, seed 0.  A is
    resident in HBM (column-major, lower triangle) before timing starts.
    value = n^3/3 over the CG time to solution, the unit of the Cholesky
    lines, so the two compare directly."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    n = args.n or 65536
    eps, recompute = 1e-6, 50
    X, B = gp_inputs.gp_problem(n, d=8, k=1, seed=0)
    Xd = torch.from_numpy(X).cuda()
    Bd = P.to_colmajor(torch.from_numpy(B))
    A = P.colmajor_empty(n, n)
    P.gp_assemble(Xd, *HP, full=False, out=A)
    ws = torch.empty(P.cg_workspace_bytes(n, 1, 128), dtype=torch.uint8, device="cuda")
    Xs = P.colmajor_empty(n, 1)
    steps, warmup = args.steps, args.warmup
    if steps == 10:
        steps = 3
    t_cg, its, rrs = [], [], []
    for rep in range(warmup + steps):
        Xs.zero_()
        torch.cuda.synchronize()
        if rep == warmup and not args.no_profile:
            P.chol_profile_reset()
            P.set_option("profile", 2)
        t0 = time.perf_counter()
        res = P.cg_solve(A, Bd, X=Xs, eps=eps, max_iter=args.cg_max_iter or 100000, recompute=recompute,
                         tile=128, workspace=ws)
        t1 = time.perf_counter()
        if not res.converged and not args.cg_max_iter:
            raise RuntimeError(f"CG did not converge: {res}")
        if rep >= warmup:
            t_cg.append((t1 - t0) * 1e3)
            its.append(res.iters[0])
            rrs.append(res.relres[0])
    P.set_option("profile", 0)
    kms, kl, kbytes = P.chol_profile_read()
    R = P.chol_residual(A, Xs, Bd)
    true_rel = float(torch.linalg.norm(R) / torch.linalg.norm(Bd))
    del ws
    torch.cuda.empty_cache()

    # the Cholesky solver on the same system: FP64 factor + forward/back substitution
    wsf = torch.empty(P.chol_factor_bytes(n, "fp64", 128), dtype=torch.uint8, device="cuda")
    b1 = P.colmajor_empty(n, 1)
    t_ch = []
    for rep in range(0 if args.no_cholesky else 1 + max(1, steps // 2)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = P.chol_factor(A, "fp64", 128, workspace=wsf, sync=False)
        b1.copy_(Bd)
        P.chol_solve(F, b1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if rep >= 1:
            t_ch.append((t1 - t0) * 1e3)
        if F.info() != 0:
            raise RuntimeError("factorisation failed")
    chol_rel = None
    if t_ch:
        Rc = P.chol_residual(A, b1, Bd)
        chol_rel = float(torch.linalg.norm(Rc) / torch.linalg.norm(Bd))

    ms = float(np.mean(t_cg))
    flops = n ** 3 / 3
    roofline = None
    if kl > 0 and kms > 0:
        ach = kbytes / (kms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": 8000.0, "unit": "GB/s",
                    "frac": round(ach / 8000.0, 4), "traffic": measured_cg_traffic(n),
                    "traffic_unit": "bytes per launch between L2 and the memory fabric (calibrated counters)",
                    "kernel": "symv_tiles_kernel<128> (both products of every stored tile, one pass over "
                              "the packed lower triangle)",
                    "launches": kl, "avg_launch_us": round(kms * 1e3 / kl, 2),
                    "algorithmic_bytes_per_launch": round(kbytes / kl)}
    out = {"metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"cg_vs_cholesky_n{n}", "n": n, "tile": 128, "rhs": 1, "eps": eps,
                      "recompute": recompute, "kernel": "SE d=8 lengthscale=1 variance=1 noise=0.1",
                      "seed": 0, "value_is": "n^3/3 / CG time to solution"},
           "roofline": roofline,
           "cg": {"time_to_solution_ms": round(ms, 2), "p50_ms": round(percentile(t_cg, 50), 2),
                  "p99_ms": round(percentile(t_cg, 99), 2), "iterations": int(max(its)),
                  "ms_per_iteration": round(ms / max(its), 4), "relres_recurrence": float(max(rrs)),
                  "relres_true": true_rel},
           "cholesky": {"time_to_solution_ms": round(float(np.mean(t_ch)), 2) if t_ch else None,
                        "relres_true": chol_rel},
           "speedup_cg_vs_cholesky": round(float(np.mean(t_ch)) / ms, 3) if t_ch else None}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_cg(args.cpu_n or 10240, eps)
    return out


def bench_fp16(args):
    """FP16 trailing updates with diagonal scaling (FP32 factor storage), FP64
    refinement to a certified 1e-10: SE kernel d=8, lengthscale 0.5, variance 1,
    noise 1, 8 right-hand sides, seed 0.  A is assembled in FP64 (lower part of
    a full n x n array: 137 GB at n = 131072) and used for the residuals."""
    import torch
    import gp_inputs
    import paper_2605_13209_amd as P
    n = args.n or 131072
    tile, k = 128, 8
    hp = (0.5, 1.0, 1.0)
    X, B = gp_inputs.gp_problem(n, d=8, k=k, seed=0)
    Xd = torch.from_numpy(X).cuda()
    Bd = P.to_colmajor(torch.from_numpy(B))
    A = P.colmajor_empty(n, n)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.gp_assemble(Xd, *hp, full=False, out=A)
    e1.record()
    e1.synchronize()
    t_asm = e0.elapsed_time(e1)
    ws = torch.empty(P.chol_factor_bytes(n, "fp16_scaled", tile), dtype=torch.uint8, device="cuda")
    xs = P.colmajor_empty(n, k)
    ts, tf, it, ce, fb = [], [], [], [], []
    for rep in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        if rep == args.warmup and not args.no_profile:
            P.chol_profile_reset()
            P.set_option("profile", 2)
        t0 = time.perf_counter()
        F = P.chol_factor(A, "fp16_scaled", tile, workspace=ws, sync=False)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        r = P.chol_refine_solve(F, Bd, A=A, noise=hp[2], tol=1e-10, method="ir", max_iter=60, out=xs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if F.info() != 0 or not r.converged:
            raise RuntimeError(f"fp16 path failed: info={F.info()} converged={r.converged} iters={r.iters}")
        if rep >= args.warmup:
            ts.append((t1 - t0) * 1e3)
            tf.append((tm - t0) * 1e3)
            it.append(r.iters)
            ce.append(r.cert)
            fb.append(r.fallback_used)
        del F
    P.set_option("profile", 0)
    flops = n ** 3 / 3
    ms = float(np.mean(ts))
    roofline = None
    kms, kl, kfl = P.chol_profile_read()
    if kl > 0 and kms > 0:
        ach = kfl / (kms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP16_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / FP16_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic(n, "f16"),
                    "traffic_unit": "bytes per launch between L2 and the memory fabric (calibrated counters)",
                    "algorithmic_bytes_per_launch": TRAFFIC_RECORDS[("f16", n)]["algorithmic_bytes_per_launch"]
                    if measured_traffic(n, "f16") else None,
                    "kernel": "update_f16_wide_kernel (Step-3 update of the trailing triangle, 2 x 2 tiles per workgroup)",
                    "launches": kl, "avg_launch_us": round(kms * 1e3 / kl, 2),
                    "avg_launch_gflop": round(kfl / kl / 1e9, 4)}
    out = {"metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f16+f32+f64", "data": "synthetic",
                      "config": {"workload": f"mixed_fp16_n{n}", "n": n, "tile": tile, "rhs": k,
                                 "kernel": "SE d=8 lengthscale=0.5 variance=1 noise=1", "seed": 0,
                                 "tol": 1e-10, "precision": "fp16 trailing updates (scaled) + fp32 storage"
                                                           " + fp64 IR"},
                      "roofline": roofline,
                      "ms": {"assemble": round(t_asm, 3), "factor": round(float(np.mean(tf)), 2),
                             "time_to_solution": round(ms, 2)},
                      "factor_gflops": round(flops / (np.mean(tf) * 1e-3) / 1e9, 1),
                      "iters": int(max(it)), "cert": float(max(ce)), "fallbacks": int(max(fb))}
    del A, ws
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        # the oracle cannot hold this matrix (137 GB); it is timed on a bounded
        # sample of the same family (FP64 Cholesky + solve with 8 right-hand sides)
        out["cpu_baseline"] = cpu_baseline(8192, hp=hp, k=k)
    return out


def measured_traffic(n: int, dtype: str):
    """Counter-measured bytes per launch of the bulk update (dtype f64, f32 or
    f16: the update's operand precision), or None when no record covers this
    order or the kernel source differs from the one the counters saw."""
    import hashlib
    rec = TRAFFIC_RECORDS.get((dtype, n))
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2605_13209_amd", "csrc", "update.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if h != rec["update_hip_sha256_16"]:
        return None
    return rec["bytes_per_launch"]


def measured_cg_traffic(n: int):
    """Counter-measured bytes per CG tile-product launch, or None when the
    order or the kernel source differs from the one the counters saw."""
    import hashlib
    src = os.path.join(ROOT, "paper_2605_13209_amd", "csrc", "cg.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if n != CG_TRAFFIC["n"] or h != CG_TRAFFIC["cg_hip_sha256_16"]:
        return None
    return CG_TRAFFIC["bytes_per_launch"]


def bench_serve(args):
    """Poisson stream of GP solves replayed in real time against the server
    (mean 200 requests/s, n = round(exp(U[ln 256, ln 8192])), 1-64 right-hand
    sides, lengthscale U[0.3, 2], noise U[0.01, 1], a quarter of the requests
    repeating a recent matrix; FP32 factor + FP64 refinement to a certified
    1e-10; HBM budget 200 GB).  A seeded sample of the completed requests is
    then checked against the oracle's refined FP64 solution, which also
    times the oracle per request (the CPU baseline)."""
    import torch
    import gp_inputs
    import oracle
    from paper_2605_13209_amd.serve import BatchedHipExecutor, HipExecutor, Server, SolveRequest
    stream = gp_inputs.serving_stream(duration_s=args.duration, rate=args.rate, seed=0)

    def to_req(r):
        return SolveRequest(X=r.features(), B=r.rhs(), lengthscale=r.lengthscale, variance=1.0,
                            noise=r.noise, key=r.key, rid=r.rid, tol=1e-10)

    if args.serve_executor == "batched":
        ex = BatchedHipExecutor(method="ir", workers=args.workers)
    else:
        ex = HipExecutor(precision="fp32", method="ir", workers=args.workers)
    with Server(ex, hbm_budget=200e9, max_inflight=args.workers) as srv:  # warm-up, not timed
        for f in [srv.submit(to_req(r)) for r in gp_inputs.serving_stream(duration_s=0.1, seed=1)[:8]]:
            f.result()
    torch.cuda.synchronize()
    pending = [to_req(r) for r in stream]  # host-side inputs prepared before the clock starts
    srv = Server(ex, hbm_budget=200e9, max_inflight=args.workers)
    futs = []
    t0 = time.perf_counter()
    for rq, r in zip(pending, stream):
        delay = t0 + r.arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        rq.t_arrival = time.perf_counter()
        futs.append(srv.submit(rq))
    results = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    if args.serve_executor == "batched":
        st["engine_steps"] = ex.steps
        ex.close()
    offered = sum(r.n ** 3 / 3 + 4.0 * r.n * r.n * r.k for r in stream) / args.duration / 1e12
    achieved = st["gflops"] / 1e3 if st["gflops"] else 0.0
    out = {"metric": METRIC, "value": round(st["gflops"], 2), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": len(futs), "warmup": 8, "ms_per_step": round(wall * 1e3 / max(1, len(futs)), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "serve_poisson", "rate_per_s": args.rate, "duration_s": args.duration,
                      "n": "round(exp(U[ln 256, ln 8192]))", "rhs": "U{1..64}", "lengthscale": "U[0.3,2]",
                      "noise": "U[0.01,1]", "repeat_keys": 0.25, "precision": "fp32 factor + FP64 IR",
                      "hbm_budget_gb": 200, "workers": args.workers, "seed": 0,
                      "executor": args.serve_executor},
           # latency-bound: the delivered rate cannot exceed the offered load
           "roofline": {"bound": "mfma", "achieved": round(achieved, 4), "peak": FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 5), "traffic": None,
                        "kernel": "all kernels of the serving loop (factor + refinement flops / wall time)",
                        "offered_tflops": round(offered, 3),
                        "note": "latency-bound workload: the offered load is a small fraction of the FP32 "
                                "matrix peak, so frac is capped by offered_tflops / peak"},
           "serving": st, "wall_s": round(wall, 3)}
    # oracle check of a seeded sample of the requests (every n <= 8192)
    rng = np.random.default_rng(7)
    sample = rng.choice(len(results), size=min(args.oracle_sample, len(results)), replace=False)
    oracle.build()
    worst, t_or, fl_or = 0.0, 0.0, 0.0
    for i in sorted(int(v) for v in sample):
        rq, res = pending[i], results[i]
        t1 = time.perf_counter()
        A = oracle.gp_assemble(rq.X, rq.lengthscale, rq.variance, rq.noise)
        L, info = oracle.cholesky(A)
        xref, _, _, failed = oracle.refine(L, A, rq.B, lam=rq.noise, tol=1e-13)
        t_or += time.perf_counter() - t1
        fl_or += rq.n ** 3 / 3
        if info != 0 or failed:
            raise RuntimeError(f"oracle failed on request {i}")
        for c in range(rq.k):
            err = float(np.linalg.norm(res.X[:, c] - xref[:, c]) / np.linalg.norm(xref[:, c]))
            worst = max(worst, err)
    out["oracle_check"] = {"requests": int(len(sample)), "max_rel_err": worst, "tol": 1e-10,
                           "passed": bool(worst <= 1e-10),
                           "reference": "oracle assembly + Cholesky-Crout + refinement with long-double "
                                        "residuals to 1e-13"}
    out["cpu_baseline"] = {"value": round(fl_or / t_or / 1e9, 3), "unit": "GFLOP/s",
                           "cores": oracle.num_threads(), "kind": "oracle",
                           "req_per_s": round(len(sample) / t_or, 3),
                           "sample": f"the {len(sample)} sampled requests solved by the oracle one after another: "
                                     f"{t_or:.2f} s; GFLOP/s = sum of n^3/3 / time"}
    return out


def chol_bytes(n, tile, es):
    N = (n + tile - 1) // tile
    return N * (N + 1) // 2 * tile * tile * es


if __name__ == "__main__":
    main()
