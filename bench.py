#!/usr/bin/env python3
"""Benchmark of the linearised eikonal solve on one MI355X.

Workload (default): 2D grid 1024 x 1024 on the unit box (h = 1/1024),
forcing = seeded smoothed noise (sigma 16 px) mapped to [1, 3], 16 seeded
point sources, hbar = 0.05, T = 16 correction terms, FP32 with per-term
power-of-two scaling and FP64 accumulation.  A step is one whole solve:
reduction of f, kernel spectrum, phi_0, T terms, logarithm.  Inputs are
resident in HBM before timing starts.

Prints ONE JSON line with grid points per second, the roofline of the
dominant kernel (algorithmic bytes per launch / event-timed launch
duration), the plain FP64 GPU solve as comparator and the CPU oracle timed
on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("grid pts/s for K-term eikonal solve, FP32-scaled vs FP64, fwd and fwd+bwd")
HBM_PEAK_GBPS = 8000.0


def alg_bytes_2d(n0, n1, H1, H0, esz, T):
    """Algorithmic HBM bytes per kernel class of a 2D forward solve: every
    pass reads its inputs once and writes its outputs once at the stored
    precision; the spectrum is the n0 x H1 half spectrum (the real DC and
    Nyquist bins share a column), the kernel spectrum the (H1+1) x (H0+1)
    orthant."""
    N = n0 * n1
    csz = 2 * esz
    spec = csz * n0 * H1
    ghat = esz * (H1 + 1) * (H0 + 1)
    return {
        "prep": esz * N,
        "ghat_row": spec,
        "ghat_col": spec + ghat,
        "phi0_row": esz * N + 8 * N + spec,
        "conv_col": 2 * spec + ghat,
        "term_row": 2 * spec + esz * N + 16 * N,
        "last_row": spec + 8 * N + esz * N,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--n", type=int, default=1024, help="grid edge of the workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1403_1937_amd as pk
    import workloads

    if not os.path.exists(pk.lib_path()):
        from paper_1403_1937_amd import build
        build.build()
    dev = torch.device("cuda:0")
    p = workloads.problem(2, args.n)
    n0, n1 = p.dims
    N = n0 * n1

    def run(precision, steps, warmup):
        dt = torch.float32 if precision == "fp32" else torch.float64
        f = torch.as_tensor(p.f.astype(np.float32 if precision == "fp32" else np.float64)).to(dev, dt)
        src = torch.as_tensor(p.src).to(dev)
        plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), precision)
        plan.check_sources(p.src)
        ws = plan.workspace(dev)
        S = torch.empty_like(f)
        for _ in range(warmup):
            plan.solve(f, src, S, ws)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            plan.solve(f, src, S, ws)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # per-kernel durations: HIP events around every launch on the solve's
        # stream, over as many solves as the timed region
        acc = {}
        for _ in range(steps):
            t = plan.solve_timed(f, src, S, ws)
            for k, (m, c) in t.items():
                a = acc.setdefault(k, [0.0, 0])
                a[0] += m
                a[1] += c
        esz = 4 if precision == "fp32" else 8
        H1, H0 = plan.padded[1] // 2, plan.padded[0] // 2
        ab = alg_bytes_2d(n0, n1, H1, H0, esz, p.T)
        kern = {}
        for k, (m, c) in acc.items():
            if c == 0:
                continue
            avg_ms = m / c
            kern[k] = {"launches_per_step": c // steps, "avg_us": 1e3 * avg_ms,
                       "alg_bytes": ab[k], "GBps": ab[k] / (avg_ms * 1e-3) / 1e9}
        total_bytes = sum(ab[k] * kern[k]["launches_per_step"] for k in kern)
        return ms, kern, total_bytes, S

    ms, kern, total_bytes, S = run(args.precision, args.steps, args.warmup)
    value = N / (ms * 1e-3)
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches_per_step"])
    d = kern[dom]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"noise2d_{n0}x{n1}_T{p.T}_src{len(p.src)}",
                   "grid": [n0, n1], "h": p.h, "hbar": p.hbar, "T": p.T,
                   "n_src": int(len(p.src)),
                   "precision": "fp32-scaled" if args.precision == "fp32" else "fp64",
                   "mode": "fwd"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["GBps"],
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": d["GBps"] / HBM_PEAK_GBPS, "traffic": None,
                     "alg_bytes_per_launch": d["alg_bytes"], "avg_us": d["avg_us"]},
        "solve_alg_GBps": total_bytes / (ms * 1e-3) / 1e9,
        "solve_alg_bytes": total_bytes,
        "kernels": kern,
    }
    if not args.no_fp64 and args.precision == "fp32":
        ms64, kern64, tb64, _ = run("fp64", max(5, args.steps // 2), 2)
        out["fp64_comparator"] = {"value": N / (ms64 * 1e-3), "ms_per_step": ms64,
                                  "solve_alg_GBps": tb64 / (ms64 * 1e-3) / 1e9,
                                  "speedup_fp32_over_fp64": ms64 / ms}
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.solve(p.f.astype(np.float64), p.src, p.h, p.hbar, p.T, nthreads=threads)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {"value": N / (t1 - t0), "unit": "grid pts/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"one full {n0}x{n1} T={p.T} solve (FP64, own radix-2 "
                                         f"FFT), {t1 - t0:.2f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
