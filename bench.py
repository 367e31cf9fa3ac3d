#!/usr/bin/env python3
"""Benchmark of the linearised eikonal solve on one MI355X.

Workload (the line's `value`): 2D grid 1024 x 1024 on the unit box
(h = 1/1024), forcing = seeded smoothed noise (sigma 16 px) mapped to [1, 3],
16 seeded point sources, hbar = 0.05, T = 16 correction terms, FP32 with
per-term power-of-two scaling and FP64 accumulation.  A step is one whole
solve: reduction of f, kernel spectrum, phi_0, T terms, logarithm.  Inputs
are resident in HBM before timing starts.

Also reported on the same JSON line:
  fp64_comparator  the plain FP64 GPU solve of the same workload
  fwd_bwd          forward (with checkpoints) + adjoint dL/df on the 2048^2,
                   T = 12, 4-source differentiation workload, FP32-scaled,
                   loss = sum over 256 receivers of (S - target)^2; also the
                   full gradient (ftilde's dependence on f, dL/dhbar)
  batched          64 uneven instances (edges from {256, 512, 1024, 2048},
                   T = 12, FP32-scaled) solved by one replay of a HIP graph
  solve3d          256^3 grid, f from 32 Gaussian blobs in [0.5, 2], one
                   source at the centre, hbar = 0.1, T = 16; FP32-scaled and
                   FP64, per-kernel classes and the dominant kernel's roofline;
                   forward with checkpoints + adjoint in FP32
  config1          the 64 x 64 bump workload (h = 1, T = 8) in FP64: latency
                   of an eager solve and of a replay of the solve captured in
                   a HIP graph
  far_field        the far-field stabilised (tilted) solve of the same
                   workload, FP64 and FP32-scaled: latency (eager and graph
                   replay), and the fraction
                   of the grid within tolerance of the direct sums; and of the
                   2048^2 differentiation workload in FP32 (4 sources),
                   tilted over all sources and per source: time, and the
                   share of the FP64 oracle's resolvable set within 1e-4,
                   against the plain solve's
  backtrack        256 descent paths on the main workload's S (Section 6),
                   path points per second
  fd               the finite-difference screened Poisson system of the main
                   workload (Section 6, the paper's second method) by CG in
                   float64
  roofline         of the dominant kernel: algorithmic bytes per launch over
                   its HIP-event-timed duration; `traffic` from the committed
                   FETCH_SIZE / WRITE_SIZE counter summary when it was taken
                   on the current kernel sources, else null
  cpu_baseline     the FP64 CPU oracle timed on the host cores (threads and
                   CPU model stated)
  accuracy         |S - S_oracle| / max(|S_oracle|, hbar) of every GPU result
                   above against the oracle on the same inputs (computed in
                   the oracle leg): the maximum on the resolvable set
                   (Lambda <= 9 FP32, <= 16 FP64) and on the wider set
                   (12 / 20), full-grid percentiles, the maximum per Lambda
                   bin and the +inf counts; for the 2048^2 gradient the
                   normwise error against the oracle's adjoint

Other modes (for profiling runs):
  --pmc-run                 a copy-calibration kernel, then a few solves of
                            the main workload with row schedules 8 and 16
                            (run under rocprofv3 --pmc)
  --traffic-summary F W     turn the counter CSVs of a FETCH_SIZE run (F) and
                            a WRITE_SIZE run (W) into the traffic summary
  --stats-summary CSV       turn a rocprofv3 kernel_stats.csv into a short
                            text summary
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("grid pts/s for K-term eikonal solve, FP32-scaled vs FP64, fwd and fwd+bwd")
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_term_row_noise2d_1024x1024_fp32.txt")
COPY_ELEMS = 64 << 20  # float32 elements of the calibration copy (256 MiB each way)


KERNEL_SOURCES_2D = ("fft_team.hpp", "geom2d.hpp", "green.hpp", "common2d.hpp", "row2d.hpp",
                     "col2d.hpp", "k2d_impl.hpp", "k2d_row16_f32.hip", "k2d_row8_f32.hip",
                     "k2d_col_f32.hip")


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """A line on stderr as each section ends (stdout carries only the JSON)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the device sources of the FP32 2D kernels: counter figures
    are valid only for these."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1403_1937_amd", "csrc")
    for name in KERNEL_SOURCES_2D:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def alg_bytes_2d(n0, n1, H1, H0, esz, T, ckpt=False):
    """Algorithmic HBM bytes per kernel class of a 2D forward solve: every
    pass reads its inputs once and writes its outputs once at the stored
    precision; the spectrum is the n0 x H1 half spectrum (the real DC and
    Nyquist bins share a column), the kernel spectrum the (H1+1) x (H0+1)
    orthant.  Each term's mantissas are stored once (into the checkpoint when
    one is kept) and the last pass sums the T stored terms in float64; with a
    checkpoint it also writes phi (8 N)."""
    N = n0 * n1
    spec = 2 * esz * n0 * H1
    ghat = esz * (H1 + 1) * (H0 + 1)
    return {
        "prep": esz * N,
        "ghat_row": spec,
        "ghat_col": spec + ghat,
        "phi0_row": 3 * esz * N + spec,                      # f in; gamma, phi_0, spectrum out
        "conv_col": 2 * spec + ghat,
        "term_row": 2 * spec + 2 * esz * N,                  # spectrum in/out, gamma, term out
        "last_row": spec + T * esz * N + esz * N + (8 * N if ckpt else 0),
        # phi_0 by FFT (many sources): kernel table and spectrum, zeroed
        # source grid, its transform and the product with the spectrum
        "phi0_fft": spec + (spec + ghat) + esz * N + (esz * N + spec) + (2 * spec + ghat),
    }


def alg_bytes_3d(dims, padded, esz, T):
    """Algorithmic bytes per kernel class of a 3D forward solve (same rule):
    s1 = n0 n1 H2 and s2 = n0 M1 H2 complex spectra, the kernel spectrum
    (H1+1)(H0+1)H2 real."""
    n0, n1, n2 = dims
    M0, M1, M2 = padded
    H0, H1, H2 = M0 // 2, M1 // 2, M2 // 2
    N = n0 * n1 * n2
    csz = 2 * esz
    s1 = csz * n0 * n1 * H2
    s2 = csz * n0 * M1 * H2
    g = esz * (H1 + 1) * (H0 + 1) * H2
    s2g = csz * n0 * (H1 + 1) * H2
    return {
        "prep": esz * N,
        "ghat_row": s1,
        "ghat_col": s1 + s2g,
        "ghat_z": s2g + g,
        "phi0_row": 3 * esz * N + s1,
        "y_fwd": s1 + s2,
        "conv_col": 2 * s2 + g,
        "y_inv": s2 + s1,
        "term_row": 2 * s1 + 2 * esz * N,
        "last_row": s1 + T * esz * N + esz * N,
    }


def alg_bytes_adjoint_2d(n0, n1, H1, H0, esz, T):
    """Algorithmic bytes of the adjoint sweep (same rule): lambda start,
    then per term a column convolution and a row pass that reads the
    checkpointed term, gamma and lambda and updates the FP64 dL/dgamma."""
    N = n0 * n1
    spec = 2 * esz * n0 * H1
    ghat = esz * (H1 + 1) * (H0 + 1)
    total = esz * N + 8 * N                                   # max |lambda|
    total += 2 * esz * N + 8 * N + 2 * esz * N + spec         # lambda, gamma, a_T spectrum
    for i in range(T, 0, -1):
        total += 2 * spec + ghat                              # b_i = kappa * a_i
        row = spec + esz * N + esz * N                        # spectrum, term, gamma or f
        if i != T:
            row += 8 * N                                      # dL/dgamma read
        if i > 1:
            row += esz * N + 8 * N + spec                     # lambda, dL/dgamma, a_{i-1}
        else:
            row += esz * N                                    # dL/df
        total += row
    return total


def read_traffic(kernel_hash: str, row_e: int):
    """Per-launch HBM bytes of the term-row kernel of schedule row_e from the
    committed counter summary, or None when it is missing or stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.loads(fh.read().split("\n---\n", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if d.get("source_hash") != kernel_hash:
        return None
    e = d.get("per_schedule", {}).get(str(row_e))
    return None if e is None else e.get("traffic_bytes_per_launch")


def _events(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return e0, e1


def run_main(pk, torch, dev, p, precision, steps, warmup, schedule=None):
    n0, n1 = p.dims[:2]
    dt = torch.float32 if precision == "fp32" else torch.float64
    f = torch.as_tensor(p.f.astype(np.float32 if precision == "fp32" else np.float64)).to(dev, dt)
    src = torch.as_tensor(p.src).to(dev)
    plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), precision)
    plan.check_sources(p.src)
    ws = plan.workspace(dev)
    if schedule is None:
        plan.autotune(ws)  # schedule choice (radix / work-group shape), untimed
    else:
        plan.set_schedule(*schedule)
    S = torch.empty_like(f)
    for _ in range(warmup):
        plan.solve(f, src, S, ws)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = _events(torch, st)
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
    if len(p.dims) == 3:
        ab = alg_bytes_3d(p.dims, plan.padded, esz, p.T)
    else:
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
    kern["schedule"] = plan.schedule
    plan.solve(f, src, S, ws)
    torch.cuda.synchronize()
    return ms, kern, total_bytes, S.double().cpu().numpy()


def run_3d(pk, torch, dev, steps, warmup):
    """The 256^3 blob workload, FP32-scaled and FP64."""
    import workloads
    p = workloads.problem(3)
    N = int(np.prod(p.dims))
    out = {"workload": "blobs3d_256x256x256_T16_src1", "unit": "grid pts/s"}
    results = {}
    for prec in ("fp32", "fp64"):
        ms, kern, tb, results[prec] = run_main(pk, torch, dev, p, prec, steps, warmup)
        kern.pop("schedule")
        dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches_per_step"])
        out[prec] = {"value": N / (ms * 1e-3), "ms_per_step": ms,
                     "solve_alg_GBps": tb / (ms * 1e-3) / 1e9, "solve_alg_bytes": tb,
                     "roofline": {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["GBps"],
                                  "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                  "frac": kern[dom]["GBps"] / HBM_PEAK_GBPS},
                     "kernels": kern}
    out["speedup_fp32_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]

    # forward with checkpoints + adjoint (FP32) for a loss at 256 receivers
    # near the source: dL/dS = 2 (S - 0.97 S_0) there, S_0 the first solve
    f = torch.as_tensor(p.f).to(dev)
    src = torch.as_tensor(p.src).to(dev)
    plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), "fp32")
    ws, ck = plan.workspace(dev), plan.checkpoint(dev)
    S = torch.empty_like(f)
    dLdf = torch.empty_like(f)
    rng = np.random.default_rng(11)
    rec = workloads.receivers_near_sources(p.dims, p.src, 256, 0.25 * p.dims[0], rng)
    ridx = torch.as_tensor(np.ravel_multi_index(tuple(rec.T), p.dims).astype(np.int64)).to(dev)
    plan.solve(f, src, S, ws)
    tgt = 0.97 * S.view(-1)[ridx]
    dLdS = torch.zeros(N, dtype=torch.float32, device=dev)

    def step():
        plan.solve(f, src, S, ws, ck)
        dLdS[ridx] = 2.0 * (S.view(-1)[ridx] - tgt)
        plan.adjoint(f, src, ck, dLdS.view(p.dims), dLdf, ws)

    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = _events(torch, st)
    e0.record(st)
    for _ in range(steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    e0.record(st)
    for _ in range(steps):
        plan.adjoint(f, src, ck, dLdS.view(p.dims), dLdf, ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / steps
    # the full gradient (ftilde(f) and hbar as well) after the same forward
    wsf = torch.empty(plan.adjoint_full_workspace_bytes, dtype=torch.uint8, device=dev)
    grads = torch.zeros(4, dtype=torch.float64, device=dev)
    plan.solve(f, src, S, wsf, ck)
    for _ in range(max(1, warmup)):
        plan.adjoint_full(f, src, ck, dLdS.view(p.dims), dLdf, grads, wsf)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        plan.adjoint_full(f, src, ck, dLdS.view(p.dims), dLdf, grads, wsf)
    e1.record(st)
    torch.cuda.synchronize()
    ms_full = e0.elapsed_time(e1) / steps
    out["fwd_bwd_fp32"] = {"value": N / (ms * 1e-3), "ms_per_step": ms, "ms_adjoint": ms_adj,
                           "ms_adjoint_full": ms_full,
                           "loss": "sum over 256 receivers near the source of (S - 0.97 S_0)^2",
                           "gradient_finite": bool(torch.isfinite(dLdf).all().item()),
                           "full_gradient_dLdhbar": float(grads[0].item())}

    def gradient(dLdS_host):
        d = torch.as_tensor(dLdS_host).to(dev, torch.float32)
        plan.solve(f, src, S, ws, ck)
        plan.adjoint(f, src, ck, d, dLdf, ws)
        return dLdf.double().cpu().numpy()

    return out, (p, results, (rec, gradient))


def run_fwd_bwd(pk, torch, dev, steps, warmup):
    """Forward with checkpoints + adjoint on the 2048^2 differentiation
    workload; dL/dS = 2 (S - target) at 256 receivers, 0 elsewhere."""
    import workloads
    p = workloads.problem(5)
    rec, f_t = workloads.loss_setup(p)
    n0, n1 = p.dims
    N = n0 * n1
    f = torch.as_tensor(p.f).to(dev)
    src = torch.as_tensor(p.src).to(dev)
    plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), "fp32")
    plan.check_sources(p.src)
    ws, ck = plan.workspace(dev), plan.checkpoint(dev)
    plan.autotune(ws)
    S = torch.empty_like(f)
    # target: the same solve for the perturbed forcing
    tgt = torch.empty_like(f)
    plan.solve(torch.as_tensor(f_t).to(dev), src, tgt, ws)
    ridx = torch.as_tensor(rec[:, 0].astype(np.int64) * n1 + rec[:, 1]).to(dev)
    dLdS = torch.zeros(N, dtype=torch.float32, device=dev)
    dLdf = torch.empty_like(f)

    def step():
        plan.solve(f, src, S, ws, ck)
        # the loss gradient w.r.t. S (a gather and a scatter of 256 values)
        dLdS[ridx] = 2.0 * (S.view(-1)[ridx] - tgt.view(-1)[ridx])
        plan.adjoint(f, src, ck, dLdS.view(n0, n1), dLdf, ws)

    st = torch.cuda.current_stream()
    e0, e1 = _events(torch, st)
    # the library's tuner times the forward solve; the adjoint's row pass
    # ranks the row schedules differently, so the row schedule of this step
    # is picked by timing the whole step (untimed, before the warm-up)
    col_e = plan.schedule["col_e"]
    best = None
    for row_e in (16, 8, 4):
        plan.set_schedule(row_e, col_e)
        step()
        e0.record(st)
        for _ in range(2):
            step()
        e1.record(st)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        if best is None or t < best[0]:
            best = (t, row_e)
    plan.set_schedule(best[1], col_e)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # forward alone with checkpoints, for the split
    e0.record(st)
    for _ in range(steps):
        plan.solve(f, src, S, ws, ck)
    e1.record(st)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / steps
    H1, H0 = plan.padded[1] // 2, plan.padded[0] // 2
    ab = alg_bytes_2d(n0, n1, H1, H0, 4, p.T, ckpt=True)
    fwd_bytes = (ab["prep"] + ab["ghat_row"] + ab["ghat_col"] + ab["phi0_row"]
                 + p.T * ab["conv_col"] + (p.T - 1) * ab["term_row"] + ab["last_row"])
    bwd_bytes = alg_bytes_adjoint_2d(n0, n1, H1, H0, 4, p.T)
    ok = bool(torch.isfinite(dLdf).all().item())

    # the full gradient (dL/df with ftilde's dependence on f, dL/dhbar): the
    # same step with sweik_solve_adjoint_full on its larger workspace
    wsf = torch.empty(plan.adjoint_full_workspace_bytes, dtype=torch.uint8, device=dev)
    grads = torch.zeros(4, dtype=torch.float64, device=dev)

    def step_full():
        plan.solve(f, src, S, wsf, ck)
        dLdS[ridx] = 2.0 * (S.view(-1)[ridx] - tgt.view(-1)[ridx])
        plan.adjoint_full(f, src, ck, dLdS.view(n0, n1), dLdf, grads, wsf)

    step_full()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        step_full()
    e1.record(st)
    torch.cuda.synchronize()
    ms_full = e0.elapsed_time(e1) / steps

    plan.solve(f, src, S, ws, ck)
    torch.cuda.synchronize()
    S_host = S.double().cpu().numpy()

    def gradient(dLdS_host):
        """dL/df of this plan's solve for a given dL/dS (host arrays)."""
        plan.solve(f, src, S, ws, ck)
        plan.adjoint(f, src, ck, torch.as_tensor(dLdS_host.astype(np.float32)).to(dev), dLdf, ws)
        torch.cuda.synchronize()
        return dLdf.double().cpu().numpy()

    out = {"workload": f"noise2d_{n0}x{n1}_T{p.T}_src{len(p.src)}_rec{len(rec)}",
            "value": N / (ms * 1e-3), "unit": "grid pts/s", "ms_per_step": ms,
            "ms_forward_with_checkpoints": ms_fwd, "ms_adjoint": ms - ms_fwd,
            "alg_bytes": fwd_bytes + bwd_bytes,
            "alg_GBps": (fwd_bytes + bwd_bytes) / (ms * 1e-3) / 1e9,
            "hbm_frac": (fwd_bytes + bwd_bytes) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "precision": "fp32-scaled", "gradient_finite": ok, "schedule": plan.schedule,
            "full_gradient": {"value": N / (ms_full * 1e-3), "ms_per_step": ms_full,
                              "ms_adjoint_full": ms_full - ms_fwd,
                              "dLdhbar": float(grads[0].item()),
                              "note": "dL/df with the ftilde(f) subgradient, and dL/dhbar"}}
    return out, (p, rec, f_t, S_host, gradient)


def run_backtrack(pk, torch, dev, steps, warmup):
    """Backtracking (Section 6) of 256 paths from seeded start points on the
    S of the 1024^2 main workload (step 0.5 cell, stop within 1 cell of a
    source): one thread per path, so the figure of merit is path points per
    second."""
    import workloads
    p = workloads.problem(2, 1024)
    f = torch.as_tensor(p.f).to(dev)
    S = pk.solve(f, p.src, p.h, p.hbar, p.T)
    rng = np.random.default_rng(2024)
    start = rng.uniform(0, 1023, size=(256, 2))
    args = dict(step=0.5, radius=1.0, max_steps=8192)
    for _ in range(max(1, warmup)):
        path, npts, st = pk.backtrack(S, p.src, start, **args)
    torch.cuda.synchronize()
    s_ = torch.cuda.current_stream()
    e0, e1 = _events(torch, s_)
    e0.record(s_)
    for _ in range(steps):
        path, npts, st = pk.backtrack(S, p.src, start, **args)
    e1.record(s_)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    npts = npts.cpu().numpy()
    st = st.cpu().numpy()
    return {"workload": "backtrack_noise2d_1024x1024_256paths", "paths": 256,
            "path_points": int(npts.sum()), "max_points": int(npts.max()),
            "reached_source": int((st == 0).sum()), "ms_per_call": ms,
            "value": float(npts.sum()) / (ms * 1e-3), "unit": "path points/s",
            "bound": "latency (one thread per path, dependent reads of S)"}


def run_large(pk, torch, dev, steps, warmup):
    """The largest grids a plan takes, in float32 (T = 16): 2D 4096 x 8192
    (16 sources) and 3D 1024^3 (one source, a 112 GiB workspace).  f is a
    smooth field made on the device; each grid also gets a constant-forcing
    solve (phi = phi_0) checked against its closed form on 4096 sampled
    points."""
    import math
    out = {}
    rng = np.random.default_rng(23)
    for dims, n_src in (((4096, 8192), 16), ((1024, 1024, 1024), 1)):
        n = max(dims)
        ax = [torch.arange(d, dtype=torch.float32, device=dev) / d for d in dims]
        if len(dims) == 2:
            f = 2.0 + 0.8 * torch.sin(6 * math.pi * ax[0])[:, None] * torch.cos(4 * math.pi * ax[1])[None, :]
        else:
            f = (1.25 + 0.35 * torch.sin(2 * math.pi * ax[0])[:, None, None]
                 * torch.cos(4 * math.pi * ax[1])[None, :, None]
                 + 0.2 * torch.sin(6 * math.pi * ax[2])[None, None, :])
        f = f.contiguous()
        src = np.stack([rng.integers(0, d, n_src) for d in dims], 1).astype(np.int32)
        src = np.unique(src, axis=0)
        h, hbar, T = 1.0 / n, 0.05 if len(dims) == 2 else 0.1, 16
        plan = pk.Plan(dims, h, hbar, T, len(src), "fp32")
        ws = plan.workspace(dev)
        d_src = torch.as_tensor(src).to(dev)
        S = torch.empty_like(f)
        for _ in range(max(1, warmup)):
            plan.solve(f, d_src, S, ws)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = _events(torch, st)
        e0.record(st)
        for _ in range(steps):
            plan.solve(f, d_src, S, ws)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        finite = float(torch.isfinite(S).float().mean().item())
        del ws, S
        # constant forcing: S = -hbar ln sum_k exp(-c |x - y_k| h / hbar)
        c = 1.3
        fc = torch.full_like(f, c)
        del f
        Sc = pk.solve(fc, src, h, hbar, 2)
        idx = np.stack([rng.integers(0, d, 4096) for d in dims], 1)
        dist = np.linalg.norm(idx[:, None, :] - src[None, :, :], axis=-1) * h
        ref = -hbar * np.log(np.exp(-c * dist / hbar).sum(axis=1))
        got = Sc[tuple(torch.as_tensor(idx.T).to(dev).long())].double().cpu().numpy()
        err = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), hbar)))
        del Sc, fc
        torch.cuda.empty_cache()
        N = int(np.prod(dims))
        name = ("noise2d" if len(dims) == 2 else "smooth3d") + "_" + "x".join(map(str, dims))
        out[f"{name}_T{T}_src{len(src)}"] = {
            "value": N / (ms * 1e-3), "unit": "grid pts/s", "ms_per_step": ms,
            "workspace_GiB": plan.workspace_bytes / 2**30, "finite_frac": finite,
            "constant_forcing_closed_form_max_rel": err, "precision": "fp32-scaled"}
    return out


def run_fd(pk, torch, dev, steps, warmup):
    """The paper's second method (Section 6): the finite-difference screened
    Poisson system of the 1024^2 main workload, CG in float64 to
    ||r|| <= 1e-10 ||b||.  Bytes per CG iteration (one kernel; float64
    vectors of N): reads r, w, s_prev, p, x, 1/diag and writes p, s, x, r,
    w (88 N; the neighbours' r, w, s, 1/diag come from cache)."""
    import workloads
    p = workloads.problem(2, 1024)
    N = p.dims[0] * p.dims[1]
    f = torch.as_tensor(p.f).to(dev, torch.float64)
    for _ in range(max(1, warmup)):
        S, info = pk.fd_solve(f, p.src, p.h, p.hbar, rtol=1e-10, return_info=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S, info = pk.fd_solve(f, p.src, p.h, p.hbar, rtol=1e-10, return_info=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps  # the call synchronises: host clock
    it = info["iterations"]
    per_it = ms / max(it, 1)
    return {"workload": "fd_noise2d_1024x1024_src16", "value": N / (ms * 1e-3),
            "unit": "grid pts/s", "ms_per_step": ms, "iterations": it,
            "rel_residual": info["rel_residual"], "us_per_iteration": per_it * 1e3,
            "iteration_alg_bytes": 88 * N,
            "iteration_GBps": 88 * N / (per_it * 1e-3) / 1e9, "precision": "fp64"}


def run_batched(pk, torch, dev, steps, warmup):
    """64 uneven instances, one HIP graph replay per step."""
    import workloads
    probs = workloads.batch_problems()
    T = probs[0].T
    # tune one plan per edge length: the batch's plans start from the table
    sched = {}
    for n in sorted({q.dims[0] for q in probs}):
        tp = pk.Plan((n, n), 1.0 / n, 0.1, T, 1, "fp32")
        tp.autotune(tp.workspace(dev))
        sched[n] = tp.schedule
    torch.cuda.empty_cache()
    b = pk.Batch([{"dims": q.dims, "h": q.h, "hbar": q.hbar, "T": q.T, "n_src": len(q.src)}
                  for q in probs], "fp32")
    fs = [torch.as_tensor(q.f).to(dev) for q in probs]
    srcs = [torch.as_tensor(q.src).to(dev) for q in probs]
    Ss = [torch.empty_like(f) for f in fs]
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device=dev)
    for _ in range(max(1, warmup)):
        b.solve(fs, srcs, Ss, ws, graph=True)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = _events(torch, st)
    e0.record(st)
    for _ in range(steps):
        b.solve(fs, srcs, Ss, ws, graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    e0.record(st)
    for _ in range(steps):
        b.solve(fs, srcs, Ss, ws, graph=False)
    e1.record(st)
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / steps
    sumN = sum(q.dims[0] * q.dims[1] for q in probs)
    total = 0
    for q in probs:
        n0, n1 = q.dims
        M0 = max(64, 1 << int(np.ceil(np.log2(2 * n0 - 1))))
        M1 = max(64, 1 << int(np.ceil(np.log2(2 * n1 - 1))))
        ab = alg_bytes_2d(n0, n1, M1 // 2, M0 // 2, 4, T)
        total += (ab["prep"] + ab["ghat_row"] + ab["ghat_col"] + ab["phi0_row"]
                  + T * ab["conv_col"] + (T - 1) * ab["term_row"] + ab["last_row"])
    sizes = {}
    for q in probs:
        sizes[q.dims[0]] = sizes.get(q.dims[0], 0) + 1
    # one instance of each edge length (the first in the batch), for the
    # accuracy figures
    sample = {}
    for j, q in enumerate(probs):
        if q.dims[0] not in sample:
            sample[q.dims[0]] = (j, q, Ss[j].double().cpu().numpy())
    out = {"workload": f"batch64_uneven_T{T}", "instances_per_edge": sizes,
            "sum_grid_pts": sumN, "value": sumN / (ms * 1e-3), "unit": "grid pts/s",
            "ms_per_step": ms, "ms_per_step_eager": ms_eager, "alg_bytes": total,
            "alg_GBps": total / (ms * 1e-3) / 1e9,
            "hbm_frac": total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, "precision": "fp32-scaled",
            "execution": "one HIP graph replay per step", "schedules": sched}
    return out, sample


def graph_latency(torch, fn, out, steps):
    """Capture fn (an enqueue of one solve into caller-owned buffers) into a
    HIP graph and time `steps` replays one by one with events: the solve's
    latency without the host's per-launch cost.  Returns (median ms, whether
    the replayed result equals the eager one bit for bit)."""
    fn()
    torch.cuda.synchronize()
    ref = out.clone()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph):
            fn()
    torch.cuda.current_stream().wait_stream(side)
    st = torch.cuda.current_stream()
    times = []
    for _ in range(steps):
        e0, e1 = _events(torch, st)
        e0.record(st)
        graph.replay()
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    same = bool(torch.equal(out, ref))
    del graph
    return float(np.median(times)), same


def run_config1(pk, torch, dev, steps, warmup):
    """The plain method on the 64 x 64 bump workload (h = 1, hbar = 0.5,
    one source at the centre, T = 8) in FP64: a few hundred kilobytes per
    solve, so the figure is the latency of one solve (median of `steps`
    event-timed solves after the warm-up)."""
    import workloads
    p = workloads.problem(1)
    f = torch.as_tensor(p.f.astype(np.float64)).to(dev)
    src = torch.as_tensor(p.src).to(dev)
    plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), "fp64")
    plan.check_sources(p.src)
    ws = plan.workspace(dev)
    S = torch.empty_like(f)
    for _ in range(max(1, warmup)):
        plan.solve(f, src, S, ws)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(steps):
        e0, e1 = _events(torch, st)
        e0.record(st)
        plan.solve(f, src, S, ws)
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    S_host = S.double().cpu().numpy()
    gms, same = graph_latency(torch, lambda: plan.solve(f, src, S, ws), S, steps)
    out = {"workload": "bumps2d_64x64_T8_src1_h1", "precision": "fp64",
           "latency_ms_median": ms, "latency_ms_min": float(min(times)),
           "value": p.dims[0] * p.dims[1] / (ms * 1e-3), "unit": "grid pts/s",
           "launches_per_solve": 4 + 2 * p.T,
           "bound": "pass latency: at 64^2 a row pass is one work-group (all 64 rows) and "
                    "every pass a chain of dependent loads, LDS exchanges and barriers "
                    "(about 8-10 us each); a graph replay takes as long as the eager solve",
           "graph_replay_latency_ms_median": gms, "graph_replay_equals_eager": same}
    return out, (p, S_host)


def run_far_field(pk, torch, dev, steps, warmup):
    """The far-field stabilised solve (sweik_solve_tilted: the plain solve
    and 8 tilt directions at 0.9 beta) on the 64 x 64 bump workload, FP64
    and FP32-scaled: latency of one solve (median of event-timed solves)."""
    import workloads
    p = workloads.problem(1)
    tilts = pk.default_tilts(8, 0.9)
    out = {"workload": "bumps2d_64x64_T8_src1_h1", "tilts": len(tilts),
           "tilt_strength": 0.9, "unit": "grid pts/s"}
    results = {}
    for prec in ("fp64", "fp32"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        f = torch.as_tensor(p.f.astype(np.float64)).to(dev, dt)
        src = torch.as_tensor(p.src).to(dev)
        plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), prec)
        ws = torch.empty(plan.tilted_workspace_bytes(len(tilts)), dtype=torch.uint8, device=dev)
        S = torch.empty_like(f)
        for _ in range(max(1, warmup)):
            plan.solve_tilted(f, src, S, ws, tilts)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        times = []
        for _ in range(steps):
            e0, e1 = _events(torch, st)
            e0.record(st)
            plan.solve_tilted(f, src, S, ws, tilts)
            e1.record(st)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        results[prec] = S.double().cpu().numpy()
        gms, same = graph_latency(torch, lambda: plan.solve_tilted(f, src, S, ws, tilts), S,
                                  steps)
        out[prec] = {"latency_ms_median": ms,
                     "value": p.dims[0] * p.dims[1] / (ms * 1e-3),
                     "graph_replay_latency_ms_median": gms, "graph_replay_equals_eager": same}
    # the 2048^2 differentiation workload's forward solve (4 sources, Lambda
    # up to ~32) in FP32: tilted over all sources, tilted per source, plain
    p5 = workloads.problem(5)
    f5 = torch.as_tensor(p5.f).to(dev)
    src5 = torch.as_tensor(p5.src).to(dev)
    plan5 = pk.Plan(p5.dims, p5.h, p5.hbar, p5.T, len(p5.src), "fp32")
    ws5 = torch.empty(plan5.tilted_workspace_bytes(len(tilts)), dtype=torch.uint8, device=dev)
    S5 = torch.empty_like(f5)
    st = torch.cuda.current_stream()
    big = {}
    for name, per_source in (("tilted", False), ("tilted_per_source", True)):
        plan5.solve_tilted(f5, src5, S5, ws5, tilts, per_source=per_source)
        torch.cuda.synchronize()
        e0, e1 = _events(torch, st)
        e0.record(st)
        for _ in range(3):
            plan5.solve_tilted(f5, src5, S5, ws5, tilts, per_source=per_source)
        e1.record(st)
        torch.cuda.synchronize()
        ms5 = e0.elapsed_time(e1) / 3
        out[f"noise2d_2048x2048_fp32_{name}"] = {
            "ms_per_solve": ms5, "value": p5.dims[0] * p5.dims[1] / (ms5 * 1e-3)}
        big[name] = S5.double().cpu().numpy()
    plan5.solve(f5, src5, S5, ws5)
    torch.cuda.synchronize()
    big["plain"] = S5.double().cpu().numpy()
    results["noise2d_2048x2048_fp32"] = (p5, big)
    return out, (p, results)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---- cpu_baseline leg ---------------------------------------------------------
# The FP64 oracle on the host cores.  This leg is the only part of the
# benchmark that runs the oracle: it times it (cpu_baseline) and computes the
# reference results that the accuracy figures compare the GPU results with.

# (resolvable set on which the tolerance is claimed, the wider set that the
# conditioning law alone would suggest) per precision, in Lambda =
# ln(max phi / phi(x)) of the oracle
LAMBDA_SETS = {"fp32": (9.0, 12.0), "fp64": (16.0, 20.0)}
TOLERANCE = {"fp32": 1e-4, "fp64": 1e-10}
LAMBDA_BINS = (0.0, 4.0, 8.0, 12.0, 16.0, 20.0, 30.0, 40.0, np.inf)


def accuracy(S, o, hbar, prec):
    """|S - S_oracle| / max(|S_oracle|, hbar) of one GPU result: the maximum
    on the resolvable set and on the wider set, full-grid percentiles, the
    maximum per Lambda bin and the +inf counts."""
    S = np.asarray(S, np.float64)
    So, phi = o["S"], o["phi"]
    pos = phi > 0
    L = np.full(phi.shape, np.inf)
    L[pos] = np.log(phi[pos].max() / phi[pos])
    with np.errstate(invalid="ignore"):
        rel = np.abs(S - So) / np.maximum(np.abs(So), hbar)
    fin = np.isfinite(S) & np.isfinite(So)

    def mx(m):
        return float(np.nan_to_num(rel[m], nan=np.inf).max()) if m.any() else None

    tight, wide = LAMBDA_SETS[prec]
    bins = {}
    for lo, hi in zip(LAMBDA_BINS[:-1], LAMBDA_BINS[1:]):
        m = (L > lo) & (L <= hi) if lo > 0 else (L <= hi)
        if m.any():
            bins[f"{lo:g}-{hi:g}"] = {"max_rel": mx(m & fin) if (m & fin).any() else None,
                                     "frac": float(m.mean()),
                                     "n_inf_gpu": int((m & np.isinf(S)).sum())}
    r_tight, r_wide = L <= tight, L <= wide
    return {"tol": TOLERANCE[prec],
            "set": f"Lambda<={tight:g}", "max_rel": mx(r_tight), "frac_set": float(r_tight.mean()),
            "within_tol": bool(mx(r_tight) is not None and mx(r_tight) <= TOLERANCE[prec]),
            "wide_set": f"Lambda<={wide:g}", "max_rel_wide": mx(r_wide),
            "frac_wide": float(r_wide.mean()),
            "p50_all": float(np.percentile(rel[fin], 50)) if fin.any() else None,
            "p99_all": float(np.percentile(rel[fin], 99)) if fin.any() else None,
            "max_rel_by_lambda": bins,
            "n_inf_gpu": int(np.isinf(S).sum()), "n_nonpositive_oracle": int((~pos).sum())}


def cpu_baseline(p, threads, budget_s=10.0):
    """The FP64 CPU oracle on the host cores: whole solves of the main
    workload, repeated until `budget_s` seconds have passed; plus one
    single-thread solve.  Also returns the oracle's result of the workload."""
    import oracle
    n0, n1 = p.dims
    f64 = p.f.astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    first = None
    while True:
        o = oracle.solve(f64, p.src, p.h, p.hbar, p.T, nthreads=threads)
        if first is None:
            first = o
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    t1 = time.perf_counter()
    oracle.solve(f64, p.src, p.h, p.hbar, p.T, nthreads=1)
    t1s = time.perf_counter() - t1
    return {"value": reps * n0 * n1 / el, "unit": "grid pts/s", "cores": threads,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{reps} full {n0}x{n1} T={p.T} solves (FP64, own radix-2 FFT) in "
                      f"{el:.1f} s on {threads} threads",
            "single_thread": {"value": n0 * n1 / t1s, "seconds_per_solve": t1s}}, first


def reference_accuracy(gpu, o_main, threads):
    """Accuracy of every GPU result against the FP64 oracle on the same
    inputs.  `gpu` holds the host copies of the GPU results per section."""
    import oracle
    out = {"reference": "FP64 CPU oracle (own FFT) on the same inputs; rel = |S - S_oracle| / "
                        "max(|S_oracle|, hbar); Lambda = ln(max phi / phi) of the oracle"}
    p, S32, S64 = gpu["main"]
    out["main"] = {"workload": f"noise2d_{p.dims[0]}x{p.dims[1]}_T{p.T}",
                   "fp32": accuracy(S32, o_main, p.hbar, "fp32")}
    if S64 is not None:
        out["main"]["fp64"] = accuracy(S64, o_main, p.hbar, "fp64")
    if "config1" in gpu:
        progress("accuracy: config1")
        p1, S1 = gpu["config1"]
        f1 = p1.f.astype(np.float64)
        od = oracle.solve(f1, p1.src, p1.h, p1.hbar, p1.T, method="direct", nthreads=threads)
        of = oracle.solve(f1, p1.src, p1.h, p1.hbar, p1.T, nthreads=threads)
        out["config1"] = {"workload": "bumps2d_64x64_T8_src1_h1",
                          "fp64_vs_oracle_fft": accuracy(S1, of, p1.hbar, "fp64"),
                          "fp64_vs_oracle_direct": accuracy(S1, od, p1.hbar, "fp64"),
                          "note": "the direct sum is the ground truth where FFT noise dominates "
                                  "(Lambda beyond ~30)"}
    if "fwd_bwd" in gpu:
        progress("accuracy: fwd_bwd")
        p5, rec, f_t, S5, gradient = gpu["fwd_bwd"]
        f5 = p5.f.astype(np.float64)
        o5 = oracle.solve(f5, p5.src, p5.h, p5.hbar, p5.T, nthreads=threads)
        t5 = oracle.solve(f_t.astype(np.float64), p5.src, p5.h, p5.hbar, p5.T, nthreads=threads)
        dLdS = np.zeros(p5.dims)
        r0, r1 = rec[:, 0], rec[:, 1]
        dLdS[r0, r1] = 2.0 * (o5["S"][r0, r1] - t5["S"][r0, r1])
        g_o, _ = oracle.adjoint(f5, p5.src, p5.h, p5.hbar, p5.T, dLdS, nthreads=threads)
        g = gradient(dLdS)
        out["fwd_bwd"] = {"workload": f"noise2d_{p5.dims[0]}x{p5.dims[1]}_T{p5.T}",
                          "forward_fp32": accuracy(S5, o5, p5.hbar, "fp32"),
                          "gradient_fp32": {
                              "normwise_rel": float(np.linalg.norm(g - g_o) / np.linalg.norm(g_o)),
                              "tol": 1e-3,
                              "dLdS": "2 (S - target) at 256 receivers, from the oracle's solves "
                                      "of f and the perturbed forcing"}}
    if "batched" in gpu:
        progress("accuracy: batched")
        res = {}
        for n, (j, q, Sq) in sorted(gpu["batched"].items()):
            oq = oracle.solve(q.f.astype(np.float64), q.src, q.h, q.hbar, q.T, nthreads=threads)
            a = accuracy(Sq, oq, q.hbar, "fp32")
            a["instance"] = j
            a["hbar"] = q.hbar
            a["n_src"] = int(len(q.src))
            res[str(n)] = a
        out["batched"] = {"sample": "the first instance of each edge length", "fp32": res}
    if "far_field" in gpu:
        progress("accuracy: far_field")
        pf, rf = gpu["far_field"]
        od = oracle.solve(pf.f.astype(np.float64), pf.src, pf.h, pf.hbar, pf.T, method="direct",
                          nthreads=threads)
        res = {"reference": "the oracle's direct sums (the ground truth at every Lambda here)"}
        big = rf.pop("noise2d_2048x2048_fp32", None)
        for prec, Sf in rf.items():
            a = accuracy(Sf, od, pf.hbar, prec)
            with np.errstate(invalid="ignore"):
                rel = np.abs(Sf - od["S"]) / np.maximum(np.abs(od["S"]), pf.hbar)
            a["frac_grid_within_tol"] = float(np.mean(np.nan_to_num(rel, nan=np.inf)
                                                      <= TOLERANCE[prec]))
            res[prec] = a
        if "config1" in gpu:  # the plain FP64 solve of the same workload, for comparison
            with np.errstate(invalid="ignore"):
                rel = np.abs(gpu["config1"][1] - od["S"]) / np.maximum(np.abs(od["S"]), pf.hbar)
            res["plain_fp64_frac_grid_within_tol"] = float(
                np.mean(np.nan_to_num(rel, nan=np.inf) <= TOLERANCE["fp64"]))
        if big is not None:
            # reference: the FP64 oracle FFT where it resolves phi (Lambda <= 16)
            p5, runs = big
            o5 = oracle.solve(p5.f.astype(np.float64), p5.src, p5.h, p5.hbar, p5.T,
                              nthreads=threads)
            phi = o5["phi"]
            L = np.full(phi.shape, np.inf)
            L[phi > 0] = np.log(phi[phi > 0].max() / phi[phi > 0])
            r64 = L <= LAMBDA_SETS["fp64"][0]
            r = {"reference": "the FP64 oracle on its resolvable set Lambda <= 16",
                 "frac_grid_in_set": float(r64.mean())}
            for name, Sr in runs.items():
                with np.errstate(invalid="ignore"):
                    e = np.abs(Sr - o5["S"]) / np.maximum(np.abs(o5["S"]), p5.hbar)
                e = np.nan_to_num(e, nan=np.inf)
                r[f"{name}_frac_of_set_within_1e-4"] = float(np.mean(e[r64] <= 1e-4))
                r[f"{name}_max_rel_on_set"] = float(e[r64].max())
            res["noise2d_2048x2048_fp32"] = r
        out["far_field"] = res
    if "solve3d" in gpu:
        progress("accuracy: solve3d")
        p3, r3, (rec3, gradient3) = gpu["solve3d"]
        f3 = p3.f.astype(np.float64)
        o3 = oracle.solve(f3, p3.src, p3.h, p3.hbar, p3.T, nthreads=threads)
        out["solve3d"] = {"workload": "blobs3d_256x256x256_T16",
                          **{k: accuracy(v, o3, p3.hbar, k) for k, v in r3.items()}}
        # the gradient of the same kind of loss, formed from the oracle's S
        idx = tuple(rec3.T)
        dLdS3 = np.zeros(p3.dims)
        dLdS3[idx] = 2.0 * (o3["S"][idx] - 0.97 * o3["S"][idx])
        g_o, _ = oracle.adjoint(f3, p3.src, p3.h, p3.hbar, p3.T, dLdS3, nthreads=threads)
        g3 = gradient3(dLdS3)
        out["solve3d"]["gradient_fp32"] = {
            "normwise_rel": float(np.linalg.norm(g3 - g_o) / np.linalg.norm(g_o)), "tol": 1e-3,
            "dLdS": "2 (S - 0.97 S) at 256 receivers near the source, S the oracle's"}
    return out


# ---- counter and trace summaries --------------------------------------------

def _counter_rows(path):
    files = [path] if os.path.isfile(path) else glob.glob(
        os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for fn in files:
        with open(fn) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value)} summed over the counter's
    instances within the dispatch."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        prev = out.get(d, (name, 0.0))
        out[d] = (name, prev[1] + v)
    return out


def traffic_summary(fetch_path, write_path, command):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the term-row
    kernel of every schedule in the runs, and of the calibration copy; the
    copy's reading over its known byte count is the factor that turns counter
    KiB into HBM bytes."""
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_path), ("WRITE_SIZE", write_path)):
        disp = _per_dispatch(_counter_rows(path), counter)
        ids = sorted(disp)
        term, copy = {}, []
        for j, d in enumerate(ids):
            name, v = disp[d]
            if "neg" in name.lower():
                copy.append(v)
            elif "k_row2<float, 2, 1024," in name:
                # term-row dispatches of a solve are followed by a column
                # pass (the last one, the log pass, by the next solve's prep)
                nxt = disp[ids[j + 1]][0] if j + 1 < len(ids) else ""
                if "k_col2" in nxt:
                    e = name.split("k_row2<float, 2, 1024,")[1].split(">")[0].strip()
                    term.setdefault(e, []).append(v)
        if not term or not copy:
            raise SystemExit(f"{counter}: no term-row or copy dispatches in {path}")
        res[counter] = {"copy_kib": float(np.mean(copy)), "copy_dispatches": len(copy),
                        "term_row_kib": {e: float(np.mean(x)) for e, x in term.items()},
                        "term_row_dispatches": {e: len(x) for e, x in term.items()}}
    copy_bytes = 4.0 * COPY_ELEMS
    f_fac = res["FETCH_SIZE"]["copy_kib"] * 1024.0 / copy_bytes
    w_fac = res["WRITE_SIZE"]["copy_kib"] * 1024.0 / copy_bytes
    per = {}
    for e in sorted(set(res["FETCH_SIZE"]["term_row_kib"]) & set(res["WRITE_SIZE"]["term_row_kib"])):
        fb = res["FETCH_SIZE"]["term_row_kib"][e] * 1024.0 / f_fac
        wb = res["WRITE_SIZE"]["term_row_kib"][e] * 1024.0 / w_fac
        per[e] = {"kernel": f"k_row2<float, ROW_TERM, 1024, {e}>", "fetch_bytes_per_launch": fb,
                  "write_bytes_per_launch": wb, "traffic_bytes_per_launch": fb + wb}
    d = {"kernel": "term_row (k_row2<float, ROW_TERM, 1024, E> for each schedule E)",
         "workload": "noise2d_1024x1024_T16_src16 fp32-scaled",
         "counters": res,
         "copy_bytes_each_way": copy_bytes,
         "fetch_factor": f_fac, "write_factor": w_fac,
         "per_schedule": per,
         "source_hash": source_hash()}
    head = ("HBM traffic of the term-row kernel (FETCH_SIZE and WRITE_SIZE, one rocprofv3\n"
            "--pmc run each, solves with row schedules 8 and 16), scaled by the same\n"
            "counters' reading for a plain float32 elementwise copy (torch.neg) of known size.\n"
            f"command: {command}\n")
    return head + "\n---\n" + json.dumps(d, indent=1) + "\n"


def sq_summary(paths, command, kernels=("k_row2<float, 2,", "k_col2<float, 1,")):
    """Per-dispatch averages of the SQ_* counters of one or more rocprofv3
    --pmc runs for the kernels whose names contain the given fragments (the
    term-row and column-convolution passes by default), with the ratios used
    to read them: cycles per wave waiting, VALU issue per SIMD, LDS
    instructions and bank-conflict cycles per wave."""
    agg, dur = {}, {}
    for path in paths:
        for r in _counter_rows(path):
            name = r["Kernel_Name"]
            key = next((k for k in kernels if k in name), None)
            if key is None:
                continue
            full = name.split("(")[0]
            d = agg.setdefault(full, {}).setdefault(r["Counter_Name"], {})
            disp = (path, int(r["Dispatch_Id"]))  # dispatch ids restart in every run
            d[disp] = d.get(disp, 0.0) + float(r["Counter_Value"])
            dur.setdefault(full, {})[disp] = (int(r["End_Timestamp"]) -
                                               int(r["Start_Timestamp"])) * 1e-3
    out = {}
    for name, cnt in agg.items():
        avg = {c: float(np.mean(list(v.values()))) for c, v in cnt.items()}
        n = {c: len(v) for c, v in cnt.items()}
        us = float(np.median(list(dur[name].values())))
        row = {"dispatches": max(n.values()), "median_us_under_counters": us, "per_dispatch": avg}
        w = avg.get("SQ_WAVES")
        if w:
            if "SQ_WAVE_CYCLES" in avg:
                row["wave_cycles_per_wave"] = avg["SQ_WAVE_CYCLES"] / w
            if "SQ_WAIT_INST_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
                row["frac_wave_cycles_waiting_inst"] = avg["SQ_WAIT_INST_ANY"] / avg["SQ_WAVE_CYCLES"]
            if "SQ_WAIT_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
                row["frac_wave_cycles_waiting_any"] = avg["SQ_WAIT_ANY"] / avg["SQ_WAVE_CYCLES"]
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
                      "SQ_INSTS_VMEM_WR", "SQ_INSTS_SMEM", "SQ_INSTS_BRANCH"):
                if c in avg:
                    row[c.lower().replace("sq_insts_", "insts_") + "_per_wave"] = avg[c] / w
        if "SQ_INSTS_VALU" in avg:
            # one wave64 VALU instruction occupies a SIMD for 4 cycles (16 lanes);
            # 1024 SIMDs at 2.4 GHz
            row["valu_issue_us_per_simd"] = avg["SQ_INSTS_VALU"] * 4 / (256 * 4) / 2.4e3
            row["valu_busy_frac"] = row["valu_issue_us_per_simd"] / us
        if "SQ_ACTIVE_INST_VALU" in avg:
            row["valu_active_us_per_simd"] = avg["SQ_ACTIVE_INST_VALU"] / (256 * 4) / 2.4e3
        out[name] = row
    head = ("SQ counters of the named kernels (per-dispatch averages over the runs; one\n"
            "rocprofv3 --pmc run per counter group), with derived ratios; valu_busy_frac is\n"
            "the VALU issue time per SIMD over the kernel's duration under the counters.\n"
            f"command: {command}\n")
    return head + "\n---\n" + json.dumps(out, indent=1) + "\n"


def stats_summary(csv_path, command, top=12):
    with open(csv_path) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    lines = [f"command: {command}", "",
             f"{'calls':>6} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'pct':>6}  kernel"]
    for r in rows[:top]:
        name = r["Name"]
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} "
                     f"{float(r['Percentage']):6.2f}  {name}")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--n", type=int, default=1024, help="grid edge of the main workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip fwd+bwd and batched")
    ap.add_argument("--only", choices=["fwd_bwd", "batched", "solve3d", "backtrack", "fd",
                                       "config1", "far_field", "large"],
                    help="run one extra section alone and print its JSON (profiling runs)")
    ap.add_argument("--pmc-run", action="store_true")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH", "WRITE"))
    ap.add_argument("--stats-summary", metavar="CSV")
    ap.add_argument("--sq-summary", nargs="+", metavar="DIR",
                    help="summarise the SQ_* counters of rocprofv3 --pmc runs")
    ap.add_argument("--sq-kernels", default="k_row2<float, 2,;k_col2<float, 1,",
                    help="kernel-name fragments for --sq-summary, separated by ';'")
    ap.add_argument("--command", default="", help="command text recorded in a summary")
    ap.add_argument("--out", help="summary output file")
    args = ap.parse_args()

    if args.traffic_summary or args.stats_summary or args.sq_summary:
        text = (traffic_summary(*args.traffic_summary, args.command) if args.traffic_summary
                else sq_summary(args.sq_summary, args.command, args.sq_kernels.split(";"))
                if args.sq_summary
                else stats_summary(args.stats_summary, args.command))
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(text)
        print(text)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 "
                                   "(independent instances would be spread over GPUs by the "
                                   "caller; a single grid is not split)"}))
        sys.exit(2)

    import torch
    import paper_1403_1937_amd as pk
    import workloads

    if not os.path.exists(pk.lib_path()):
        raise SystemExit(f"{pk.lib_path()} is not built: run paper_1403_1937_amd/build.py")
    dev = torch.device("cuda:0")
    p = workloads.problem(2, args.n)
    n0, n1 = p.dims
    N = n0 * n1

    if args.only:
        fn = {"fwd_bwd": run_fwd_bwd, "batched": run_batched, "solve3d": run_3d,
              "backtrack": run_backtrack, "fd": run_fd, "config1": run_config1,
              "far_field": run_far_field, "large": run_large}[args.only]
        r = fn(pk, torch, dev, args.steps, args.warmup)
        print(json.dumps(r[0] if isinstance(r, tuple) else r))
        return

    if args.pmc_run:
        a = torch.rand(COPY_ELEMS, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
        for sched in ((8, 16), (16, 16)):  # the two row schedules the tuner picks at 1024^2
            ms, _, _, _ = run_main(pk, torch, dev, p, "fp32", args.steps, args.warmup, sched)
            print(f"pmc run, schedule {sched}: {ms:.3f} ms per solve", flush=True)
        return

    ms, kern, total_bytes, S_main = run_main(pk, torch, dev, p, args.precision, args.steps,
                                             args.warmup)
    progress(f"main workload: {ms:.3f} ms per solve")
    gpu = {}  # host copies of the GPU results, for the accuracy figures
    value = N / (ms * 1e-3)
    sched = kern.pop("schedule")
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches_per_step"])
    d = kern[dom]
    traffic = read_traffic(source_hash(), sched["row_e"]) if (
        dom == "term_row" and args.precision == "fp32" and args.n == 1024) else None
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
                   "mode": "fwd", "schedule": sched},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["GBps"],
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": d["GBps"] / HBM_PEAK_GBPS, "traffic": traffic,
                     "alg_bytes_per_launch": d["alg_bytes"], "avg_us": d["avg_us"]},
        "solve_alg_GBps": total_bytes / (ms * 1e-3) / 1e9,
        "solve_alg_bytes": total_bytes,
        "kernels": kern,
    }
    S64_main = None
    if not args.no_fp64 and args.precision == "fp32":
        ms64, _, tb64, S64_main = run_main(pk, torch, dev, p, "fp64", max(5, args.steps // 2), 2)
        out["fp64_comparator"] = {"value": N / (ms64 * 1e-3), "ms_per_step": ms64,
                                  "solve_alg_GBps": tb64 / (ms64 * 1e-3) / 1e9,
                                  "speedup_fp32_over_fp64": ms64 / ms}
        progress(f"fp64 comparator: {ms64:.3f} ms per solve")
    gpu["main"] = (p, S_main, S64_main) if args.precision == "fp32" else (p, None, S_main)
    if not args.no_extra:
        out["config1"], gpu["config1"] = run_config1(pk, torch, dev, max(20, args.steps), 3)
        progress("config1")
        out["far_field"], gpu["far_field"] = run_far_field(pk, torch, dev, max(10, args.steps // 2), 2)
        progress("far_field")
        out["fwd_bwd"], gpu["fwd_bwd"] = run_fwd_bwd(pk, torch, dev, max(3, args.steps // 2), 2)
        progress("fwd_bwd")
        out["batched"], gpu["batched"] = run_batched(pk, torch, dev, max(3, args.steps // 4), 1)
        progress("batched")
        out["solve3d"], gpu["solve3d"] = run_3d(pk, torch, dev, max(3, args.steps // 4), 1)
        progress("solve3d")
        out["backtrack"] = run_backtrack(pk, torch, dev, max(3, args.steps // 4), 1)
        progress("backtrack")
        out["fd"] = run_fd(pk, torch, dev, 3, 1)
        progress("fd")
        out["large_grids"] = run_large(pk, torch, dev, 3, 1)
        progress("large_grids")
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"], o_main = cpu_baseline(p, threads)
        progress("cpu_baseline")
        if args.precision == "fp32":
            out["accuracy"] = reference_accuracy(gpu, o_main, threads)
            progress("accuracy against the oracle")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
