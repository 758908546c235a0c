#!/usr/bin/env python3
"""Benchmark of the MI355X MGWR solver: space-time unknowns per second to a
1e-10 relative residual, mixed precision against FP64, on one GPU.

Workload (default "1d"): the 1D time-fractional heat equation on (0,1) x (0,1]
with N = 4095 interior points and M = 16384 time steps, alpha in {0.3, 0.7},
forcing = manufactured term of u = t^2 sin(pi x) plus a seeded 20-mode random
field (paper_1608_05400_amd.workloads.config2).  One step solves both alpha
problems from u = 0 with a V(1,1) cycle until the FP64 residual is reduced by
--tol in the max norm.  Inputs are resident in HBM before the timed region.

Modes: "fp32" (FP32 history products in the cycle on the error equation,
FP64 double-double refinement; the reported value on this workload), "fp64"
(Algorithm 1 in FP64 on u; on the default workload it stops at its rounding
floor above the tolerance, flagged in the JSON line), "bf16x3" (split-BF16
matrix-core history products where the autotuner finds them faster, else
FP32), "fp64r" (FP64 cycle on the error with double-double refinement: the
FP64 method that reaches the tolerance).  Each mode's `dtype` lists the
arithmetic its Toeplitz products actually ran in, from the library's
per-launch records, and `products_ms_per_step` their time by arithmetic.

Before the timed steps each handle is autotuned (FFT or dense route per
level, tile shapes of the dense product kernels, and D&C base blocks with
--smoother auto/dc); the tuning time is reported apart from the timed steps,
like handle creation.  The timed steps issue the products one by one between
HIP events (the roofline's launch times); one more step replays the recorded
HIP graphs and is reported beside them.

The default run also measures, as `extra_workloads`, the 2D problem
(N = 511 per dimension, M = 2048, alpha = 0.4, u = t^2 sin(pi x) sin(pi y)),
the 2D problem with a non-smooth solution (N = 1023, M = 1024, alpha = 0.3,
u = (t^alpha + t^2) sin(pi x) sin(pi y)), both in the split-BF16 mode, and
the batch of 256 independent 1D problems of uneven size (N in {127..2047},
M in {256..8192}, alpha in (0.1, 0.9), seeded; every stage of their cycles
is one launch over all problems still iterating) in the FP32 mode, each
also in plain FP64.  `cpu_baseline` is the oracle's direct solve of the
first problem, all of it, timed on the host's cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "space-time unknowns/sec to 1e-10 rel residual, mixed vs FP64 MGWR, 1 GPU"
PEAK_TFLOPS = {0: 78.6, 1: 157.3, 2: 2500.0}   # MI355X dense: FP64, FP32, BF16 MFMA


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workloads(name):
    from paper_1608_05400_amd import workloads as W
    if name == "1d":
        return [W.config2(0.3), W.config2(0.7)], "1d_N4095_M16384_alpha0.3+0.7"
    if name == "2d":
        return [W.manufactured_2d(511, 2048, 0.4)], "2d_N511_M2048_alpha0.4"
    if name == "2dns":
        return [W.nonsmooth_2d(1023, 1024, 0.3)], "2d_nonsmooth_N1023_M1024_alpha0.3"
    if name == "small":
        return [W.manufactured_1d()], "1d_N63_M64_alpha0.5"
    if name == "batch":
        return W.batch_1d(), "batch256_1d_N127-2047_M256-8192"
    raise SystemExit(f"unknown workload {name}")


def sampled_error(w, u_dev, npts=4096, seed=0):
    """Max relative error of u against the exact discrete solution at sampled
    space-time points, from the oracle's modal solve (the forcing is a finite
    sum of sine modes)."""
    import oracle
    rng = np.random.default_rng(seed)
    v = oracle.modal_solve(w.dims, w.N, w.M, w.alpha, w.kx, w.s, ky=w.ky)
    m = rng.integers(1, w.M + 1, size=npts)
    m[:64] = w.M
    n = rng.integers(1, w.N + 1, size=npts)
    l = rng.integers(1, w.N + 1, size=npts) if w.dims == 2 else np.ones(npts, dtype=np.int64)
    ref = oracle.modal_eval(w.dims, w.N, w.M, w.kx, v, np.stack([m, n, l], 1), ky=w.ky)
    import torch
    if w.dims == 1:
        idx = (m - 1) * w.N + (n - 1)
    else:
        idx = (m - 1) * w.N * w.N + (l - 1) * w.N + (n - 1)
    got = u_dev.reshape(-1)[torch.from_numpy(idx).to(u_dev.device)].cpu().numpy()
    return float(np.abs(got - ref).max() / np.abs(ref).max())


class _BatchRunner:
    """The whole workload as one batch handle."""

    def __init__(self, B, wls, mode, smoother):
        self.b = B.Batch([w.N for w in wls], [w.M for w in wls], [w.alpha for w in wls],
                         [w.T for w in wls], dims=wls[0].dims, precision=mode, maxit=40, smoother=smoother)

    def autotune(self):
        return self.b.autotune()

    def solve(self, fs, us, tol):
        _, infos = self.b.solve(fs, us, tol=tol)
        return infos

    def profile(self, on):
        self.b.profile(on)

    def records(self):
        return self.b.profile_records()

    def close(self):
        self.b.close()


class _SingleRunner:
    """One handle per problem, solved one after the other."""

    def __init__(self, B, wls, mode, smoother):
        self.ss = [B.Solver(w.N, w.M, w.alpha, T=w.T, dims=w.dims, precision=mode, maxit=40, smoother=smoother)
                   for w in wls]

    def autotune(self):
        return [s.autotune() for s in self.ss][0]

    def solve(self, fs, us, tol):
        return [s.solve(f, u, tol=tol) for s, f, u in zip(self.ss, fs, us)]

    def profile(self, on):
        for s in self.ss:
            s.profile(on)

    def records(self):
        return [r for s in self.ss for r in s.profile_records()]

    def close(self):
        for s in self.ss:
            s.close()


def run_mode(mode, wls, fs, steps, warmup, tol, check, profile, batch=False, autotune=True,
             smoother="inverse", graph_step=True):
    """Autotune, warm up, then time `steps` solves of every problem of the
    workload in one precision mode; returns (results, product records)."""
    import torch
    from paper_1608_05400_amd import binding as B
    runner = (_BatchRunner if batch else _SingleRunner)(B, wls, mode, smoother)
    us = [torch.zeros((w.M, w.N) if w.dims == 1 else (w.M, w.N, w.N), dtype=torch.float64, device="cuda")
          for w in wls]
    tuning = None
    t_tune = 0.0
    if autotune:
        t = time.perf_counter()
        tuning = runner.autotune()
        t_tune = time.perf_counter() - t
        log(f"{mode}: autotuned in {t_tune:.1f} s: {tuning}")
    infos = []
    for it in range(warmup):
        runner.solve(fs, us, tol)
        log(f"{mode}: warmup {it + 1}/{warmup} done")
    # the timed steps bracket every product launch with HIP events (so the
    # launches are issued one by one); one more step replays the recorded
    # HIP graphs, the path of repeated solves, and is reported beside them
    if profile:
        runner.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        infos = runner.solve(fs, us, tol)
        log(f"{mode}: step {k + 1}/{steps} done, iters {summ([i['iters'] for i in infos])}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    records = []
    if profile:
        records = runner.records()
        runner.profile(False)
    ms_graph = None
    if graph_step:
        runner.solve(fs, us, tol)   # records the graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        runner.solve(fs, us, tol)
        torch.cuda.synchronize()
        ms_graph = 1e3 * (time.perf_counter() - t)
        log(f"{mode}: graph-replay step {ms_graph:.1f} ms")
    unknowns = sum(w.unknowns for w in wls)
    res = {
        "mode": mode,
        "dtype": dtype_label(records),
        "products_ms_per_step": products_by_dtype(records, steps),
        "value": unknowns * steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "iters": summ([i["iters"] for i in infos]),
        "status": summ([i["status"] for i in infos]),
        "relres": summ([i["relres"] for i in infos]),
        "mean_factor": summ([round(i["mean_factor"], 5) for i in infos]),
        "ms_per_step_graph_replay": ms_graph,
        "tuning": tuning,
        "tune_s": round(t_tune, 2),
    }
    if check:
        idx = range(len(wls)) if len(wls) <= 4 else sorted(range(len(wls)), key=lambda i: -wls[i].unknowns)[:4]
        res["err_vs_oracle"] = [sampled_error(wls[i], us[i]) for i in idx]
    runner.close()
    del us
    torch.cuda.empty_cache()
    return res, records


def summ(v):
    """A per-problem list, or its summary for long lists."""
    if len(v) <= 8:
        return v
    if isinstance(v[0], str):
        return {k: v.count(k) for k in sorted(set(v))}
    return {"min": min(v), "max": max(v), "mean": sum(v) / len(v)}


def measured_traffic(kernel_name):
    """HBM bytes per launch of a kernel from the committed counter runs
    (profiles/traffic.json), or None when the kernel source has changed since
    the counters were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        rec = json.load(open(os.path.join(here, "profiles", "traffic.json"))).get(kernel_name)
        src = open(os.path.join(here, "paper_1608_05400_amd", "csrc", "mgwr_kernels.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec


HBM_PEAK_GBS = 8000.0


DTYPE_OF_MODE = {0: "f64", 1: "f32", 2: "bf16x3"}


def products_by_dtype(records, steps):
    """Milliseconds per step of the Toeplitz products by the arithmetic they
    ran in (kernel id bits 4..7), from the per-launch records."""
    out = {}
    for r in records:
        k = DTYPE_OF_MODE[(r["kernel"] >> 4) & 15]
        out[k] = out.get(k, 0.0) + r["ms"]
    return {k: round(v / max(1, steps), 3) for k, v in sorted(out.items(), key=lambda kv: -kv[1])}


def dtype_label(records):
    """The arithmetic the products actually ran in, FP64 first ("f64+f32")."""
    seen = {DTYPE_OF_MODE[(r["kernel"] >> 4) & 15] for r in records}
    order = [d for d in ("f64", "f32", "bf16x3") if d in seen]
    return "+".join(order) if order else None


def roofline_of(records, steps, batch=False):
    """Dominant Toeplitz-product kernel class (largest total time) and its
    achieved rate from the per-launch HIP events.  Dense kernels: algorithmic
    FLOP/s against the matrix cores of their dtype.  FFT route: the products'
    own bytes (operand read once, epilogue reads and writes, as the library
    records them per product) per second against HBM, with the bytes of the
    passes' work arrays added in `pass_structure`; for one problem the
    class's finest-level launches (all its levels share the three kernels),
    for a batch all its launches."""
    if not records:
        return None
    from paper_1608_05400_amd import binding as B
    by = {}
    for r in records:
        d = by.setdefault(r["kernel"], {"ms": 0.0, "flops": 0.0, "n": 0})
        d["ms"] += r["ms"]
        d["flops"] += r["flops"]
        d["n"] += 1
    kid = max(by, key=lambda k: by[k]["ms"])
    d = by[kid]
    mode = (kid >> 4) & 15
    share = round(d["ms"] / sum(v["ms"] for v in by.values()), 3)
    rs = [r for r in records if r["kernel"] == kid]
    if (kid >> 8) == 4:
        if not batch:
            top = max(r["level"] for r in rs)
            rs = [r for r in rs if r["level"] == top]
        ms = sum(r["ms"] for r in rs)
        nbytes = sum(r["bytes"] for r in rs)
        pbytes = sum(r["bytes"] + r["pass_bytes"] for r in rs)
        achieved = nbytes / (ms * 1e-3) / 1e9
        out = {
            "bound": "hbm",
            "kernel": B.kernel_name(kid),
            "dtype": "f64" if mode == 0 else "f32",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": nbytes / len(rs),
            "bytes_definition": "the product's own bytes: operand read once + epilogue reads and writes",
            "pass_structure": {
                "bytes_per_launch": pbytes / len(rs),
                "achieved": round(pbytes / (ms * 1e-3) / 1e9, 1),
                "frac": round(pbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "definition": "own bytes + the complex work arrays written and read between the passes",
            },
            "launches": len(rs),
            "launches_per_step": round(len(rs) / max(1, steps), 2),
            "avg_launch_ms": round(ms / len(rs), 4),
            "share_of_product_time": share,
        }
        if not batch:
            out["level"] = top
            out["P"] = sorted(set(r["P"] for r in rs))
            out["M"] = rs[0]["M"]
            tr = measured_traffic(out["kernel"])
            if tr and tr.get("level") == top and tr.get("P") == out["P"]:
                out["traffic"] = tr["bytes_per_launch"]
                out["traffic_unit"] = "bytes/launch (FETCH_SIZE x %g + WRITE_SIZE x %g)" % (tr["fetch_factor"],
                                                                                           tr["write_factor"])
        return out
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[mode]
    nbytes = sum(r["bytes"] for r in rs)
    out = {
        "bound": "mfma",
        "kernel": B.kernel_name(kid),
        "dtype": DTYPE_OF_MODE[mode],
        "achieved": round(achieved, 2),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": None,
        "bytes_per_launch": nbytes / len(rs),
        "hbm_gbs_of_own_bytes": round(nbytes / (d["ms"] * 1e-3) / 1e9, 1),
        "launches": d["n"],
        "launches_per_step": round(d["n"] / max(1, steps), 2),
        "avg_launch_ms": round(d["ms"] / d["n"], 4),
        "avg_launch_gflop": round(d["flops"] / d["n"] / 1e9, 3),
        "share_of_product_time": share,
    }
    if mode == 2:
        out["issued_frac"] = round(3 * achieved / peak, 4)   # three BF16 passes per product
    tr = measured_traffic(out["kernel"])
    if tr:
        out["traffic"] = tr["bytes_per_launch"]
        out["traffic_unit"] = "bytes/launch (FETCH_SIZE x %g + WRITE_SIZE x %g)" % (tr["fetch_factor"],
                                                                                   tr["write_factor"])
    return out


def kernel_table(records, steps):
    """Per (kernel, level, columns) totals of the product launches."""
    by = {}
    for r in records:
        k = (r["name"], r["level"], r["P"])
        d = by.setdefault(k, [0, 0.0, 0.0])
        d[0] += 1
        d[1] += r["ms"]
        d[2] += r["flops"]
    rows = []
    for (name, lev, P), (n, ms, fl) in sorted(by.items(), key=lambda kv: -kv[1][1]):
        rows.append({"kernel": name, "level": lev, "P": P, "launches_per_step": n / steps,
                     "ms_per_step": ms / steps, "avg_ms": ms / n, "tflops": fl / (ms * 1e-3) / 1e12})
    return rows


def bench_fas(B, args):
    """The nonlinear problem of Section 7 on Table 5's largest grid (N = 255,
    M = 256, D(u) = 1 + u^2, c = 1, f = 1, V(0,1) FAS to a 1e-10 max-norm
    reduction) for the four fractional orders of the table: one step solves
    all four as one batch (mgwr_fas_solve_batch).  The oracle's FAS iteration on the same problems is the CPU
    baseline.  Prints one JSON line."""
    import torch
    import oracle
    N, M, alphas = 255, 256, (0.1, 0.4, 0.7, 1.0)
    f = torch.ones((M, N), dtype=torch.float64, device="cuda")
    us = [torch.zeros((M, N), dtype=torch.float64, device="cuda") for _ in alphas]

    def step():   # the four problems as one batch: their kernels overlap
        return B.fas_solve_batch([f] * len(alphas), us, alphas, tol=args.tol)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    unknowns = len(alphas) * M * N
    err = max(float(np.abs(u.cpu().numpy() - oracle.nl_solve(N, M, a, np.ones((M, N)), tol=args.tol)[0]).max())
              for u, a in zip(us, alphas)) if not args.no_check else None
    line = {"metric": "space-time unknowns/sec to 1e-10 rel residual, nonlinear FAS (Section 7, Table 5 grid)",
            "value": unknowns / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "fas_1d_N255_M256_alpha0.1,0.4,0.7,1.0", "cycle": "V(0,1)", "tol": args.tol},
            "iters": [i["iters"] for i in infos], "max_diff_vs_oracle": err}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        for a in alphas:
            oracle.nl_solve(N, M, a, np.ones((M, N)), tol=args.tol)
        s_cpu = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": unknowns / s_cpu, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
                                "sample": f"the oracle's FAS solves of the same four problems: {s_cpu:.2f} s"}
    log(f"fas: {line['value']:.4g} unknowns/s, {ms:.1f} ms per step of four solves, iters {line['iters']}")
    print(json.dumps(line), flush=True)


def bench_products(B, args):
    """The dense matrix-core Toeplitz products on their own (mgwr_toeplitz_apply
    on a handle with the FFT route off), at the shapes of the benchmark
    workloads: the residual product of the 1D N = 4095, M = 16384 problem
    (T_M times all 4095 columns) and a smoother product of the 2D N = 511,
    M = 2048 problem (one colour, 130560 columns), in FP64, FP32 and split
    BF16.  Per-launch times from the library's HIP events; algorithmic flops
    2 x (multiply-adds not structurally zero).  Prints one JSON line."""
    import torch
    shapes = [("1d_residual_N4095_M16384", 1, 4095, 16384, 0.3, 4095),
              ("2d_smoother_N511_M2048", 2, 511, 2048, 0.4, 130560)]
    out = {}
    for name, dims, N, M, alpha, P in shapes:
        X = torch.randn((M, P), dtype=torch.float64, device="cuda")
        for prec in ("fp64", "fp32", "bf16x3"):
            with B.Solver(N, M, alpha, dims=dims, fft=0, precision=prec) as s:
                # T_M for the residual, the finest level's inverse column for the smoother
                which = -1 if "residual" in name else s.levels() - 1
                C = torch.empty_like(X)
                for _ in range(args.warmup):
                    s.toeplitz_apply(X, which=which, precision=prec, C=C)
                torch.cuda.synchronize()
                s.profile(True)
                for _ in range(args.steps):
                    s.toeplitz_apply(X, which=which, precision=prec, C=C)
                recs = s.profile_records()
                s.profile(False)
            ms = sum(r["ms"] for r in recs) / len(recs)
            fl = recs[0]["flops"]
            tf = fl / (ms * 1e-3) / 1e12
            out[f"{name}_{prec}"] = {"kernel": recs[0]["name"], "avg_ms": round(ms, 4), "gflop": round(fl / 1e9, 2),
                                     "tflops": round(tf, 1), "peak": PEAK_TFLOPS[{"fp64": 0, "fp32": 1, "bf16x3": 2}[prec]],
                                     "launches": len(recs)}
            log(f"{name} {prec}: {recs[0]['name']} {ms:.3f} ms, {tf:.1f} TFLOP/s")
        del X
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "products", "results": out}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, levels=0):
    """The oracle's direct time-stepping solve of one problem of the workload
    (all M time levels unless `levels` > 0), timed on the host's cores; the
    rate is the unknowns it solved per second, without extrapolation."""
    import oracle
    f = w.forcing()
    oracle.direct_solve(w.dims, w.N, w.M, w.alpha, f, Mstop=16)   # load, page in
    Ms = w.M if levels <= 0 else min(levels, w.M)
    t = time.perf_counter()
    oracle.direct_solve(w.dims, w.N, w.M, w.alpha, f, Mstop=Ms)
    ts = time.perf_counter() - t
    unknowns = w.unknowns * Ms // w.M
    what = "all" if Ms == w.M else f"the first {Ms} of the {w.M}"
    return {"value": unknowns / ts, "unit": "unknowns/s", "cores": oracle.max_threads(), "kind": "oracle",
            "cpu": cpu_model(), "seconds": round(ts, 2),
            "sample": (f"the oracle's direct time-stepping solve (Thomas per level, O(N M^2) history sum) "
                       f"of {w.name}, {what} time levels: {unknowns} unknowns in {ts:.2f} s")}


def calibrate_copy(mib=512, reps=3):
    """A plain device-to-device copy of known size (for scaling the HBM
    byte counters of a profiler run: each copy reads and writes mib MiB)."""
    import torch
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": reps}), flush=True)


# Precision modes per workload, the first one reported as `value`: the mixed
# mode whose products actually run there.  On the 1D N = 4095, M = 16384
# problems and on the batch every mixed product takes the FP32 FFT route (the
# split-BF16 products lose to it at M >= 4096 and on the batch's many small
# levels, so the split-BF16 mode's tuner picks the same FP32 products); on
# the 2D workload the split-BF16 matrix-core products win on the levels with
# many columns and are chosen there.
DEFAULT_MODES = {"1d": "fp32,fp64,bf16x3,fp64r", "2d": "bf16x3,fp64,fp32,fp64r",
                 "2dns": "bf16x3,fp64,fp32,fp64r", "small": "fp32,fp64,bf16x3,fp64r",
                 "batch": "fp32,fp64,bf16x3,fp64r"}
# Workloads measured after the default one and reported beside it (mixed
# mode and plain FP64, fewer steps).
EXTRA = {"2d": "bf16x3,fp64", "2dns": "bf16x3,fp64", "batch": "fp32,fp64"}


def log_kernels(mode, res, recs, steps):
    for row in kernel_table(recs, steps)[:14]:
        log(f"  {row['kernel']:22s} lvl {row['level']:2d} P {row['P']:6d}: "
            f"{row['launches_per_step']:5.1f}/step {row['ms_per_step']:8.2f} ms/step "
            f"avg {row['avg_ms']:7.3f} ms {row['tflops']:7.1f} TFLOP/s")
    log(f"{mode}: {res['value']:.4g} unknowns/s, {res['ms_per_step']:.1f} ms/step, dtype {res['dtype']}, "
        f"iters {res['iters']}, relres {res['relres']}, err {res.get('err_vs_oracle')}")


def compare_fp64(line, results, primary):
    """Speedup of the primary mode over the FP64 modes; a mode that stops
    short of the tolerance (plain FP64 stagnates at its rounding floor on
    the 1D workload) is flagged: its rate is not to the same accuracy."""
    p = results[primary]
    for m in ("fp64", "fp64r"):
        if m in results and primary != m:
            line["speedup_vs_" + m] = p["value"] / results[m]["value"]
            st = results[m]["status"]   # per problem, or counts per status
            line[m + "_reaches_tol"] = all(x == "ok" for x in st) if isinstance(st, list) else set(st) == {"ok"}


def run_workload(name, modes, args, steps, warmup, all_steps=True):
    """Every mode of one workload; returns (results, rooflines, name)."""
    import torch
    wls, wname = make_workloads(name)
    fs = [w.forcing_torch("cuda").contiguous() for w in wls]
    torch.cuda.synchronize()
    log(f"workload {wname}: {sum(w.unknowns for w in wls)} unknowns per step")
    results, rooflines = {}, {}
    for i, mode in enumerate(modes):
        k = steps if (i < 2 or all_steps is False) else 1
        res, recs = run_mode(mode, wls, fs, k, warmup if i < 2 else 1, args.tol, not args.no_check,
                             profile=not args.no_profile, batch=name == "batch",
                             autotune=not args.no_autotune, smoother=args.smoother, graph_step=i < 2 and all_steps)
        results[mode] = res
        rooflines[mode] = roofline_of(recs, k, batch=name == "batch")
        log_kernels(mode, res, recs, k)
    del fs
    torch.cuda.empty_cache()
    return results, rooflines, wname


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="1d", choices=["1d", "2d", "2dns", "small", "batch", "fas", "products"])
    ap.add_argument("--smoother", default="inverse", choices=["inverse", "dc", "auto"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 512 MiB device copy three times (profiler counter calibration)")
    ap.add_argument("--modes", default=None, help="comma-separated precision modes, the first one reported")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-levels", type=int, default=0,
                    help="time the oracle on the first K time levels only (default: the whole solve)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2D, 2D non-smooth and batch workloads of the default run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (one problem or one batch per GPU); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.calibrate_copy:
        calibrate_copy()
        return
    from paper_1608_05400_amd import binding as B
    B.load()
    if args.workload == "fas":
        return bench_fas(B, args)
    if args.workload == "products":
        return bench_products(B, args)
    modes = [m.strip() for m in (args.modes or DEFAULT_MODES[args.workload]).split(",") if m.strip()]
    results, rooflines, wname = run_workload(args.workload, modes, args, args.steps, args.warmup)
    primary = modes[0]
    p = results[primary]
    line = {
        "metric": METRIC,
        "value": p["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": p["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": p["dtype"] or "f64",
        "data": "synthetic",
        "config": {"workload": wname, "mode": primary, "cycle": "V(1,1)", "tol": args.tol,
                   "norm": "max", "smoother": args.smoother, "autotuned": not args.no_autotune},
        "roofline": rooflines.get(primary),
        "modes": results,
        "rooflines": rooflines,
    }
    compare_fp64(line, results, primary)
    if args.workload == "1d" and not args.no_extra and not args.modes:
        extra = {}
        for name, ms in EXTRA.items():
            em = ms.split(",")
            r, rl, en = run_workload(name, em, args, min(args.steps, 2), 1, all_steps=False)
            e = {"workload": en, "mode": em[0], "value": r[em[0]]["value"], "unit": "unknowns/s",
                 "ms_per_step": r[em[0]]["ms_per_step"], "dtype": r[em[0]]["dtype"],
                 "roofline": rl[em[0]], "modes": r}
            compare_fp64(e, r, em[0])
            extra[name] = e
        line["extra_workloads"] = extra
    if not args.no_cpu_baseline:
        wls, _ = make_workloads(args.workload)
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(wls[0], args.cpu_levels)
        log(f"cpu baseline: {line['cpu_baseline']['value']:.4g} unknowns/s in {line['cpu_baseline']['seconds']} s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
