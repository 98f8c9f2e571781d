#!/usr/bin/env python3
"""Benchmark of the lens-equation hot path on one MI355X.

Workload: the cluster-scale single-plane case (2 elliptical dPIE halos + 300 circular
dPIE members on the Sec. 3.4 scaling relations, 2048^2 grid over 200", 60 sources /
150 images, 1024 parameter samples), synthetic and seeded.

One step = one pass of the hot path over that batch:
  maps   a1-a3+a7: expansion, halo sums, epilogue and A3 fields on the 2048^2 grid (MIXED)
  chi2   a1+a4:    source-plane chi^2 for 1024 samples x 150 images (MIXED)
  find   a5:       image finder for 60 sources on the 2048^2 grid (MIXED + FP64 containment)
The headline value is halo x point lens evaluations per second over the whole step.

Prints one JSON line (see the repository's design notes for the accounting).
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

PEAK_FP32_VECTOR = 157.3e12    # MI355X published FP32 vector peak [FLOP/s]
# algorithmic FLOPs of one circular dPIE member at one point, alpha + Hessian (closed form
# of the oracle, transcendental = 1): see the design notes
F_CPJE = 39


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (see the design notes "
              "for how the work would shard).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2609_08649_amd import lensfield as lf
    from paper_2609_08649_amd import workloads as W

    dev = torch.device("cuda", 0)
    cfg = W.config2()
    model = cfg["model"]
    grid = cfg["grid"]
    ctx = lf.Context(0)
    m = ctx.upload_model(model)
    H = m.n_halos
    P = grid["nx"] * grid["ny"]
    params = torch.as_tensor(cfg["params"], device=dev)
    truth = params[:1].contiguous()
    a_maps = ctx.adis(model["z_d"], 2.0)
    out_names = ("alpha_x", "alpha_y", "psi11", "psi12", "psi22", "kappa", "gamma1", "gamma2", "detA", "mu",
                 "beta_x", "beta_y")
    bufs = {k: torch.empty((1, P), dtype=torch.float64, device=dev) for k in out_names}
    bufs["flags"] = torch.empty((1, P), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        ctx.lens_maps(m, truth, 1, grid, a_maps, lf.LF_PREC_MIXED, outputs=out_names, out=bufs, stream=stream)

    evals_per_step = H * P
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    L = lf.lib()
    L.lf_profile_reset(ctx.handle)
    L.lf_profile_enable(ctx.handle, 1)
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.lf_profile_enable(ctx.handle, 0)
    import ctypes as C
    tot, cnt = C.c_double(), C.c_int64()
    L.lf_profile_read(ctx.handle, b"maps_lean", C.byref(tot), C.byref(cnt))
    lean_ms = tot.value / max(1, cnt.value)
    ms = (t1 - t0) * 1e3 / args.steps
    n_mem = len(model["members"]["x"])
    flops_lean = n_mem * P * F_CPJE
    achieved = flops_lean / (lean_ms * 1e-3)

    # plain FP64 path of the same maps, for the precision comparison
    def step64():
        ctx.lens_maps(m, truth, 1, grid, a_maps, lf.LF_PREC_FP64, outputs=out_names, out=bufs, stream=stream)
    step64()
    torch.cuda.synchronize()
    t = time.perf_counter()
    n64 = max(1, args.steps // 2)
    for _ in range(n64):
        step64()
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t) * 1e3 / n64

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(model, cfg, grid, args.cpu_seconds)

    res = {
        "metric": "halo x point lens evals/s (alpha+Jacobian)",
        "value": evals_per_step / (ms * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "cluster single plane: 2 elliptical dPIE + 300 circular dPIE members, "
                               "2048^2 grid over 200\", maps step", "halos": H, "points": P,
                   "precision": "mixed (FP32 member terms, FP64 accumulation and epilogue)"},
        "fp64_path_evals_per_s": evals_per_step / (ms64 * 1e-3),
        "roofline": {"bound": "alu", "kernel": "maps_lean", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
                     "avg_launch_ms": lean_ms, "flops_per_launch": flops_lean},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    m.release()
    ctx.close()


def cpu_baseline(model, cfg, grid, seconds):
    """The FP64 oracle (as it stands) on a bounded sample of the same maps workload."""
    from oracle import oracle as orc
    from paper_2609_08649_amd import workloads as W
    tab = orc.expand(model, cfg["params"][0])
    x, y = W.grid_points(grid)
    rng = np.random.default_rng(0)
    nth = orc.nthreads_default()
    n = 2000
    t = 0.0
    while True:
        idx = rng.choice(x.size, n, replace=False)
        t0 = time.perf_counter()
        orc.maps(tab, x[idx], y[idx], 0.6, nthreads=nth)
        t = time.perf_counter() - t0
        if t > seconds / 4 or n >= 200000:
            break
        n = int(n * min(8.0, max(2.0, seconds / 4 / max(t, 1e-3))))
    evals = n * tab.shape[0]
    return {"value": evals / t, "unit": "evals/s", "cores": nth, "kind": "oracle",
            "sample": "%d random grid points x %d halos of the 2048^2 maps workload (alpha, Hessian, third "
                      "derivatives by AD), %.1f s" % (n, tab.shape[0], t)}


if __name__ == "__main__":
    main()
