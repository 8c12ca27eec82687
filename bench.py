#!/usr/bin/env python
"""Benchmark of the partial-sky SHT hot path on one MI355X.

A step is one synthesis followed by one adjoint synthesis (every stage of
the path: Legendre recurrence on the rings, Theta and phi FFT stages, NUFFT
interpolation / spreading) of one coefficient set / one map over the
workload's points, with inputs resident in HBM.  The metric is
synth+adjoint points/s = npoints / (time of one step).

The default workload is the spin-2, lmax 2048, FP64, epsilon 1e-10
SPT-3G-like rectangle (RA [-50, 50] x Dec [-71, -41] deg at 1 arcmin with
2.5 arcmin RMS jitter, ~5.97M points).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2603_17166_amd import synthetic as syn  # noqa: E402

WORKLOADS = {
    "spt1658-l2048-s2-fp64": lambda: syn.spt_like(2048),
    "cap10-l128-s0-fp64": lambda: syn.cap_small(),
    "spt1501-l4096-s2-fp32": lambda: syn.spt_fine("fp32"),
    "spt1501-l4096-s2-fp64": lambda: syn.spt_fine("fp64"),
    "rect999-l3000-s2-fp64": lambda: syn.autograd_patch(),
}
DEFAULT = "spt1658-l2048-s2-fp64"

PEAK_FP64_VECTOR = 78.6e12   # FLOP/s, MI355X, FMA counted as 2
PEAK_FP32_VECTOR = 157.3e12
PEAK_HBM = 8.0e12            # B/s


def leg_flops_per_triple(spin: int) -> int:
    """Algorithmic FLOPs per (ring, m, l) of the Legendre step: per recurrence
    mu_{l+1} = c mu_l - mu_{l-1} with c = (A +/- B) - A y one FMA for c and one
    for the step (4 FLOPs), one recurrence for spin 0 and two for spin > 0,
    plus four real multiply-adds (8 FLOPs) for the complex accumulation."""
    return (8 if spin else 4) + 8


def nufft_flops_per_point(W: int) -> int:
    """Algorithmic FLOPs per point of interpolation / spreading: W^2 taps of a
    real weight times a complex value (2 FMAs) plus the W row weights (2W FMAs)
    and the outer products of the two kernel vectors."""
    return 4 * W * W + 4 * W


def cpu_baseline(w, n_sample: int) -> dict:
    import oracle

    idx = w.subsample(n_sample)
    th, ph = w.theta[idx], w.phi[idx]
    a = w.alm()
    f = syn.gaussian_map(idx.shape[0], 9001)
    t0 = time.perf_counter()
    oracle.synth(a, th, ph, w.lmax, w.spin)
    t1 = time.perf_counter()
    oracle.adjoint(f, th, ph, w.lmax, w.spin)
    t2 = time.perf_counter()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": idx.shape[0] / (t2 - t0), "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded points of the workload, one synthesis + one adjoint, direct sum in long double "
                      "(synth %.1f s, adjoint %.1f s)" % (idx.shape[0], t1 - t0, t2 - t1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-points", type=int, default=64, help="oracle check of the synthesized map")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        return 2

    import torch

    import oracle
    from paper_2603_17166_amd.plan import Plan

    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]()
    a_np = w.alm()
    t0 = time.perf_counter()
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info
    a = torch.as_tensor(a_np, device="cuda")
    fmap = torch.as_tensor(w.adjoint_map(np.complex64 if info["map_is_fp32"] else np.complex128), device="cuda")
    out_map = torch.empty(w.npoints, dtype=plan.map_dtype, device="cuda")
    out_alm = torch.empty_like(a)
    plan.workspace(1)

    for _ in range(args.warmup):
        plan.synth(a, out=out_map)
        plan.adjoint(fmap, out=out_alm)
    torch.cuda.synchronize()

    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.synth(a, out=out_map)
        plan.adjoint(fmap, out=out_alm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = plan.timing()
    plan.set_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = w.npoints / (ms_per_step * 1e-3)

    # accuracy of this run's synthesis on a seeded subsample
    idx = w.subsample(args.check_points)
    ref = oracle.synth(a_np, w.theta[idx], w.phi[idx], w.lmax, w.spin)
    got = out_map.cpu().numpy()[idx].astype(np.complex128)
    rel_err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    # roofline of the dominant kernel
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    dom = max(avg, key=lambda k: avg[k])
    W = info["nufft_w"]
    if dom in ("leg_synth", "leg_adj"):
        flops = info["legendre_triples"] * leg_flops_per_triple(w.spin)
        roof = {"bound": "alu", "achieved": flops / (avg[dom] * 1e-3) / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s"}
    elif dom in ("interp", "spread") and not info["map_is_fp32"]:
        flops = w.npoints * nufft_flops_per_point(W)
        roof = {"bound": "alu", "achieved": flops / (avg[dom] * 1e-3) / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s"}
    else:
        cs = 8 if info["map_is_fp32"] else 16
        grid = info["rows_used"] * info["nphi_grid"] * cs
        nbytes = grid + w.npoints * (16 + 4 + cs)
        roof = {"bound": "hbm", "achieved": nbytes / (avg[dom] * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom

    line = {
        "metric": "synth+adjoint points/s at eps=1e-10 FP64 vs eps=1e-5 FP32; p50/p99 latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if info["map_is_fp32"] else "f64",
        "data": "synthetic (seeded points and coefficients)",
        "config": {"workload": w.name, "npoints": w.npoints, "lmax": w.lmax, "spin": w.spin, "epsilon": w.epsilon,
                   "precision": w.precision, "Lmax": info["Lmax"], "mmax": info["mmax"], "nufft_w": W,
                   "grid": [info["rows_used"], info["nphi_grid"]], "legendre_triples": info["legendre_triples"]},
        "rel_err_vs_oracle": rel_err,
        "plan_s": plan_s,
        "stage_ms": {k: round(avg[k], 4) for k in avg},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
