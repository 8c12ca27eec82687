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


STAGE_KERNEL = {"leg_synth": "psht::k_leg_synth", "leg_adj": "psht::k_leg_adjoint", "theta_synth": "psht::k_theta_synth",
                "theta_adj": "psht::k_theta_adjoint", "phi_synth": "psht::k_phi_synth", "phi_adj": "psht::k_phi_adjoint",
                "interp": "psht::k_interp", "spread": "psht::k_spread"}


def measured_traffic(stage: str, workload: str):
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counts (profiles/traffic.json), or None when there
    are none for this workload or the kernel's sources changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if stage not in STAGE_KERNEL or not os.path.exists(path):
        return None
    with open(path) as fh:
        table = json.load(fh).get(workload, {})
    for name, e in table.items():
        if not name.startswith(STAGE_KERNEL[stage] + "<"):
            continue
        h = hashlib.sha256()
        for f in e["sources"]:
            with open(os.path.join(ROOT, "paper_2603_17166_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != e["source_sha256_16"]:
            return None
        return {"bytes": e["fetch_bytes"] + e["write_bytes"], "read_bytes": e["fetch_bytes"],
                "write_bytes": e["write_bytes"], "kernel": name}
    return None


def stage_avgs(stages: dict) -> dict:
    return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}


def roofline(w, info, avg: dict) -> dict:
    """Roofline of the dominant kernel from live HIP-event timings."""
    dom = max(avg, key=lambda k: avg[k])
    W = info["nufft_w"]
    if dom in ("leg_synth", "leg_adj"):
        flops = info["legendre_triples"] * leg_flops_per_triple(w.spin)
        roof = {"bound": "alu", "achieved": flops / (avg[dom] * 1e-3) / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "work": "%.4g FLOP per launch (%d per (ring, m, l) triple)" % (
                    flops, leg_flops_per_triple(w.spin))}
    elif dom in ("interp", "spread") and not info["map_is_fp32"]:
        flops = w.npoints * nufft_flops_per_point(W)
        roof = {"bound": "alu", "achieved": flops / (avg[dom] * 1e-3) / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "work": "%.4g FLOP per launch (%d per point)" % (flops, nufft_flops_per_point(W))}
    else:
        cs = 8 if info["map_is_fp32"] else 16
        grid = info["rows_used"] * info["nphi_grid"] * cs
        nbytes = grid + w.npoints * (16 + 4 + cs)
        roof = {"bound": "hbm", "achieved": nbytes / (avg[dom] * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "work": "%.4g B per launch" % nbytes}
    roof["frac"] = roof["achieved"] / roof["peak"]
    t = measured_traffic(dom, w.name)
    roof["traffic"] = t["bytes"] if t else None
    if t:
        roof["traffic_detail"] = "HBM bytes per launch of %s: read %.4g, write %.4g (rocprofv3 FETCH_SIZE x2.0, " \
                                 "WRITE_SIZE x1.0 by a 1 GiB copy)" % (t["kernel"], t["read_bytes"], t["write_bytes"])
    roof["kernel"] = dom
    roof["launch_ms"] = avg[dom]
    return roof


def time_steps(plan, a, fmap, out_map, out_alm, steps: int, which: str) -> float:
    """Seconds for `steps` calls of synth, adjoint or both, bracketed by device synchronisation."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        if which in ("synth", "both"):
            plan.synth(a, out=out_map)
        if which in ("adjoint", "both"):
            plan.adjoint(fmap, out=out_alm)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def oracle_error(w, a_np, out_map, n: int, log=None) -> float:
    """Relative L2 error of the synthesized map on a seeded subsample of n points,
    evaluated by the oracle in chunks of 1000 points (a progress line each)."""
    import oracle

    idx = w.subsample(n)
    got = out_map.cpu().numpy()[idx].astype(np.complex128)
    ref = np.empty_like(got)
    for c in range(0, idx.shape[0], 1000):
        sl = slice(c, c + 1000)
        ref[sl] = oracle.synth(a_np, w.theta[idx[sl]], w.phi[idx[sl]], w.lmax, w.spin)
        if log and idx.shape[0] > 1000:
            log("%s: oracle check %d / %d points" % (w.name, min(c + 1000, idx.shape[0]), idx.shape[0]))
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def run_transform(w, steps: int, warmup: int, check_points: int, log) -> dict:
    """Plan, warm up, time synth+adjoint steps (with per-stage HIP events) and
    synth-only / adjoint-only loops; oracle error on a subsample."""
    import torch

    from paper_2603_17166_amd.plan import Plan

    a_np = w.alm()
    t0 = time.perf_counter()
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info
    log("plan %s: %.2f s, Lmax %d mmax %d W %d" % (w.name, plan_s, info["Lmax"], info["mmax"], info["nufft_w"]))
    a = torch.as_tensor(a_np, device="cuda")
    fmap = torch.as_tensor(w.adjoint_map(np.complex64 if info["map_is_fp32"] else np.complex128), device="cuda")
    out_map = torch.empty(w.npoints, dtype=plan.map_dtype, device="cuda")
    out_alm = torch.empty_like(a)
    plan.workspace(1)
    time_steps(plan, a, fmap, out_map, out_alm, warmup, "both")
    # per-stage breakdown (events around every stage launch), outside the timed steps
    plan.set_timing(True)
    time_steps(plan, a, fmap, out_map, out_alm, min(steps, 5), "both")
    avg = stage_avgs(plan.timing())
    # timed steps: events around the dominant kernel's launches only, for its roofline
    dom = max(avg, key=lambda k: avg[k])
    plan.set_timing(True, stages=(dom,))
    t_both = time_steps(plan, a, fmap, out_map, out_alm, steps, "both")
    avg[dom] = stage_avgs(plan.timing())[dom]
    plan.set_timing(False)
    t_syn = time_steps(plan, a, fmap, out_map, out_alm, steps, "synth")
    t_adj = time_steps(plan, a, fmap, out_map, out_alm, steps, "adjoint")
    err = oracle_error(w, a_np, out_map, check_points, log)
    res = {"plan": plan, "info": info, "plan_s": plan_s, "ms_per_step": t_both * 1e3 / steps, "avg": avg,
           "synth_ms": t_syn * 1e3 / steps, "adjoint_ms": t_adj * 1e3 / steps, "rel_err": err}
    log("%s: %.3f ms/step (synth %.3f, adjoint %.3f), rel err %.2e" % (
        w.name, res["ms_per_step"], res["synth_ms"], res["adjoint_ms"], err))
    return res


def batched_maps(w, nmaps: int, steps: int, check_points: int, log) -> dict:
    """nmaps coefficient sets / maps per call on one plan (the Legendre
    synthesis runs as one MFMA pass per group of up to 8 maps)."""
    import torch

    import oracle
    from paper_2603_17166_amd.plan import Plan

    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    alms = [w.alm()] + [syn.gaussian_alm(w.lmax, w.spin, syn.SEED_ALM + 100 + i) for i in range(nmaps - 1)]
    a = torch.stack([torch.as_tensor(x, device="cuda") for x in alms])
    f = torch.stack([torch.as_tensor(w.adjoint_map(np.complex64 if plan.info["map_is_fp32"] else np.complex128),
                                     device="cuda")] * nmaps)
    out_map = torch.empty((nmaps, w.npoints), dtype=plan.map_dtype, device="cuda")
    out_alm = torch.empty_like(a)
    plan.workspace(nmaps)
    time_steps(plan, a, f, out_map, out_alm, 1, "both")
    plan.set_timing(True)
    time_steps(plan, a, f, out_map, out_alm, 1, "both")
    avg = stage_avgs(plan.timing())
    plan.set_timing(False)
    t_both = time_steps(plan, a, f, out_map, out_alm, steps, "both")
    idx = w.subsample(check_points)
    ref = oracle.synth(alms[-1], w.theta[idx], w.phi[idx], w.lmax, w.spin)
    err = float(np.linalg.norm(out_map[-1].cpu().numpy()[idx] - ref) / np.linalg.norm(ref))
    plan.close()
    ms = t_both * 1e3 / steps
    res = {"nmaps": nmaps, "ms_per_step": ms, "points_per_s": nmaps * w.npoints / (ms * 1e-3),
           "leg_synth_ms_per_map": avg["leg_synth"] / nmaps, "rel_err_vs_oracle_last_map": err,
           "stage_ms_per_launch": {k: round(v, 4) for k, v in avg.items()}}
    log("batched %d maps: %.3f ms per step (synth + adjoint of all maps), rel err %.2e" % (nmaps, ms, err))
    return res


def precision_form(steps: int, check_points: int, log) -> dict:
    """FP32 (eps 1e-5) vs FP64 (eps 1e-10) on the 1501 deg^2, lmax 4096 patch."""
    out = {}
    for prec in ("fp32", "fp64"):
        w = syn.spt_fine(prec)
        r = run_transform(w, steps, 2, check_points, log)
        out[prec] = {"epsilon": w.epsilon, "points_per_s": w.npoints / (r["ms_per_step"] * 1e-3),
                     "ms_per_step": r["ms_per_step"], "synth_ms": r["synth_ms"], "adjoint_ms": r["adjoint_ms"],
                     "rel_err_vs_oracle": r["rel_err"], "rel_err_points": check_points, "plan_s": r["plan_s"],
                     "stage_ms": {k: round(v, 4) for k, v in r["avg"].items()}}
        r["plan"].close()
    out["workload"] = "spt1501-l4096-s2 (%d points)" % syn.spt_fine("fp32").npoints
    out["fp32_speedup"] = out["fp32"]["points_per_s"] / out["fp64"]["points_per_s"]
    return out


def served(n_requests: int, load: float, log) -> dict:
    """Served mix: discs of 2/5/10/20 deg, lmax 512..4096, spin 0/2, 50/50 synth/adjoint, FP32 eps 1e-5."""
    import torch

    from paper_2603_17166_amd.serve import (PlanKey, Server, TorchExecutor, latency_stats, poisson_arrivals,
                                            run_closed_loop, run_open_loop)

    eps = 1e-5
    ex = TorchExecutor(n_slots=4)
    npts = {}
    maps = {}
    for r in syn.SERVED_RADII:
        th, ph = syn.served_patch(r)
        ex.add_patch("disc%g" % r, th, ph)
        npts[r] = th.shape[0]
        maps[r] = torch.as_tensor(syn.gaussian_map(th.shape[0], syn.SEED_MAP + 4 + int(r), np.complex64), device="cuda")
    alms = {}
    for lmax in syn.SERVED_LMAX:
        for spin in syn.SERVED_SPINS:
            alms[(lmax, spin)] = torch.as_tensor(syn.gaussian_alm(lmax, spin, syn.SEED_ALM + 4 + lmax + spin),
                                                 device="cuda")

    def specs_of(mix):
        out = []
        for radius, lmax, spin, op, _ in mix:
            key = PlanKey("disc%g" % radius, lmax, spin, eps, "fp32")
            out.append((key, op, alms[(lmax, spin)] if op == "synth" else maps[radius]))
        return out

    srv = Server(ex, memory_budget=96 << 30, n_slots=4, max_batch=4)
    # warm-up: every combination once (creates and caches all plans)
    t0 = time.perf_counter()
    combos = [(r, l, s, op, 0) for r in syn.SERVED_RADII for l in syn.SERVED_LMAX for s in syn.SERVED_SPINS
              for op in ("synth", "adjoint")]
    run_closed_loop(srv, specs_of(combos))
    torch.cuda.synchronize()
    log("served: %d plans created in %.1f s" % (srv.plans_created, time.perf_counter() - t0))
    mix = specs_of(syn.served_mix(n_requests, seed=syn.SEED_MAP + 4))
    reqs, secs = run_closed_loop(srv, mix)
    sat = len(reqs) / secs
    log("served: saturation %.1f requests/s" % sat)
    rate = load * sat
    offs = poisson_arrivals(len(mix), rate, syn.SEED_MAP + 44)
    reqs = run_open_loop(srv, mix, offs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    pts = sum(npts[float(r.key.patch[4:])] for r in reqs)
    span = max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)
    st.update({"load": load, "arrival_rate_per_s": rate, "saturation_requests_per_s": sat,
               "points_per_s": pts / span, "saturation_points_per_s": pts / secs, "batches": srv.n_batches,
               "max_concurrent": srv.max_concurrent, "plans_resident": len(srv.plans),
               "resident_gb": srv.resident / 1e9, "errors": sum(1 for r in reqs if r.error)})
    log("served at %.1fx saturation: p50 %.2f ms, p99 %.2f ms" % (load, st["p50_ms"], st["p99_ms"]))
    srv.close()
    return st


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=1536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-points", type=int, default=64, help="oracle check of the synthesized map")
    ap.add_argument("--no-extras", action="store_true", help="skip the precision-form and served-mix runs")
    ap.add_argument("--precision-check-points", type=int, default=32,
                    help="oracle subsample of the precision form (10000 takes about 6 min per precision on 16 cores)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate as a fraction of saturation")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (use --gpus 1)", file=sys.stderr)
        return 2

    import torch

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n, "launches": 5}), flush=True)
        return 0
    w = WORKLOADS[args.workload]()
    r = run_transform(w, args.steps, args.warmup, args.check_points, log)
    info, avg = r["info"], r["avg"]
    ms_per_step = r["ms_per_step"]
    line = {
        "metric": "synth+adjoint points/s at eps=1e-10 FP64 vs eps=1e-5 FP32; p50/p99 latency",
        "value": w.npoints / (ms_per_step * 1e-3),
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
                   "precision": w.precision, "Lmax": info["Lmax"], "mmax": info["mmax"], "nufft_w": info["nufft_w"],
                   "grid": [info["rows_used"], info["nphi_grid"]], "legendre_triples": info["legendre_triples"]},
        "synth_points_per_s": w.npoints / (r["synth_ms"] * 1e-3),
        "adjoint_points_per_s": w.npoints / (r["adjoint_ms"] * 1e-3),
        "transforms_per_s": 2.0 / (ms_per_step * 1e-3),
        "rel_err_vs_oracle": r["rel_err"],
        "plan_s": r["plan_s"],
        "stage_ms": {k: round(avg[k], 4) for k in avg},
        "roofline": roofline(w, info, avg),
    }
    r["plan"].close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
        log("cpu baseline: %.1f points/s" % line["cpu_baseline"]["value"])
    if not args.no_extras:
        line["batched_maps"] = batched_maps(w, 8, max(3, args.steps // 4), 16, log)
        line["batched_maps"]["speedup_per_map"] = line["batched_maps"]["points_per_s"] / line["value"]
        line["precision_form"] = precision_form(max(3, args.steps // 4), args.precision_check_points, log)
        line["served"] = served(args.serve_requests, args.serve_load, log)
        line["served_vs_fp64_single"] = line["served"]["points_per_s"] / line["value"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
