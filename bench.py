#!/usr/bin/env python
"""Benchmark of the partial-sky SHT hot path on one MI355X.

A step is one synthesis followed by one adjoint synthesis (every stage of
the path: Legendre recurrence on the rings, Theta and phi FFT stages, NUFFT
interpolation / spreading) of one coefficient set / one map over the
workload's points, with inputs resident in HBM.  The metric is
synth+adjoint points/s = npoints / (time of one step).

The headline workload is the spin-2, lmax 4096 patch of 1501 deg^2
(RA [-48.4, 48.4] x Dec [-70, -42] deg at 0.5 arcmin with 2.5 arcmin RMS
jitter, 21.6 M points) at epsilon 1e-10 in FP64 against epsilon 1e-5 in the
FP32 form: `value` is the FP64 rate, the `fp32` object the FP32 form's, each
with its roofline, per-stage fractions and its error against stored oracle
results on a seeded 10 000-point subsample (synthesis) and on 20 480 seeded
coefficients of the adjoint of a map supported on that subsample.  Prints
one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2603_17166_amd import synthetic as syn  # noqa: E402

WORKLOADS = {
    "spt1501-l4096-s2-fp64": lambda: syn.spt_fine("fp64"),
    "spt1501-l4096-s2-fp32": lambda: syn.spt_fine("fp32"),
    "spt1658-l2048-s2-fp64": lambda: syn.spt_like(2048),
    "cap10-l128-s0-fp64": lambda: syn.cap_small(),
    "rect999-l3000-s2-fp64": lambda: syn.autograd_patch(),
}
HEADLINE = ("spt1501-l4096-s2-fp64", "spt1501-l4096-s2-fp32")
FIXTURE = os.path.join(ROOT, "tests", "golden", "spt1501_l4096_s2.npz")

PEAK_FP64_VECTOR = 78.6e12   # FLOP/s, MI355X, FMA counted as 2
PEAK_FP32_VECTOR = 157.3e12
PEAK_HBM = 8.0e12            # B/s


# ----------------------------------------------------------- algorithmic work

def leg_flops_per_triple(spin: int) -> int:
    """Algorithmic FLOPs per (ring, m, l) triple of the Legendre step, the
    per-unit figure of the measurement plan (about 13 for spin 0, 18 for
    spin > 0: one or two three-term recurrences plus the complex
    accumulation)."""
    return 18 if spin else 13


def nufft_flops_per_point(W: int) -> int:
    """Algorithmic FLOPs per point of interpolation / spreading with a W x W
    kernel support: 8 W^2 + 16 W (the measurement plan's per-point figure)."""
    return 8 * W * W + 16 * W


def stage_work(w, info) -> dict:
    """Per stage: (bound, algorithmic amount per launch, peak) -- FLOP against
    the FP64 vector peak for the Legendre stages and the FP64 NUFFT, bytes
    against HBM for the FFT stages, the FP32 NUFFT and the fills (every array
    written once and read once: F, V, U, the points' coordinates and values,
    the coefficients of m <= mmax)."""
    fp32 = bool(info["map_is_fp32"])
    cs = 8 if fp32 else 16
    ncol = 2 * info["mmax"] + 1
    nring = info["Lmax"] + 1
    rows, nphi = info["rows_used"], info["nphi_grid"]
    F = ncol * nring * 16
    V = rows * ncol * cs
    U = rows * nphi * cs
    n = w.npoints
    lmax = w.lmax
    alm_all = 2 * 16 * (lmax + 1) * (lmax + 2) // 2
    leg = ("alu", info["legendre_triples"] * leg_flops_per_triple(w.spin), PEAK_FP64_VECTOR)
    if fp32:
        nu_i = ("hbm", U + n * (16 + cs), PEAK_HBM)
        nu_s = nu_i
    else:
        nu_i = ("alu", n * nufft_flops_per_point(info["nufft_w"]), PEAK_FP64_VECTOR)
        nu_s = nu_i
    return {
        "leg_synth": leg,
        "theta_synth": ("hbm", F + V, PEAK_HBM),
        "phi_synth": ("hbm", V + U, PEAK_HBM),
        "interp": nu_i,
        "grid_zero": ("hbm", U, PEAK_HBM),
        "spread": nu_s,
        "phi_adj": ("hbm", U + V, PEAK_HBM),
        "theta_adj": ("hbm", V + F, PEAK_HBM),
        "alm_zero": ("hbm", alm_all, PEAK_HBM),
        "leg_adj": leg,
    }


STAGE_KERNEL = {"leg_synth": ("psht::k_leg_synth<", "psht::k_leg_synth_seg<"),
                "leg_adj": ("psht::k_leg_adj_seg6<", "psht::k_leg_adj_seg4<"),
                "theta_synth": ("psht::k_theta_synth<",), "theta_adj": ("psht::k_theta_adjoint<",),
                "phi_synth": ("psht::k_phi_synth<",), "phi_adj": ("psht::k_phi_adjoint<",),
                "interp": ("psht::k_interp<",), "spread": ("psht::k_spread<",)}


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
        if not name.startswith(STAGE_KERNEL[stage]):
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


def stage_fractions(w, info, avg: dict, step_ms: float) -> dict:
    """Roofline fraction of every stage and of the whole step: a stage's
    roofline time is its algorithmic work at peak; the end-to-end fraction is
    the sum of the stages' roofline times over the measured step time."""
    work = stage_work(w, info)
    out, roof_ms = {}, 0.0
    for k, t in avg.items():
        if t <= 0 or k not in work:
            continue
        bound, amount, peak = work[k]
        ideal = amount / peak * 1e3
        roof_ms += ideal
        out[k] = {"ms": round(t, 4), "bound": bound, "roofline_ms": round(ideal, 4), "frac": round(ideal / t, 3)}
    return {"stages": out, "roofline_ms": roof_ms, "end_to_end_frac": roof_ms / step_ms}


def roofline(w, info, avg: dict) -> dict:
    """Roofline of the dominant kernel from live HIP-event timings."""
    dom = max(avg, key=lambda k: avg[k])
    bound, amount, peak = stage_work(w, info)[dom]
    if bound == "alu":
        per = leg_flops_per_triple(w.spin) if dom.startswith("leg") else nufft_flops_per_point(info["nufft_w"])
        unit_name = "(ring, m, l) triple" if dom.startswith("leg") else "point"
        roof = {"bound": "alu", "achieved": amount / (avg[dom] * 1e-3) / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "work": "%.4g FLOP per launch (%d per %s)" % (amount, per, unit_name)}
    else:
        roof = {"bound": "hbm", "achieved": amount / (avg[dom] * 1e-3) / 1e9, "peak": peak / 1e9, "unit": "GB/s",
                "work": "%.4g B per launch" % amount}
    roof["frac"] = roof["achieved"] / roof["peak"]
    t = measured_traffic(dom, w.name)
    roof["traffic"] = t["bytes"] if t else None
    if t:
        roof["traffic_detail"] = "HBM bytes per launch of %s: read %.4g, write %.4g (rocprofv3 FETCH_SIZE x2.0, " \
                                 "WRITE_SIZE x1.0 by a 1 GiB copy)" % (t["kernel"], t["read_bytes"], t["write_bytes"])
    roof["kernel"] = dom
    roof["launch_ms"] = avg[dom]
    return roof


# ----------------------------------------------------------------- timing

def time_steps(plan, a, fmap, out_map, out_alm, steps: int, which: str, per_step: list | None = None) -> float:
    """Seconds for `steps` calls of synth, adjoint or both, bracketed by device
    synchronisation; with `per_step`, HIP events on the launch stream around
    every step append each step's milliseconds."""
    import torch

    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        if per_step is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record()
        if which in ("synth", "both"):
            plan.synth(a, out=out_map)
        if which in ("adjoint", "both"):
            plan.adjoint(fmap, out=out_alm)
        if per_step is not None:
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record()
            ev.append((e0, e1))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    if per_step is not None:
        per_step.extend(e0.elapsed_time(e1) for e0, e1 in ev)
    return t


def run_transform(w, steps: int, warmup: int, log) -> dict:
    """Plan, warm up, per-stage HIP-event breakdown (untimed steps), timed
    synth+adjoint steps (events around the dominant kernel and around every
    step), synth-only and adjoint-only loops."""
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
    plan.set_timing(True)
    time_steps(plan, a, fmap, out_map, out_alm, min(steps, 5), "both")
    avg = stage_avgs(plan.timing())
    dom = max(avg, key=lambda k: avg[k])
    plan.set_timing(True, stages=(dom,))
    per_step: list = []
    t_both = time_steps(plan, a, fmap, out_map, out_alm, steps, "both", per_step)
    avg[dom] = stage_avgs(plan.timing())[dom]
    plan.set_timing(False)
    t_syn = time_steps(plan, a, fmap, out_map, out_alm, steps, "synth")
    t_adj = time_steps(plan, a, fmap, out_map, out_alm, steps, "adjoint")
    res = {"plan": plan, "info": info, "plan_s": plan_s, "ms_per_step": t_both * 1e3 / steps, "avg": avg,
           "synth_ms": t_syn * 1e3 / steps, "adjoint_ms": t_adj * 1e3 / steps,
           "step_ms_median": float(np.median(per_step)), "step_ms_p90": float(np.percentile(per_step, 90)),
           "a_np": a_np, "out_map": out_map}
    log("%s: %.3f ms/step (median %.3f, p90 %.3f; synth %.3f, adjoint %.3f)" % (
        w.name, res["ms_per_step"], res["step_ms_median"], res["step_ms_p90"], res["synth_ms"], res["adjoint_ms"]))
    return res


def fixture_errors(w, plan, out_map) -> dict:
    """Errors against the stored oracle results of the lmax 4096 patch: the
    synthesis on the 10 000-point subsample, and the adjoint of a map that is
    non-zero only there, on the stored coefficients (the coefficient inner
    product's weights: m = 0 real parts once, m > 0 twice)."""
    import torch

    if not os.path.exists(FIXTURE):
        return {"error": "fixture missing"}
    fx = np.load(FIXTURE)
    idx = fx["idx"]
    if not np.array_equal(idx, w.subsample(idx.shape[0])):
        return {"error": "subsample differs from the fixture's"}
    got = out_map.cpu().numpy()[idx].astype(np.complex128)
    ref = fx["synth"]
    synth_err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    g = torch.zeros(w.npoints, dtype=plan.map_dtype, device="cuda")
    g[torch.as_tensor(idx, device="cuda")] = torch.as_tensor(fx["adj_in"].astype(
        np.complex64 if plan.info["map_is_fp32"] else np.complex128), device="cuda")
    at = plan.adjoint(g).cpu().numpy()
    k = fx["adj_k"]
    m, _ = syn.alm_m_l(w.lmax)
    mk = m[k]
    wgt = np.where(mk == 0, 1.0, 2.0)
    got_a = at[:, k]
    ref_a = fx["adj_out"]
    got_a = np.where(mk == 0, got_a.real + 0j, got_a)
    ref_a = np.where(mk == 0, ref_a.real + 0j, ref_a)
    num = float(np.sum(wgt * np.abs(got_a - ref_a) ** 2))
    den = float(np.sum(wgt * np.abs(ref_a) ** 2))
    return {"synth_rel_l2": synth_err, "synth_points": int(idx.shape[0]), "adjoint_rel_l2": math.sqrt(num / den),
            "adjoint_from_points": int(idx.shape[0]), "adjoint_coefficients": int(k.shape[0]),
            "bar": 10 * w.epsilon}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, n_all: int, n_one: int, log) -> dict:
    """The oracle (direct sums in long double) on the host: a seeded sample of
    the workload's points with every host core, and a smaller one on one core."""
    import oracle

    idx = w.subsample(max(n_all, n_one))
    a = w.alm()
    res = {}
    for label, n, threads in (("every", n_all, 0), ("one", n_one, 1)):
        sub = idx[:n]
        th, ph = w.theta[sub], w.phi[sub]
        f = syn.gaussian_map(sub.shape[0], 9001)
        t0 = time.perf_counter()
        oracle.synth(a, th, ph, w.lmax, w.spin, nthreads=threads)
        t1 = time.perf_counter()
        oracle.adjoint(f, th, ph, w.lmax, w.spin, nthreads=threads)
        t2 = time.perf_counter()
        res[label] = (sub.shape[0], t1 - t0, t2 - t1)
        log("cpu baseline (%s core): %d points, synth %.1f s, adjoint %.1f s" % (label, sub.shape[0], t1 - t0, t2 - t1))
    n, ts, ta = res["every"]
    n1, ts1, ta1 = res["one"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n / (ts + ta), "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded points of the workload (lmax %d, spin %d), one synthesis + one adjoint, direct sums "
                      "in long double on every host core (synth %.1f s, adjoint %.1f s)" % (n, w.lmax, w.spin, ts, ta),
            "cpu_model": cpu_model(), "value_1core": n1 / (ts1 + ta1),
            "sample_1core": "%d points on one core (synth %.1f s, adjoint %.1f s)" % (n1, ts1, ta1)}


# ----------------------------------------------------------------- extras

def small_line(w, steps: int, warmup: int, log) -> dict:
    r = run_transform(w, steps, warmup, log)
    out = {"workload": w.name, "npoints": w.npoints, "points_per_s": w.npoints / (r["ms_per_step"] * 1e-3),
           "ms_per_step": r["ms_per_step"], "step_ms_median": r["step_ms_median"], "step_ms_p90": r["step_ms_p90"],
           "synth_ms": r["synth_ms"], "adjoint_ms": r["adjoint_ms"], "plan_s": r["plan_s"],
           "roofline": roofline(w, r["info"], r["avg"]),
           "adjoint_segment": r["info"]["adj_segment"], "adjoint_waves": r["info"]["adj_waves"],
           "adjoint_rings_per_lane": r["info"]["adj_rings_per_lane"], "synth_segment": r["info"]["syn_segment"]}
    out.update(stage_fractions(w, r["info"], r["avg"], r["step_ms_median"]))
    r["plan"].close()
    return out


def autograd_step(steps: int, log) -> dict:
    """One optimisation step of loss = ||synth(alm) - d||^2 on the 999 deg^2,
    lmax 3000, spin-2 patch (FP64): forward synthesis, backward through the
    adjoint kernel; d = synthesis of a second coefficient set + 1 % noise."""
    import torch

    from paper_2603_17166_amd.autograd import SynthFn
    from paper_2603_17166_amd.plan import Plan

    w = syn.autograd_patch()
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    d0 = plan.synth(torch.as_tensor(w.alm(1), device="cuda"))
    rms = float(d0.abs().pow(2).mean().sqrt())
    d = d0 + torch.as_tensor(syn.complex_noise(w.npoints, 0.01 * rms, syn.SEED_MAP + 50 + w.seed_base), device="cuda")
    a = torch.as_tensor(w.alm(0), device="cuda").requires_grad_(True)

    def one():
        a.grad = None
        loss = (SynthFn.apply(a, plan) - d).abs().pow(2).sum()
        loss.backward()
        return loss

    for _ in range(2):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.close()
    log("autograd step (%s): %.3f ms" % (w.name, ms))
    return {"workload": w.name, "npoints": w.npoints, "ms_per_step": ms, "points_per_s": w.npoints / (ms * 1e-3),
            "note": "forward synthesis + loss + backward (adjoint kernel) per step"}


def full_sky_speedup(workloads, steps: int, log) -> dict:
    """The partial-sky method against the full-sky mode (rings over the whole
    sphere, Lmax = lmax) on the same points, coefficients and accuracy: one
    synthesis + one adjoint each, and the speed-up beside the plan's predicted
    one, 1 / ((1 + eps_apo)(1 - cos theta_max)), the estimate of Table I's
    'predicted' column."""
    import torch

    from paper_2603_17166_amd.plan import Plan

    out = {}
    for w in workloads:
        a = torch.as_tensor(w.alm(), device="cuda")
        res = {}
        for mode in ("partial", "full_sky"):
            plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision, full_sky=(mode == "full_sky"))
            fmap = torch.as_tensor(w.adjoint_map(np.complex64 if plan.info["map_is_fp32"] else np.complex128),
                                   device="cuda")
            om = torch.empty(w.npoints, dtype=plan.map_dtype, device="cuda")
            oa = torch.empty_like(a)
            plan.workspace(1)
            time_steps(plan, a, fmap, om, oa, 1, "both")
            t = time_steps(plan, a, fmap, om, oa, steps, "both")
            res[mode] = {"ms_per_step": t * 1e3 / steps, "Lmax": plan.info["Lmax"],
                         "legendre_triples": plan.info["legendre_triples"],
                         "predicted_speedup": plan.info["predicted_speedup"]}
            plan.close()
        sp = res["full_sky"]["ms_per_step"] / res["partial"]["ms_per_step"]
        out[w.name] = {"partial_ms": res["partial"]["ms_per_step"], "full_sky_ms": res["full_sky"]["ms_per_step"],
                       "speedup": sp, "predicted_speedup": res["partial"]["predicted_speedup"],
                       "Lmax": [res["partial"]["Lmax"], res["full_sky"]["Lmax"]],
                       "legendre_triples_ratio": res["full_sky"]["legendre_triples"] /
                       res["partial"]["legendre_triples"]}
        log("full sky vs partial %s: %.3f vs %.3f ms, speed-up %.2f (predicted %.2f)" % (
            w.name, res["full_sky"]["ms_per_step"], res["partial"]["ms_per_step"], sp,
            res["partial"]["predicted_speedup"]))
    return out


def rotation_triples(lmax: int) -> int:
    """(l, m, m') with 0 <= m <= l, |m'| <= l, l <= lmax: the recurrence steps of the rotation."""
    m = np.arange(lmax + 1)[:, None]
    mp = np.abs(np.arange(-lmax, lmax + 1))[None, :]
    return int(np.sum(lmax + 1 - np.maximum(m, mp)))


def patch_frame(lmax: int, npoints: int, steps: int, log) -> dict:
    """Rotation into the patch frame (Sec. II, step 1) at the largest workload's
    size: coefficients of both components at lmax 4096 (FP64 ALU bound:
    16 FLOP per (l, m, m') step, 8 for the d recurrence and 4 per component
    for the accumulation) and the points with their spin angle (HBM bound:
    16 bytes read and 24 written per point)."""
    import torch

    from paper_2603_17166_amd import rotate as rot

    ang = rot.patch_angles(147.0 * math.pi / 180, 0.3, 0.25)
    a = torch.as_tensor(syn.gaussian_alm(lmax, 2, 4242), device="cuda")
    rot.rotate_alm(a, lmax, *ang)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        out = rot.rotate_alm(a, lmax, *ang)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    tri = rotation_triples(lmax)
    tflops = 16.0 * tri / (ms * 1e-3) / 1e12
    del out
    th = torch.rand(npoints, dtype=torch.float64, device="cuda") * 0.3
    ph = torch.rand(npoints, dtype=torch.float64, device="cuda") * 6.28
    rot.rotate_points(th, ph, *ang)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        rot.rotate_points(th, ph, *ang)
    ev[1].record()
    torch.cuda.synchronize()
    pms = ev[0].elapsed_time(ev[1]) / steps
    gbs = 40.0 * npoints / (pms * 1e-3) / 1e9
    log("patch frame: rotate_alm lmax %d x2: %.2f ms (%.1f TFLOP/s FP64); points %d: %.3f ms (%.0f GB/s)" % (
        lmax, ms, tflops, npoints, pms, gbs))
    return {"rotate_alm": {"lmax": lmax, "components": 2, "ms": ms, "triples": tri,
                           "roofline": {"bound": "alu", "achieved": tflops, "peak": 78.6, "unit": "TFLOP/s",
                                        "frac": tflops / 78.6, "flop_per_triple": 16}},
            "rotate_points": {"npoints": npoints, "ms": pms,
                              "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                           "frac": gbs / 8000.0, "bytes_per_point": 40}}}


def plan_rules(w, steps: int, log) -> dict:
    """Lmax rules on one workload: eq. Lmax2, the least-work rule, and Lmax
    tuned to the spectrum of the seeded coefficients (C_l = (l+1)^-2, Sec.
    II.D); one synthesis + one adjoint each, the synthesis' difference from
    the eq. Lmax2 plan (both within epsilon of the exact map)."""
    import torch

    from paper_2603_17166_amd.plan import Plan

    a = torch.as_tensor(w.alm(), device="cuda")
    l = np.arange(w.lmax + 1)
    out, ref = {}, None
    for name, kw in (("band", {}), ("cost", {"lmax_rule": "cost"}), ("tuned", {"cl": 1.0 / (1.0 + l) ** 2})):
        t0 = time.time()
        plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision, **kw)
        plan_s = time.time() - t0
        fmap = torch.as_tensor(w.adjoint_map(np.complex64 if plan.info["map_is_fp32"] else np.complex128),
                               device="cuda")
        om = torch.empty(w.npoints, dtype=plan.map_dtype, device="cuda")
        oa = torch.empty_like(a)
        plan.workspace(1)
        time_steps(plan, a, fmap, om, oa, 1, "both")
        t = time_steps(plan, a, fmap, om, oa, steps, "both")
        f = plan.synth(a)
        torch.cuda.synchronize()
        if ref is None:
            ref = f.clone()
        err = float(torch.linalg.vector_norm(f - ref) / torch.linalg.vector_norm(ref))
        out[name] = {"ms_per_step": t * 1e3 / steps, "Lmax": plan.info["Lmax"], "eps_apo": plan.info["eps_apo"],
                     "legendre_triples": plan.info["legendre_triples"], "plan_s": plan_s,
                     "predicted_error": plan.info["predicted_error"], "synth_rel_diff_vs_band": err}
        log("Lmax rule %s: Lmax %d, %.3f ms per synth+adjoint, diff vs band %.1e" % (
            name, plan.info["Lmax"], t * 1e3 / steps, err))
        plan.close()
    return out


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
    res = {"workload": w.name, "nmaps": nmaps, "ms_per_step": ms, "points_per_s": nmaps * w.npoints / (ms * 1e-3),
           "leg_synth_ms_per_map": avg["leg_synth"] / nmaps, "rel_err_vs_oracle_last_map": err,
           "stage_ms_per_launch": {k: round(v, 4) for k, v in avg.items()}}
    log("batched %d maps: %.3f ms per step (synth + adjoint of all maps), rel err %.2e" % (nmaps, ms, err))
    return res


def serial_gpu_time(srv, mix, log, reps: int = 5) -> dict:
    """GPU time of the mix's requests, each kind run alone: `reps` launches
    back to back on one stream of the server's resident plans, HIP events
    around them.  The mix-weighted mean is the GPU work per request; its
    inverse bounds the request rate of one GPU without overlap."""
    import torch

    stream = torch.cuda.Stream()
    per_kind, count = {}, {}
    for key, op, data in mix:
        count[(key, op)] = count.get((key, op), 0) + 1
        if (key, op) in per_kind or key not in srv.plans:
            continue
        plan = srv.plans[key].handle
        x = data.unsqueeze(0)
        ws = torch.empty(max(1, plan.info["workspace_bytes_per_map"]), dtype=torch.uint8, device="cuda")
        fn = plan.synth if op == "synth" else plan.adjoint
        with torch.cuda.stream(stream):
            fn(x, stream=stream, workspace=ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn(x, stream=stream, workspace=ws)
            e1.record(stream)
        e1.synchronize()
        per_kind[(key, op)] = e0.elapsed_time(e1) / reps
    n = sum(c for k, c in count.items() if k in per_kind)
    mean_ms = sum(per_kind[k] * c for k, c in count.items() if k in per_kind) / max(n, 1)
    log("served: %.3f ms of GPU time per request (kinds alone), %.0f requests/s without overlap" %
        (mean_ms, 1e3 / mean_ms))
    return {"serial_gpu_ms_per_request": mean_ms, "gpu_bound_requests_per_s": 1e3 / mean_ms}


def served(n_requests: int, load: float, log, single_fp64: int = 0, max_batch: int = 8,
           policy: str = "sjf") -> dict:
    """Served mix: discs of 2/5/10/20 deg, lmax 512..4096, spin 0/2, 50/50
    synth/adjoint, FP32 eps 1e-5.  With single_fp64 > 0, the first that many
    requests of the same mix are also run one at a time (no batching, no
    overlap) on FP64 eps 1e-10 plans, the plain-FP64-single rate of the same
    requests."""
    import torch

    from paper_2603_17166_amd.plan import Plan
    from paper_2603_17166_amd.serve import (PlanKey, Server, TorchExecutor, latency_stats, percentile,
                                            poisson_arrivals, run_closed_loop, run_open_loop)

    eps = 1e-5
    ex = TorchExecutor(n_slots=4)
    npts, maps, maps64, patches = {}, {}, {}, {}
    for r in syn.SERVED_RADII:
        th, ph = syn.served_patch(r)
        patches[r] = (th, ph)
        ex.add_patch("disc%g" % r, th, ph)
        npts[r] = th.shape[0]
        m = syn.gaussian_map(th.shape[0], syn.SEED_MAP + 4 + int(r), np.complex64)
        maps[r] = torch.as_tensor(m, device="cuda")
        maps64[r] = torch.as_tensor(m.astype(np.complex128), device="cuda")
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

    srv = Server(ex, memory_budget=96 << 30, n_slots=4, max_batch=max_batch, policy=policy)
    t0 = time.perf_counter()
    combos = [(r, l, s, op, 0) for r in syn.SERVED_RADII for l in syn.SERVED_LMAX for s in syn.SERVED_SPINS
              for op in ("synth", "adjoint")]
    run_closed_loop(srv, specs_of(combos))
    torch.cuda.synchronize()
    log("served: %d plans created in %.1f s" % (srv.plans_created, time.perf_counter() - t0))
    raw_mix = syn.served_mix(n_requests, seed=syn.SEED_MAP + 4)
    mix = specs_of(raw_mix)
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
    kinds = {}
    for r in reqs:
        if r.error is None:
            kinds.setdefault("%s-l%d-%s" % (r.key.patch, r.key.lmax, r.op), []).append(r.latency * 1e3)
    st.update({"policy": policy, "max_batch": max_batch, "load": load, "arrival_rate_per_s": rate,
               "saturation_requests_per_s": sat,
               "points_per_s": pts / span, "saturation_points_per_s": pts / secs, "batches": srv.n_batches,
               "max_concurrent": srv.max_concurrent, "plans_resident": len(srv.plans),
               "resident_gb": srv.resident / 1e9, "errors": sum(1 for r in reqs if r.error),
               "latency_ms_by_kind": {k: {"p50": round(percentile(v, 50), 3), "p99": round(percentile(v, 99), 3),
                                          "n": len(v)} for k, v in sorted(kinds.items())}})
    log("served at %.1fx saturation: p50 %.2f ms, p99 %.2f ms" % (load, st["p50_ms"], st["p99_ms"]))
    st.update(serial_gpu_time(srv, mix, log))
    srv.close()
    if single_fp64 > 0:
        sub = raw_mix[:single_fp64]
        plans = {}
        for radius, lmax, spin, op, _ in sub:
            key = (radius, lmax, spin)
            if key not in plans:
                th, ph = patches[radius]
                plans[key] = Plan(th, ph, lmax, spin, 1e-10, "fp64")
                plans[key].workspace(1)
        for p in plans.values():  # warm up every plan once
            p.synth(alms[(p.lmax, p.spin)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pts64 = 0
        for radius, lmax, spin, op, _ in sub:
            p = plans[(radius, lmax, spin)]
            if op == "synth":
                p.synth(alms[(lmax, spin)])
            else:
                p.adjoint(maps64[radius])
            torch.cuda.synchronize()
            pts64 += npts[radius]
        secs64 = time.perf_counter() - t0
        for p in plans.values():
            p.close()
        st["fp64_single_same_requests"] = {"requests": len(sub), "points_per_s": pts64 / secs64,
                                           "note": "the first requests of the same mix, FP64 eps 1e-10 plans, one "
                                                   "request at a time with a device synchronisation after each"}
        st["served_vs_fp64_single"] = st["points_per_s"] / (pts64 / secs64)
        log("served vs plain FP64 single on the same requests: %.2fx" % st["served_vs_fp64_single"])
    return st


# ------------------------------------------------------------------- main

def headline(steps: int, warmup: int, log) -> tuple:
    out = {}
    for name in HEADLINE:
        w = WORKLOADS[name]()
        r = run_transform(w, steps, warmup, log)
        fx = fixture_errors(w, r["plan"], r["out_map"])
        log("%s: vs stored oracle %s" % (name, fx))
        d = {"workload": name, "epsilon": w.epsilon, "precision": w.precision,
             "value": w.npoints / (r["ms_per_step"] * 1e-3), "ms_per_step": r["ms_per_step"],
             "step_ms_median": r["step_ms_median"], "step_ms_p90": r["step_ms_p90"],
             "synth_points_per_s": w.npoints / (r["synth_ms"] * 1e-3),
             "adjoint_points_per_s": w.npoints / (r["adjoint_ms"] * 1e-3),
             "transforms_per_s": 2.0 / (r["ms_per_step"] * 1e-3), "plan_s": r["plan_s"],
             "vs_oracle": fx, "roofline": roofline(w, r["info"], r["avg"]),
             "dtype": "f32+f64" if r["info"]["map_is_fp32"] else "f64"}
        d.update(stage_fractions(w, r["info"], r["avg"], r["step_ms_median"]))
        d["info"] = r["info"]
        r["plan"].close()
        out[name] = (w, d)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None, choices=sorted(WORKLOADS),
                    help="time only this workload (one line, no extras); default: the lmax 4096 FP64/FP32 pair")
    ap.add_argument("--cpu-sample", type=int, default=192, help="oracle points on every host core")
    ap.add_argument("--cpu-sample-1core", type=int, default=12, help="oracle points on one core")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads and the served mix")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate as a fraction of saturation")
    ap.add_argument("--serve-policy", default="sjf", choices=("fifo", "sjf"),
                    help="admission order: oldest first, or cheapest plan first with an age limit")
    ap.add_argument("--serve-max-batch", type=int, default=8,
                    help="requests of one kind per launch (8: the maps of one batched Legendre pass)")
    ap.add_argument("--serve-fp64-single", type=int, default=300,
                    help="requests of the served mix also run one at a time on FP64 plans")
    ap.add_argument("--full-sky-only", action="store_true", help="only the full-sky vs partial comparison")
    ap.add_argument("--patch-frame-only", action="store_true", help="only the rotation into the patch frame")
    ap.add_argument("--served-only", action="store_true", help="only the served mix")
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
    if args.patch_frame_only:
        print(json.dumps(patch_frame(4096, 21_600_000, 3, log)), flush=True)
        return 0
    if args.served_only:
        print(json.dumps(served(args.serve_requests, args.serve_load, log, args.serve_fp64_single,
                                args.serve_max_batch, args.serve_policy)), flush=True)
        return 0
    if args.full_sky_only:
        print(json.dumps(full_sky_speedup([syn.spt_like(2048), syn.spt_fine("fp64")], 3, log)), flush=True)
        return 0
    metric = "synth+adjoint points/s at eps=1e-10 FP64 vs eps=1e-5 FP32; p50/p99 latency"
    base = {"metric": metric, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic (seeded points and coefficients)"}
    if args.workload:
        w = WORKLOADS[args.workload]()
        d = small_line(w, args.steps, args.warmup, log)
        line = dict(base, value=d["points_per_s"], ms_per_step=d["ms_per_step"],
                    dtype="f32+f64" if w.precision == "fp32" else "f64",
                    config={"workload": w.name, "npoints": w.npoints, "lmax": w.lmax, "spin": w.spin,
                            "epsilon": w.epsilon, "precision": w.precision}, roofline=d.pop("roofline"))
        line.update(d)
        print(json.dumps(line), flush=True)
        return 0

    pair = headline(args.steps, args.warmup, log)
    w64, d64 = pair[HEADLINE[0]]
    w32, d32 = pair[HEADLINE[1]]
    info = d64.pop("info")
    info32 = d32.pop("info")
    line = dict(base)
    line.update({
        "value": d64["value"], "ms_per_step": d64["ms_per_step"], "dtype": "f64",
        "config": {"workload": "spt1501-l4096-s2 (eps 1e-10 FP64 vs eps 1e-5 FP32)", "npoints": w64.npoints,
                   "lmax": w64.lmax, "spin": w64.spin, "epsilon": w64.epsilon, "precision": "fp64",
                   "Lmax": info["Lmax"], "mmax": info["mmax"], "nufft_w": info["nufft_w"],
                   "grid": [info["rows_used"], info["nphi_grid"]], "legendre_triples": info["legendre_triples"],
                   "adjoint_segment": info["adj_segment"], "adjoint_waves": info["adj_waves"],
                   "adjoint_rings_per_lane": info["adj_rings_per_lane"], "synth_segment": info["syn_segment"]},
        "step_ms_median": d64["step_ms_median"], "step_ms_p90": d64["step_ms_p90"],
        "synth_points_per_s": d64["synth_points_per_s"], "adjoint_points_per_s": d64["adjoint_points_per_s"],
        "transforms_per_s": d64["transforms_per_s"], "plan_s": d64["plan_s"], "vs_oracle": d64["vs_oracle"],
        "roofline": d64["roofline"], "stages": d64["stages"], "end_to_end_frac": d64["end_to_end_frac"],
        "fp32": dict(d32, config={"Lmax": info32["Lmax"], "mmax": info32["mmax"], "nufft_w": info32["nufft_w"],
                                  "grid": [info32["rows_used"], info32["nphi_grid"]],
                                  "legendre_triples": info32["legendre_triples"],
                                  "adjoint_segment": info32["adj_segment"], "adjoint_waves": info32["adj_waves"],
                                  "adjoint_rings_per_lane": info32["adj_rings_per_lane"],
                                  "synth_segment": info32["syn_segment"]}),
        "fp32_vs_fp64": d32["value"] / d64["value"],
    })
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w64, args.cpu_sample, args.cpu_sample_1core, log)
    if not args.no_extras:
        ex = {}
        ex["cap10-l128-s0-fp64"] = small_line(syn.cap_small(), args.steps, args.warmup, log)
        w2 = syn.spt_like(2048)
        ex["spt1658-l2048-s2-fp64"] = small_line(w2, args.steps, args.warmup, log)
        ex["rect999-l3000-s2-fp64-autograd"] = autograd_step(max(3, args.steps // 4), log)
        ex["batched_maps"] = batched_maps(w2, 8, max(3, args.steps // 4), 16, log)
        ex["batched_maps"]["speedup_per_map"] = ex["batched_maps"]["points_per_s"] / \
            ex["spt1658-l2048-s2-fp64"]["points_per_s"]
        line["other_workloads"] = ex
        line["full_sky_vs_partial"] = full_sky_speedup([w2, syn.spt_fine("fp64")], 3, log)
        line["lmax_rules"] = plan_rules(w32, 3, log)
        line["lmax_rules_disc10"] = plan_rules(syn.served_disc(10.0, 4096, 2), 5, log)
        line["patch_frame"] = patch_frame(w64.lmax, w64.npoints, 3, log)
        line["served"] = served(args.serve_requests, args.serve_load, log, args.serve_fp64_single,
                                args.serve_max_batch, args.serve_policy)
        if "served_vs_fp64_single" in line["served"]:
            line["served_vs_fp64_single"] = line["served"]["served_vs_fp64_single"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
