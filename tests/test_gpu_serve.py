"""Serving form on the GPU: every result of a served mix (continuous
batching, overlapping slots) equals the same request run alone, within the
stated tolerance, and agrees with the oracle."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan
from paper_2603_17166_amd.serve import PlanKey, Server, TorchExecutor, latency_stats, poisson_arrivals, run_open_loop

pytestmark = pytest.mark.gpu
EPS = 1e-5


def say(*a):
    print(*a, flush=True)


def _mix(n):
    patches = {r: syn.served_patch(r) for r in (2.0, 5.0)}
    specs = syn.served_mix(n, seed=77, radii=(2.0, 5.0), lmaxes=(512, 1024))
    reqs = []
    for radius, lmax, spin, op, seed in specs:
        key = PlanKey("disc%g" % radius, lmax, spin, EPS, "fp32")
        if op == "synth":
            data = torch.as_tensor(syn.gaussian_alm(lmax, spin, seed), device="cuda")
        else:
            data = torch.as_tensor(syn.gaussian_map(patches[radius][0].shape[0], seed, np.complex64), device="cuda")
        reqs.append((key, op, data))
    return patches, reqs


def _rel(a, b):
    a = a.cpu().numpy().astype(np.complex128)
    b = b.cpu().numpy().astype(np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_served_mix_equals_alone():
    patches, specs = _mix(48)
    say("served mix: %d requests over %d patches" % (len(specs), len(patches)))
    # alone: one plan per key, one request at a time, synchronised
    plans = {}
    alone = []
    for key, op, data in specs:
        if key not in plans:
            th, ph = patches[float(key.patch[4:])]
            plans[key] = Plan(th, ph, key.lmax, key.spin, key.epsilon, key.precision)
        p = plans[key]
        out = p.synth(data) if op == "synth" else p.adjoint(data)
        torch.cuda.synchronize()
        alone.append(out.clone())
    for p in plans.values():
        p.close()
    say("alone done")

    ex = TorchExecutor(n_slots=4)
    for r, (th, ph) in patches.items():
        ex.add_patch("disc%g" % r, th, ph)
    srv = Server(ex, memory_budget=16 << 30, n_slots=4, max_batch=4)
    offs = poisson_arrivals(len(specs), 4000.0, 5)
    reqs = run_open_loop(srv, specs, offs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    say("mix: %s, batches %d, max concurrent %d" % (st, srv.n_batches, srv.max_concurrent))
    assert all(r.error is None for r in reqs)
    assert srv.max_concurrent > 1
    assert any(r.batch_size > 1 for r in reqs)
    worst = 0.0
    for r, ref in zip(reqs, alone):
        worst = max(worst, _rel(r.result, ref))
    say("worst served-vs-alone rel L2 %.2e" % worst)
    assert worst <= 10 * EPS

    # two of the served results against the oracle (synthesis on a subsample, adjoint in full)
    for r in reqs:
        if r.op == "synth" and r.key.lmax == 512:
            th, ph = patches[float(r.key.patch[4:])]
            idx = np.sort(np.random.default_rng(3).choice(th.shape[0], 200, replace=False))
            ref = oracle.synth(r.data.cpu().numpy(), th[idx], ph[idx], r.key.lmax, r.key.spin)
            err = float(np.linalg.norm(r.result.cpu().numpy()[idx] - ref) / np.linalg.norm(ref))
            say("served synth vs oracle rel L2 %.2e" % err)
            assert err <= 10 * EPS
            break
    srv.close()
