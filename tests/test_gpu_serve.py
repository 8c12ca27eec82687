"""Serving form on the GPU, over the whole served mix: discs of 2, 5, 10 and
20 deg, lmax 512 .. 4096, spin 0 and 2, synthesis and adjoint (FP32,
eps 1e-5).  Every served result (continuous batching, overlapping slots)
equals the same request run alone within 10 eps, and for every (radius,
lmax, spin) one synthesis and one adjoint are checked against stored oracle
results (tests/golden/served_discs.npz: a 64-point synthesis subsample, and
the adjoint of a map on 64 points at 2048 seeded coefficients)."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan
from paper_2603_17166_amd.serve import (PlanKey, Server, TorchExecutor, latency_stats, poisson_arrivals,
                                        run_closed_loop, run_open_loop)

pytestmark = pytest.mark.gpu
EPS = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "served_discs.npz")


def say(*a):
    print(*a, flush=True)


def _code(radius, lmax, spin):
    return int(100 * radius) + lmax // 512 + spin


def _rel(a, b):
    a = a.cpu().numpy().astype(np.complex128)
    b = b.cpu().numpy().astype(np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _requests(patches, fx):
    """Every (radius, lmax, spin, op) once with random data, plus, per
    (radius, lmax, spin), the synthesis and the adjoint of the stored oracle
    checks; shuffled with a fixed seed.  Entries: (key, op, data, check)."""
    out = []
    for r in syn.SERVED_RADII:
        n = patches[r][0].shape[0]
        for lmax in syn.SERVED_LMAX:
            for spin in syn.SERVED_SPINS:
                key = PlanKey("disc%g" % r, lmax, spin, EPS, "fp32")
                c = _code(r, lmax, spin)
                pre = "r%g_l%d_s%d_" % (r, lmax, spin)
                out.append((key, "synth", torch.as_tensor(syn.gaussian_alm(lmax, spin, 6000 + c), device="cuda"),
                            None))
                out.append((key, "adjoint", torch.as_tensor(syn.gaussian_map(n, 6100 + c, np.complex64),
                                                             device="cuda"), None))
                out.append((key, "synth", torch.as_tensor(syn.gaussian_alm(lmax, spin, 5000 + c), device="cuda"),
                            ("synth", fx[pre + "idx"], fx[pre + "synth"])))
                g = np.zeros(n, dtype=np.complex64)
                g[fx[pre + "idx"]] = fx[pre + "adj_in"]
                out.append((key, "adjoint", torch.as_tensor(g, device="cuda"),
                            ("adjoint", fx[pre + "adj_k"], fx[pre + "adj_out"])))
    perm = syn.rng(77).permutation(len(out))
    return [out[i] for i in perm]


def _check_oracle(res, check, lmax):
    kind, sel, ref = check
    if kind == "synth":
        got = res.cpu().numpy()[sel].astype(np.complex128)
        return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    m, _ = syn.alm_m_l(lmax)
    mk = m[sel]
    got = res.cpu().numpy()[:, sel]
    w = np.where(mk == 0, 1.0, 2.0)
    g = np.where(mk == 0, got.real + 0j, got)
    r = np.where(mk == 0, ref.real + 0j, ref)
    return math.sqrt(float(np.sum(w * np.abs(g - r) ** 2)) / float(np.sum(w * np.abs(r) ** 2)))


def test_served_mix_equals_alone_and_oracle():
    fx = np.load(FIXTURE)
    patches = {r: syn.served_patch(r) for r in syn.SERVED_RADII}
    reqs_spec = _requests(patches, fx)
    say("served mix: %d requests over %d patches, %d plan kinds" % (
        len(reqs_spec), len(patches), len({k for k, _, _, _ in reqs_spec})))
    # alone: one plan per key, one request at a time, synchronised
    plans = {}
    alone = []
    for key, op, data, _ in reqs_spec:
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
    srv = Server(ex, memory_budget=64 << 30, n_slots=4, max_batch=4)
    specs = [(k, op, d) for k, op, d, _ in reqs_spec]
    offs = poisson_arrivals(len(specs), 3000.0, 5)
    reqs = run_open_loop(srv, specs, offs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    say("mix: %s, batches %d, max concurrent %d" % (st, srv.n_batches, srv.max_concurrent))
    assert all(r.error is None for r in reqs)
    assert srv.max_concurrent > 1
    assert any(r.batch_size > 1 for r in reqs)
    worst, worst_at = 0.0, None
    for r, ref in zip(reqs, alone):
        e = _rel(r.result, ref)
        if e > worst:
            worst, worst_at = e, (r.key, r.op)
    say("worst served-vs-alone rel L2 %.2e at %s" % (worst, worst_at))
    assert worst <= 10 * EPS

    checked = set()
    worst_o = 0.0
    for r, (_, _, _, check) in zip(reqs, reqs_spec):
        if check is None:
            continue
        e = _check_oracle(r.result, check, r.key.lmax)
        worst_o = max(worst_o, e)
        checked.add((r.key.patch, r.key.lmax, r.key.spin, r.op))
        assert e <= 10 * EPS, (r.key, r.op, e)
    say("served vs stored oracle: %d (radius, lmax, spin, op) checked, worst rel L2 %.2e" % (len(checked), worst_o))
    assert len(checked) == len(syn.SERVED_RADII) * len(syn.SERVED_LMAX) * len(syn.SERVED_SPINS) * 2
    srv.close()

    # the same requests once more, all queued at once, admitted cheapest plan
    # first: the order changes, the results do not
    ex2 = TorchExecutor(n_slots=4)
    for r, (th, ph) in patches.items():
        ex2.add_patch("disc%g" % r, th, ph)
    srv2 = Server(ex2, memory_budget=64 << 30, n_slots=4, max_batch=8, policy="sjf")
    reqs2, _ = run_closed_loop(srv2, specs)
    torch.cuda.synchronize()
    assert all(r.error is None for r in reqs2)
    assert len(srv2.costs) == 2 * len({k for k, _, _ in specs}) and all(c > 0 for c in srv2.costs.values())
    worst2 = max(_rel(r.result, ref) for r, ref in zip(reqs2, alone))
    say("cheapest-first served vs alone: worst rel L2 %.2e" % worst2)
    assert worst2 <= 10 * EPS
    srv2.close()
