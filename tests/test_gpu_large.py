"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration bench.py times: the whole point set goes through the GPU, the
oracle checks a seeded subsample (synthesis) or the adjoint of a map that is
non-zero only on a seeded subsample (every coefficient compared)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _run(w, n_synth, n_adj):
    say("workload %s: %d points, lmax %d, spin %d, eps %g, %s" % (w.name, w.npoints, w.lmax, w.spin, w.epsilon,
                                                                    w.precision))
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    say("  plan: Lmax %d mmax %d W %d grid %dx%d" % (plan.info["Lmax"], plan.info["mmax"], plan.info["nufft_w"],
                                                     plan.info["rows_used"], plan.info["nphi_grid"]))
    a = w.alm()
    f = plan.synth(torch.as_tensor(a, device="cuda")).cpu().numpy().astype(np.complex128)
    idx = w.subsample(n_synth)
    ref = oracle.synth(a, w.theta[idx], w.phi[idx], w.lmax, w.spin)
    err = float(np.linalg.norm(f[idx] - ref) / np.linalg.norm(ref))
    say("  synth rel L2 on %d points: %.3e" % (idx.shape[0], err))
    assert err <= 10 * w.epsilon

    idx = w.subsample(n_adj)
    g = np.zeros(w.npoints, dtype=np.complex128)
    g[idx] = syn.gaussian_map(idx.shape[0], 9100)
    gt = torch.as_tensor(g.astype(np.complex64 if plan.info["map_is_fp32"] else np.complex128), device="cuda")
    at = plan.adjoint(gt).cpu().numpy()
    aref = oracle.adjoint(gt.cpu().numpy().astype(np.complex128)[idx], w.theta[idx], w.phi[idx], w.lmax, w.spin)
    d = at - aref
    aerr = math.sqrt(oracle.alm_dot(d, d, w.lmax) / oracle.alm_dot(aref, aref, w.lmax))
    say("  adjoint rel L2 from %d points: %.3e" % (idx.shape[0], aerr))
    assert aerr <= 10 * w.epsilon

    # dot-product test on the full point set
    h = torch.as_tensor(w.adjoint_map(np.complex64 if plan.info["map_is_fp32"] else np.complex128), device="cuda")
    ah = plan.adjoint(h).cpu().numpy()
    lhs = oracle.map_dot(f, h.cpu().numpy().astype(np.complex128))
    rhs = oracle.alm_dot(a, ah, w.lmax)
    dot = abs(lhs - rhs) / (np.linalg.norm(f) * np.linalg.norm(h.cpu().numpy()))
    say("  dot-product relative mismatch: %.3e" % dot)
    assert dot <= (1e-5 if plan.info["map_is_fp32"] else 1e-11)
    plan.close()


def test_spt_like_lmax2048_fp64():
    _run(syn.spt_like(2048), 400, 120)


def test_spt_fine_lmax4096_fp32():
    _run(syn.spt_fine("fp32"), 150, 60)


def test_spt_fine_lmax4096_fp64():
    _run(syn.spt_fine("fp64"), 150, 60)


def test_shuffled_order_matches_raster():
    """Raster and shuffled point order give the same map per point."""
    w = syn.spt_like(2048)
    ws = w.shuffled()
    perm = syn.rng(syn.SEED_POINTS + 100 + w.seed_base).permutation(w.npoints)
    a = torch.as_tensor(w.alm(), device="cuda")
    f1 = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon).synth(a).cpu().numpy()
    f2 = Plan(ws.theta, ws.phi, ws.lmax, ws.spin, ws.epsilon).synth(a).cpu().numpy()
    assert np.max(np.abs(f1[perm] - f2)) <= 1e-12 * np.max(np.abs(f1))
