"""Multi-map calls.  Synthesis: the batched Legendre pass (groups of 5..8
maps through FP64 MFMA); adjoint: one Legendre pass per map behind the
shared call.  Every map of a call against the oracle (10 epsilon) and
against the one-map call, including group splits (nmaps > 8), the polar
rescaling regime, odd spins, the full-sky fallback, the FP32 form and the
gradient forms; the multi-map adjoint is also checked as the exact transpose
of the batched synthesis."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
DEG = math.pi / 180.0


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [
    # lmax, spin, cap radius (deg), npoints, eps, precision, nmaps
    (96, 2, 12.0, 2000, 1e-10, "fp64", 5),
    (128, 0, 10.0, 3000, 1e-10, "fp64", 8),
    (80, 1, 20.0, 1500, 1e-10, "fp64", 5),
    (64, 3, 30.0, 1500, 1e-12, "fp64", 9),
    (200, 2, 6.0, 3000, 1e-10, "fp64", 11),
    (256, 2, 15.0, 3000, 1e-5, "fp32", 8),
    (40, 2, 150.0, 1500, 1e-10, "fp64", 6),   # full-sky fallback
    (700, 2, 3.0, 2500, 1e-10, "fp64", 5),    # deep polar: rescaled seeds
    (64, 2, 12.0, 1500, 1e-10, "fp64", 4),    # below the batching threshold: one pass per map
]


@pytest.mark.parametrize("lmax,spin,radius,n,eps,prec,nm", CASES)
def test_batched_synth_vs_oracle_and_single(lmax, spin, radius, n, eps, prec, nm):
    say("case lmax %d spin %d cap %g n %d eps %g %s nmaps %d" % (lmax, spin, radius, n, eps, prec, nm))
    th, ph = syn.uniform_cap(n, radius * DEG, 7100 + lmax)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    alms = [syn.gaussian_alm(lmax, spin, 7200 + i) for i in range(nm)]
    a = torch.stack([torch.as_tensor(x, device="cuda") for x in alms])
    fb = plan.synth(a).cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(n, min(n, 300), replace=False))
    worst_o, worst_s = 0.0, 0.0
    for i in range(nm):
        ref = oracle.synth(alms[i], th[idx], ph[idx], lmax, spin)
        worst_o = max(worst_o, rel(fb[i][idx], ref))
        single = plan.synth(a[i]).cpu().numpy()
        worst_s = max(worst_s, rel(fb[i], single))
    say("  worst vs oracle %.2e, vs one-map path %.2e" % (worst_o, worst_s))
    assert worst_o <= 10 * eps
    assert worst_s <= (1e-6 if prec == "fp32" else 1e-12)
    plan.close()


def alm_rel(a, b, lmax):
    d = a - b
    return math.sqrt(max(oracle.alm_dot(d, d, lmax), 0.0) / oracle.alm_dot(b, b, lmax))


@pytest.mark.parametrize("lmax,spin,radius,n,eps,prec,nm", CASES)
def test_multimap_adjoint_vs_oracle_and_single(lmax, spin, radius, n, eps, prec, nm):
    say("adjoint case lmax %d spin %d cap %g n %d eps %g %s nmaps %d" % (lmax, spin, radius, n, eps, prec, nm))
    th, ph = syn.uniform_cap(n, radius * DEG, 7500 + lmax)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    fp32 = bool(plan.info["map_is_fp32"])
    maps = [syn.gaussian_map(n, 7600 + i).astype(np.complex64 if fp32 else np.complex128) for i in range(nm)]
    f = torch.stack([torch.as_tensor(x, device="cuda") for x in maps])
    ab = plan.adjoint(f).cpu().numpy()
    worst_o, worst_s = 0.0, 0.0
    for i in range(min(nm, 3)):
        ref = oracle.adjoint(maps[i].astype(np.complex128), th, ph, lmax, spin)
        worst_o = max(worst_o, alm_rel(ab[i], ref, lmax))
    for i in range(nm):
        single = plan.adjoint(f[i]).cpu().numpy()
        worst_s = max(worst_s, alm_rel(ab[i], single, lmax))
    say("  worst vs oracle %.2e, vs one-map path %.2e" % (worst_o, worst_s))
    assert worst_o <= 10 * eps
    assert worst_s <= (1e-6 if prec == "fp32" else 1e-12)
    m, l = syn.alm_m_l(lmax)
    assert np.all(ab[:, :, l < spin] == 0)
    assert np.all(ab[:, :, m == 0].imag == 0)
    plan.close()


def test_multimap_adjoint_is_transpose_of_batched_synth():
    lmax, spin, eps, nm = 128, 2, 1e-10, 6
    th, ph = syn.uniform_cap(2500, 14 * DEG, 7700)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    a = [syn.gaussian_alm(lmax, spin, 7710 + i) for i in range(nm)]
    f = [syn.gaussian_map(2500, 7720 + i) for i in range(nm)]
    sa = plan.synth(torch.stack([torch.as_tensor(x, device="cuda") for x in a])).cpu().numpy()
    at = plan.adjoint(torch.stack([torch.as_tensor(x, device="cuda") for x in f])).cpu().numpy()
    for i in range(nm):
        lhs = oracle.map_dot(sa[i], f[i])
        rhs = oracle.alm_dot(a[i], at[i], lmax)
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(sa[i]) * np.linalg.norm(f[i])


def test_multimap_adjoint_gradient_form():
    lmax, spin, eps = 96, 2, 1e-10
    th, ph = syn.uniform_cap(2000, 12 * DEG, 7800)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    f = torch.stack([torch.as_tensor(syn.gaussian_map(2000, 7810 + i), device="cuda") for i in range(5)])
    gb = plan.adjoint_grad(f).cpu().numpy()
    for i in range(5):
        assert alm_rel(gb[i], plan.adjoint_grad(f[i]).cpu().numpy(), lmax) <= 1e-12


def test_batched_gradient_form():
    lmax, spin, eps = 96, 2, 1e-10
    th, ph = syn.uniform_cap(2000, 12 * DEG, 7300)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    a = torch.stack([torch.as_tensor(syn.gaussian_alm(lmax, spin, 7310 + i), device="cuda") for i in range(6)])
    gb = plan.synth_grad(a).cpu().numpy()
    for i in range(6):
        assert rel(gb[i], plan.synth_grad(a[i]).cpu().numpy()) <= 1e-12


def test_batched_full_size_spt_like():
    """8 maps at once on the 1658 deg^2 lmax 2048 patch (~6M points), each
    checked against the oracle on a seeded subsample."""
    w = syn.spt_like(2048)
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    alms = [syn.gaussian_alm(w.lmax, w.spin, 7400 + i) for i in range(8)]
    a = torch.stack([torch.as_tensor(x, device="cuda") for x in alms])
    fb = plan.synth(a)
    idx = w.subsample(48)
    worst = 0.0
    for i in range(8):
        ref = oracle.synth(alms[i], w.theta[idx], w.phi[idx], w.lmax, w.spin)
        worst = max(worst, rel(fb[i].cpu().numpy()[idx], ref))
    say("spt-like batched 8 maps: worst rel L2 vs oracle %.2e" % worst)
    assert worst <= 10 * w.epsilon
    plan.close()
