"""Autograd form: gradients of real losses through SynthFn / AdjointFn.

The loss L(a) = ||synth(a) - d||^2 is exactly quadratic in (Re, Im) of every
coefficient, so central differences carry no truncation error and must
match the analytic gradient to rounding (1e-7 relative in FP64).  The
analytic gradient is also compared with the oracle: for m >= 1 it is twice
the adjoint synthesis of dL/df, for m = 0 the adjoint itself (real).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.autograd import AdjointFn, SynthFn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _coords(lmax, spin, mmax, n, seed, stratified=False):
    """n random (component, l, m, part) coordinates with l >= spin, m <= min(l, mmax); m = 0 only real.
    stratified: coordinate i draws m from the i-th of n equal bins of [0, mmax], so the set spans every order."""
    r = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        if stratified:
            i = len(out)
            lo, hi = (i * (mmax + 1)) // n, max((i * (mmax + 1)) // n + 1, ((i + 1) * (mmax + 1)) // n)
            m = int(r.integers(lo, hi))
        else:
            m = int(r.integers(0, mmax + 1))
        l = int(r.integers(max(m, spin), lmax + 1))
        part = 0 if m == 0 else int(r.integers(0, 2))
        out.append((int(r.integers(0, 2)), l, m, part))
    return out


def _fd_check(plan, a0, d, coords, h):
    """Central differences of L(a) = sum |synth(a) - d|^2 against autograd."""
    a = a0.clone().requires_grad_(True)
    f = SynthFn.apply(a, plan)
    loss = (f - d).abs().pow(2).sum()
    loss.backward()
    g = a.grad.detach().cpu().numpy()
    lmax = plan.lmax
    an, fd = [], []
    for comp, l, m, part in coords:
        idx = m * (2 * lmax + 1 - m) // 2 + l
        step = h if part == 0 else 1j * h
        ap, am = a0.clone(), a0.clone()
        ap[comp, idx] += step
        am[comp, idx] -= step
        with torch.no_grad():
            lp = float((plan.synth(ap) - d).abs().pow(2).sum())
            lm = float((plan.synth(am) - d).abs().pow(2).sum())
        fd.append((lp - lm) / (2 * h))
        an.append(g[comp, idx].real if part == 0 else g[comp, idx].imag)
    an, fd = np.array(an), np.array(fd)
    return float(np.max(np.abs(an - fd)) / np.max(np.abs(an))), g


@pytest.mark.parametrize("spin", [0, 2])
def test_synth_gradient_small(spin):
    lmax, eps = 64, 1e-10
    th, ph = syn.uniform_cap(2000, 12.0 * math.pi / 180.0, 70 + spin)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    a0 = torch.as_tensor(syn.gaussian_alm(lmax, spin, 71), device="cuda")
    d = torch.as_tensor(syn.gaussian_map(th.shape[0], 72) * 0.1, device="cuda")
    coords = _coords(lmax, spin, plan.info["mmax"], 20, 73 + spin)
    err, g = _fd_check(plan, a0, d, coords, 0.5)
    say("spin %d: finite-difference vs autograd, max rel %.2e" % (spin, err))
    assert err <= 1e-7
    # against the oracle: dL/df = 2 (f - d); gradient = adjoint x {1 at m = 0, 2 at m >= 1}
    f = oracle.synth(a0.cpu().numpy(), th, ph, lmax, spin)
    gref = oracle.adjoint(2.0 * (f - d.cpu().numpy()), th, ph, lmax, spin)
    m, _ = syn.alm_m_l(lmax)
    gref = gref * np.where(m == 0, 1.0, 2.0)[None, :]
    dd = g - gref
    rel = math.sqrt(oracle.alm_dot(dd, dd, lmax) / oracle.alm_dot(gref, gref, lmax))
    say("spin %d: autograd gradient vs oracle rel L2 %.2e" % (spin, rel))
    assert rel <= 10 * eps
    assert np.all(g[:, m == 0].imag == 0.0)
    plan.close()


def test_adjoint_gradient_small():
    lmax, spin, eps = 48, 2, 1e-10
    th, ph = syn.uniform_cap(1500, 10.0 * math.pi / 180.0, 80)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    f0 = torch.as_tensor(syn.gaussian_map(th.shape[0], 81), device="cuda")
    b = torch.as_tensor(syn.gaussian_alm(lmax, spin, 82), device="cuda")
    f = f0.clone().requires_grad_(True)
    loss = (AdjointFn.apply(f, plan) - b).abs().pow(2).sum()
    loss.backward()
    g = f.grad.detach().cpu().numpy()
    r = np.random.default_rng(83)
    an, fd = [], []
    for _ in range(16):
        p, part, h = int(r.integers(0, th.shape[0])), int(r.integers(0, 2)), 0.5
        step = h if part == 0 else 1j * h
        fp, fm = f0.clone(), f0.clone()
        fp[p] += step
        fm[p] -= step
        with torch.no_grad():
            lp = float((plan.adjoint(fp) - b).abs().pow(2).sum())
            lm = float((plan.adjoint(fm) - b).abs().pow(2).sum())
        fd.append((lp - lm) / (2 * h))
        an.append(g[p].real if part == 0 else g[p].imag)
    an, fd = np.array(an), np.array(fd)
    err = float(np.max(np.abs(an - fd)) / np.max(np.abs(an)))
    say("adjoint: finite-difference vs autograd, max rel %.2e" % err)
    assert err <= 1e-7
    # oracle: dL/da~ = 2 (a~ - b); map gradient = synth of it with m >= 1 halved
    at = oracle.adjoint(f0.cpu().numpy(), th, ph, lmax, spin)
    ga = 2.0 * (at - b.cpu().numpy())
    m, _ = syn.alm_m_l(lmax)
    gref = oracle.synth(ga * np.where(m == 0, 1.0, 0.5)[None, :], th, ph, lmax, spin)
    rel = float(np.linalg.norm(g - gref) / np.linalg.norm(gref))
    say("adjoint: autograd gradient vs oracle rel L2 %.2e" % rel)
    assert rel <= 10 * eps
    plan.close()


def test_fp32_plan_gradient_vs_oracle():
    lmax, spin, eps = 96, 2, 1e-5
    th, ph = syn.uniform_cap(3000, 15.0 * math.pi / 180.0, 90)
    plan = Plan(th, ph, lmax, spin, eps, "fp32")
    a = torch.as_tensor(syn.gaussian_alm(lmax, spin, 91), device="cuda").requires_grad_(True)
    f = SynthFn.apply(a, plan)
    assert f.dtype == torch.complex64
    gm = syn.gaussian_map(th.shape[0], 92).astype(np.complex64)
    (f * torch.as_tensor(gm, device="cuda").conj()).real.sum().backward()
    g = a.grad.cpu().numpy()
    m, _ = syn.alm_m_l(lmax)
    gref = oracle.adjoint(gm.astype(np.complex128), th, ph, lmax, spin) * np.where(m == 0, 1.0, 2.0)[None, :]
    dd = g - gref
    rel = math.sqrt(oracle.alm_dot(dd, dd, lmax) / oracle.alm_dot(gref, gref, lmax))
    say("fp32 plan: gradient vs oracle rel L2 %.2e" % rel)
    assert rel <= 10 * eps
    plan.close()


def test_autograd_patch_lmax3000_full_size():
    """Map-fitting loss on the 999 deg^2, lmax 3000, spin-2 patch (~3.6M points):
    d = synth(second alm set) + 1% complex white noise; 20 coordinates by
    central differences."""
    w = syn.autograd_patch()
    say("autograd patch: %d points" % w.npoints)
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    a2 = torch.as_tensor(w.alm(1), device="cuda")
    d0 = plan.synth(a2)
    rms = float(d0.abs().pow(2).mean().sqrt())
    d = d0 + torch.as_tensor(syn.complex_noise(w.npoints, 0.01 * rms, syn.SEED_MAP + 50 + w.seed_base), device="cuda")
    a0 = torch.as_tensor(w.alm(0), device="cuda")
    # 20 coordinates whose orders span 0 .. mmax (one per twentieth of the range)
    coords = _coords(w.lmax, w.spin, plan.info["mmax"], 20, 95, stratified=True)
    say("autograd patch: orders checked %s (mmax %d)" % (sorted(c[2] for c in coords), plan.info["mmax"]))
    assert max(c[2] for c in coords) >= 0.9 * plan.info["mmax"]
    err, g = _fd_check(plan, a0, d, coords, 2.0)
    say("autograd patch: finite-difference vs autograd, max rel %.2e" % err)
    assert err <= 1e-7
    m, _ = syn.alm_m_l(w.lmax)
    assert np.all(g[:, m > plan.info["mmax"]] == 0)
    plan.close()
