"""Full-sky mode and long transforms on the GPU, against the oracle.

The full-sky mode evaluates the Fourier-sphere synthesis of Sec. I.B on rings
over the whole sphere (theta_max = pi, window 1, Lmax >= lmax): up to the
NUFFT error it is the textbook transform for any point set.  The long-transform
paths are the Theta grid as two N2-point transforms (even / odd rows, used when
the grid exceeds one workgroup's LDS) and phi rows in four parts (rows above
twice the LDS limit); both are also forced on small plans here.  Bar: relative
L2 <= 10 eps against the oracle."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
DEG = math.pi / 180
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.as_tensor(x).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def alm_rel(a, b, lmax):
    d = a - b
    return math.sqrt(max(oracle.alm_dot(d, d, lmax), 0.0) / oracle.alm_dot(b, b, lmax))


def _check(plan, th, ph, a, lmax, spin, eps, tag):
    fp32 = bool(plan.info["map_is_fp32"])
    f = plan.synth(dev(a)).cpu().numpy().astype(np.complex128)
    ref = oracle.synth(a, th, ph, lmax, spin)
    e1 = rel(f, ref)
    g = syn.gaussian_map(th.shape[0], 9300 + lmax).astype(np.complex64 if fp32 else np.complex128)
    at = plan.adjoint(dev(g)).cpu().numpy()
    e2 = alm_rel(at, oracle.adjoint(g.astype(np.complex128), th, ph, lmax, spin), lmax)
    say("  %s: synth %.2e adjoint %.2e (eps %g)" % (tag, e1, e2, eps))
    assert e1 <= 10 * eps and e2 <= 10 * eps
    assert plan.dropped_points() == 0
    return f, at


@pytest.mark.parametrize("spin,eps,prec", [(0, 1e-10, "fp64"), (2, 1e-10, "fp64"), (2, 1e-5, "fp32"),
                                           (1, 1e-8, "fp64")])
def test_full_sky_whole_sphere_vs_oracle(spin, eps, prec):
    """Points over the whole sphere, poles included."""
    lmax = 64
    th, ph = syn.uniform_cap(3000, math.pi, 9400 + spin)
    th = np.concatenate([th, [0.0, math.pi, math.pi / 2]])
    ph = np.concatenate([ph, [1.0, 2.0, 3.0]])
    plan = Plan(th, ph, lmax, spin, eps, prec, full_sky=True)
    info = plan.info
    say("full sky lmax %d spin %d %s: Lmax %d, theta_max %.6f, window 1" % (lmax, spin, prec, info["Lmax"],
                                                                          info["theta_max"]))
    assert info["full_sky"] == 1 and info["theta_max"] == math.pi and info["Lmax"] >= lmax
    _check(plan, th, ph, syn.gaussian_alm(lmax, spin, 9500 + spin), lmax, spin, eps, "whole sphere")
    plan.close()


def test_full_sky_and_partial_agree_on_a_cap():
    """On a cap both modes give the transform: each against the oracle, and
    the full-sky mode runs more rings (its Lmax is lmax, the partial one's is
    about lmax theta_max / pi)."""
    lmax, spin, eps = 200, 2, 1e-10
    th, ph = syn.uniform_cap(4000, 15 * DEG, 9600)
    a = syn.gaussian_alm(lmax, spin, 9601)
    pf = Plan(th, ph, lmax, spin, eps, "fp64", full_sky=True)
    pp = Plan(th, ph, lmax, spin, eps, "fp64")
    assert pf.info["Lmax"] >= lmax > 2 * pp.info["Lmax"]
    ff, af = _check(pf, th, ph, a, lmax, spin, eps, "full sky")
    fp_, ap = _check(pp, th, ph, a, lmax, spin, eps, "partial")
    assert rel(ff, fp_) <= 20 * eps
    pf.close()
    pp.close()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_theta_grid_as_two_transforms(prec, eps, monkeypatch):
    """The Theta grid as two N2-point transforms (even and odd rows), forced
    on a small plan."""
    monkeypatch.setenv("PSHT_THETA_SPLIT", "1")
    lmax, spin = 160, 2
    th, ph = syn.uniform_cap(5000, 25 * DEG, 9700)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    _check(plan, th, ph, syn.gaussian_alm(lmax, spin, 9701), lmax, spin, eps, "theta split " + prec)
    plan.close()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_phi_rows_in_four_parts(prec, eps, monkeypatch):
    """phi rows as four transforms of Nphi / 4 points (orders folded onto
    their entries in the synthesis), forced on a small plan."""
    monkeypatch.setenv("PSHT_PHI_PARTS", "4")
    lmax, spin = 160, 2
    th, ph = syn.uniform_cap(5000, 25 * DEG, 9800)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    assert plan.info["nphi_grid"] % 4 == 0
    _check(plan, th, ph, syn.gaussian_alm(lmax, spin, 9801), lmax, spin, eps, "phi parts " + prec)
    plan.close()


def test_full_sky_lmax4096_stored_oracle():
    """Full-sky mode on the 21.6 M points of the lmax 4096 patch (FP64,
    eps 1e-10): N2 = 8281 (10240-point tier), the Theta grid of 16 562 rows as
    two transforms; against the stored oracle results of the patch."""
    fx = np.load(os.path.join(HERE, "golden", "spt1501_l4096_s2.npz"))
    w = syn.spt_fine("fp64")
    idx = fx["idx"]
    assert np.array_equal(idx, w.subsample(idx.shape[0]))
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, "fp64", full_sky=True)
    info = plan.info
    say("full sky lmax 4096: Lmax %d, n2 %d, Theta grid %d, phi grid %d" % (info["Lmax"], info["n2"],
                                                                            info["ntheta_grid"], info["nphi_grid"]))
    assert info["full_sky"] == 1 and info["ntheta_grid"] > 10240
    f = plan.synth(dev(w.alm())).cpu().numpy()[idx]
    e1 = rel(f, fx["synth"])
    g = torch.zeros(w.npoints, dtype=torch.complex128, device="cuda")
    g[torch.as_tensor(idx, device="cuda")] = dev(fx["adj_in"].astype(np.complex128))
    at = plan.adjoint(g).cpu().numpy()
    k = fx["adj_k"]
    m, _ = syn.alm_m_l(w.lmax)
    mk = m[k]
    wt = np.where(mk == 0, 1.0, 2.0)
    ga = np.where(mk == 0, at[:, k].real + 0j, at[:, k])
    ra = np.where(mk == 0, fx["adj_out"].real + 0j, fx["adj_out"])
    e2 = math.sqrt(float(np.sum(wt * np.abs(ga - ra) ** 2)) / float(np.sum(wt * np.abs(ra) ** 2)))
    say("  synth %.2e, adjoint %.2e" % (e1, e2))
    assert e1 <= 1e-9 and e2 <= 1e-9
    plan.close()


def test_table1_lmax10000_spt_field():
    """Table I's lmax 10000 SPT-3G row (theta* = 35 deg) at eps 1e-7: phi rows
    of 25 600 points in four parts; synthesis on 8 points and the adjoint of a
    map on 8 points (20 000 coefficients compared) against the oracle."""
    lmax, spin, eps = 10000, 0, 1e-7
    th, ph = syn.uniform_cap(20000, 35 * DEG, 9900)
    plan = Plan(th, ph, lmax, spin, eps, "fp64")
    info = plan.info
    say("lmax 10000: Lmax %d, mmax %d, phi grid %d, predicted speed-up %.2f" % (
        info["Lmax"], info["mmax"], info["nphi_grid"], info["predicted_speedup"]))
    assert info["nphi_grid"] > 2 * 10240
    sel = np.sort(syn.rng(9901).choice(th.shape[0], 8, replace=False))
    a = syn.gaussian_alm(lmax, spin, 9902)
    f = plan.synth(dev(a)).cpu().numpy()
    e1 = rel(f[sel], oracle.synth(a, th[sel], ph[sel], lmax, spin))
    g = np.zeros(th.shape[0], dtype=np.complex128)
    g[sel] = syn.gaussian_map(8, 9903)
    at = plan.adjoint(dev(g)).cpu().numpy()
    ref = oracle.adjoint(g[sel], th[sel], ph[sel], lmax, spin)
    k = np.sort(syn.rng(9904).choice(syn.nalm(lmax), 20000, replace=False))
    m, _ = syn.alm_m_l(lmax)
    mk = m[k]
    wt = np.where(mk == 0, 1.0, 2.0)
    ga = np.where(mk == 0, at[:, k].real + 0j, at[:, k])
    ra = np.where(mk == 0, ref[:, k].real + 0j, ref[:, k])
    e2 = math.sqrt(float(np.sum(wt * np.abs(ga - ra) ** 2)) / float(np.sum(wt * np.abs(ra) ** 2)))
    say("  synth %.2e, adjoint %.2e" % (e1, e2))
    assert e1 <= 10 * eps and e2 <= 10 * eps
    plan.close()
