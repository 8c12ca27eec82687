"""Plan options on the GPU, against the oracle.

* Lmax tuned to the field's power spectrum (Sec. II.D): the plan takes the
  smallest smooth Lmax whose predicted error (eqs. s2m, st, cm, cms) for that
  spectrum stays below epsilon / 2.  For fields drawn from that spectrum
  (C_l = (l+1)^-2, the spectrum of the seeded coefficients) the synthesis on
  the smaller grid still meets epsilon.
* The Kaiser-Bessel and Slepian (PSWF) apodization bells (Sec. II.C) and the
  least-work Lmax rule (footnote to eq. Lmax2): synthesis and adjoint within
  10 epsilon (relative L2), the bar of the other parity tests."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("lmax,radius,eps,spin,prec", [(1024, 5, 1e-5, 2, "fp32"), (512, 3, 1e-8, 0, "fp64"),
                                                       (1024, 3, 1e-10, 2, "fp64")])
def test_tuned_plan_meets_epsilon(lmax, radius, eps, spin, prec):
    say("tuned plan: lmax %d, %g deg, eps %g, spin %d, %s" % (lmax, radius, eps, spin, prec))
    th, ph = syn.uniform_cap(400, radius * DEG, 8100 + lmax)
    l = np.arange(lmax + 1)
    cl = 1.0 / (1.0 + l) ** 2
    plan = Plan(th, ph, lmax, spin, eps, prec, cl=cl)
    info = plan.info
    assert info["Lmax"] < info["Lmax_rule"] and 0 < info["predicted_error"] <= 0.5 * eps
    a = syn.gaussian_alm(lmax, spin, 8200 + lmax)
    ref = oracle.synth(a, th, ph, lmax, spin)
    f = plan.synth(torch.as_tensor(a).cuda()).cpu().numpy().astype(np.complex128)
    e = float(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    say("  Lmax %d (rule %d), predicted %.2e, measured %.2e" % (info["Lmax"], info["Lmax_rule"],
                                                                info["predicted_error"], e))
    assert e <= 2 * eps
    assert plan.dropped_points() == 0
    plan.close()


def _alm_rel(a, b, lmax):
    d = a - b
    return math.sqrt(max(oracle.alm_dot(d, d, lmax), 0.0) / oracle.alm_dot(b, b, lmax))


@pytest.mark.parametrize("window,rule,lmax,radius,eps,spin,prec", [
    ("kb", "band", 1024, 10, 1e-10, 2, "fp64"), ("pswf", "band", 1024, 10, 1e-10, 2, "fp64"),
    ("kb", "band", 512, 20, 1e-5, 0, "fp32"), ("pswf", "band", 512, 20, 1e-5, 2, "fp32"),
    ("es", "cost", 1024, 10, 1e-10, 2, "fp64"), ("pswf", "cost", 512, 5, 1e-8, 1, "fp64")])
def test_bells_and_cost_rule_vs_oracle(window, rule, lmax, radius, eps, spin, prec):
    say("window %s, rule %s: lmax %d, %g deg, eps %g, spin %d, %s" % (window, rule, lmax, radius, eps, spin, prec))
    th, ph = syn.uniform_cap(400, radius * DEG, 8300 + lmax + spin)
    plan = Plan(th, ph, lmax, spin, eps, prec, window=window, lmax_rule=rule)
    assert plan.info["window"] == {"es": 0, "kb": 1, "pswf": 2}[window]
    a = syn.gaussian_alm(lmax, spin, 8400 + lmax)
    ref = oracle.synth(a, th, ph, lmax, spin)
    f = plan.synth(torch.as_tensor(a).cuda()).cpu().numpy().astype(np.complex128)
    e1 = float(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    fp32 = bool(plan.info["map_is_fp32"])
    g = syn.gaussian_map(th.shape[0], 8500 + lmax).astype(np.complex64 if fp32 else np.complex128)
    at = plan.adjoint(torch.as_tensor(g).cuda()).cpu().numpy()
    e2 = _alm_rel(at, oracle.adjoint(g.astype(np.complex128), th, ph, lmax, spin), lmax)
    say("  Lmax %d, eps_apo %.3f: synth %.2e adjoint %.2e" % (plan.info["Lmax"], plan.info["eps_apo"], e1, e2))
    assert e1 <= 10 * eps and e2 <= 10 * eps
    assert plan.dropped_points() == 0
    plan.close()
