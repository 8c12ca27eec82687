"""GPU parity of the lmax 4096, spin-2, 21.6 M-point patch (1501 deg^2 at
0.5 arcmin) in both precisions, at full size, against stored oracle results
(tests/golden/spt1501_l4096_s2.npz, written by tests/golden/make_fixtures.py
from the CPU oracle alone): the synthesis on a seeded 10 000-point
subsample, and the adjoint of a map that is non-zero only on that subsample
on 20 480 seeded coefficients.  Bar: relative L2 <= 10 eps (eps 1e-5 for the
FP32 form, 1e-10 for FP64)."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "spt1501_l4096_s2.npz")


def say(*a):
    print(*a, flush=True)


def weighted_rel(got, ref, mk):
    """Relative L2 under the coefficient inner product (m = 0: real parts once; m > 0 twice)."""
    w = np.where(mk == 0, 1.0, 2.0)
    g = np.where(mk == 0, got.real + 0j, got)
    r = np.where(mk == 0, ref.real + 0j, ref)
    return math.sqrt(float(np.sum(w * np.abs(g - r) ** 2)) / float(np.sum(w * np.abs(r) ** 2)))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_spt1501_lmax4096_vs_stored_oracle(prec):
    fx = np.load(FIXTURE)
    w = syn.spt_fine(prec)
    idx = fx["idx"]
    say("spt1501 lmax 4096 %s: %d points, eps %g; fixture subsample %d" % (prec, w.npoints, w.epsilon, idx.shape[0]))
    assert np.array_equal(idx, w.subsample(idx.shape[0]))
    assert np.array_equal(fx["theta"], w.theta[idx]) and np.array_equal(fx["phi"], w.phi[idx])
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision)
    fp32 = bool(plan.info["map_is_fp32"])
    assert fp32 == (prec == "fp32")
    f = plan.synth(torch.as_tensor(w.alm(), device="cuda")).cpu().numpy()[idx].astype(np.complex128)
    err = float(np.linalg.norm(f - fx["synth"]) / np.linalg.norm(fx["synth"]))
    say("  synth rel L2 on %d points: %.3e" % (idx.shape[0], err))
    assert err <= 10 * w.epsilon

    g = torch.zeros(w.npoints, dtype=plan.map_dtype, device="cuda")
    g[torch.as_tensor(idx, device="cuda")] = torch.as_tensor(
        fx["adj_in"].astype(np.complex64 if fp32 else np.complex128), device="cuda")
    at = plan.adjoint(g).cpu().numpy()
    k = fx["adj_k"]
    m, l = syn.alm_m_l(w.lmax)
    aerr = weighted_rel(at[:, k], fx["adj_out"], m[k])
    say("  adjoint rel L2 on %d coefficients: %.3e" % (k.shape[0], aerr))
    assert aerr <= 10 * w.epsilon
    assert np.all(at[:, l < w.spin] == 0)
    assert np.all(at[:, m == 0].imag == 0)
    plan.close()


@pytest.mark.parametrize("prec,opts", [
    ("fp32", {"cl": "red"}), ("fp64", {"cl": "red"}), ("fp64", {"window": "kb"}), ("fp64", {"window": "pswf"}),
    ("fp32", {"window": "pswf"}), ("fp64", {"lmax_rule": "cost"}), ("fp32", {"lmax_rule": "cost"})])
def test_spt1501_plan_options_vs_stored_oracle(prec, opts):
    """The plan options at full size, against the same stored oracle results:
    Lmax tuned to the coefficients' spectrum C_l = (l+1)^-2 (Sec. II.D), the
    Kaiser-Bessel and Slepian bells (Sec. II.C) and the least-work Lmax rule
    (footnote to eq. Lmax2); synthesis and adjoint within 10 eps."""
    fx = np.load(FIXTURE)
    w = syn.spt_fine(prec)
    idx = fx["idx"]
    kw = dict(opts)
    if kw.get("cl") == "red":
        kw["cl"] = 1.0 / (1.0 + np.arange(w.lmax + 1)) ** 2
    plan = Plan(w.theta, w.phi, w.lmax, w.spin, w.epsilon, w.precision, **kw)
    info = plan.info
    say("spt1501 lmax 4096 %s %s: Lmax %d (rule %d), eps_apo %.4f, predicted %.2e" % (
        prec, sorted(opts), info["Lmax"], info["Lmax_rule"], info["eps_apo"], info["predicted_error"]))
    if "cl" in opts:
        assert info["Lmax"] <= info["Lmax_rule"] and 0 < info["predicted_error"] <= 0.5 * w.epsilon
    f = plan.synth(torch.as_tensor(w.alm(), device="cuda")).cpu().numpy()[idx].astype(np.complex128)
    err = float(np.linalg.norm(f - fx["synth"]) / np.linalg.norm(fx["synth"]))
    fp32 = bool(plan.info["map_is_fp32"])
    g = torch.zeros(w.npoints, dtype=plan.map_dtype, device="cuda")
    g[torch.as_tensor(idx, device="cuda")] = torch.as_tensor(
        fx["adj_in"].astype(np.complex64 if fp32 else np.complex128), device="cuda")
    at = plan.adjoint(g).cpu().numpy()
    k = fx["adj_k"]
    m, _ = syn.alm_m_l(w.lmax)
    aerr = weighted_rel(at[:, k], fx["adj_out"], m[k])
    say("  synth %.3e adjoint %.3e" % (err, aerr))
    assert err <= 10 * w.epsilon and aerr <= 10 * w.epsilon
    assert plan.dropped_points() == 0
    plan.close()
