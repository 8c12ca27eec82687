"""Seeded random configurations against the oracle.

Each case draws lmax, spin, cap radius (up to 179 degrees: the full-sky
fallback), epsilon, precision, point count and layout (uniform caps or tight
clusters) from a fixed generator, and checks the synthesis on up to 200 points
and the adjoint of a map supported on them against the oracle's direct sums
(Sec. I definitions) at <= 10 eps.  The draws reach the segmented and the plain
Legendre work lists, the full-sky fallback, FP32 and FP64 plans, single points
and points that share one NUFFT cell.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan

pytestmark = pytest.mark.gpu
DEG = math.pi / 180
NCASES = 48


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def draw(case):
    r = np.random.default_rng(41000 + case)
    lmax = int(r.choice([0, 1, 2, 5, 17, 64, 100, 257, 400, 511, 700, 1024]))
    spin = int(r.integers(0, min(3, lmax) + 1))
    rad = float(r.choice([0.05, 0.3, 1.0, 2.5, 7.0, 15.0, 30.0, 60.0, 89.0, 120.0, 179.0]))
    eps = float(r.choice([1e-4, 1e-6, 1e-8, 1e-10, 1e-12]))
    prec = str(r.choice(["auto", "fp64", "fp32"])) if eps >= 1e-6 else "fp64"
    n = int(r.choice([1, 7, 200, 3000, 12000]))
    if r.integers(2) == 0:
        th, ph = syn.uniform_cap(n, rad * DEG, 41500 + case)
        layout = "cap"
    else:  # tight clusters around five points of the cap
        th0, ph0 = syn.uniform_cap(5, rad * DEG, 41500 + case)
        k = r.integers(0, 5, n)
        sc = float(r.choice([1e-7, 1e-4, 1e-2]))
        th = np.clip(th0[k] + sc * r.standard_normal(n), 0.0, rad * DEG)
        ph = ph0[k] + sc * r.standard_normal(n)
        layout = "cluster %g" % sc
    idx = np.sort(r.choice(n, min(n, 200), replace=False))
    return lmax, spin, rad, eps, prec, th, ph, idx, layout


@pytest.mark.parametrize("case", range(NCASES))
def test_random_config(case):
    lmax, spin, rad, eps, prec, th, ph, idx, layout = draw(case)
    say("case %d: lmax %d spin %d cap %g deg eps %g %s, %d points (%s)" %
        (case, lmax, spin, rad, eps, prec, th.shape[0], layout))
    p = Plan(th, ph, lmax, spin, eps, prec)
    fp32 = bool(p.info["map_is_fp32"])
    a = syn.gaussian_alm(lmax, spin, 42000 + case)
    f = p.synth(torch.as_tensor(a, device="cuda")).cpu().numpy().astype(np.complex128)
    ref = oracle.synth(a, th[idx], ph[idx], lmax, spin)
    es = float(np.linalg.norm(f[idx] - ref) / np.linalg.norm(ref))
    g = np.zeros(th.shape[0], dtype=np.complex64 if fp32 else np.complex128)
    g[idx] = syn.gaussian_map(len(idx), 42500 + case)
    at = p.adjoint(torch.as_tensor(g, device="cuda")).cpu().numpy()
    aref = oracle.adjoint(g[idx].astype(np.complex128), th[idx], ph[idx], lmax, spin)
    d = at - aref
    ea = math.sqrt(max(oracle.alm_dot(d, d, lmax), 0.0) / oracle.alm_dot(aref, aref, lmax))
    say("  synthesis %.2e, adjoint %.2e (segment %d, full sky %d)" %
        (es, ea, p.info["syn_segment"], p.info["full_sky"]))
    assert es <= 10 * eps and ea <= 10 * eps
    assert p.dropped_points() == 0
    p.close()
