"""CPU tests of the library's host side: the C ABI exports, the kernels'
own Legendre seeds/tables (evaluated on the host), the plan parameter rules
(Table I, the error model of eq. s2m), the window and the polar cut-offs."""
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2603_17166_amd import _lib
from paper_2603_17166_amd.plan import legendre_column, plan_geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEG = math.pi / 180


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "psht.h")).read()
    declared = set(re.findall(r"\b(psht_[a-z_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    lib = _lib.load()
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("lmax,s,m,theta", [
    (64, 0, 0, 0.3), (64, 2, 1, 1.2), (64, 2, 5, 2.9), (64, 3, 1, 0.7), (300, 2, 150, 0.9),
    (300, 0, 299, 1.5), (2048, 2, 1400, 0.7), (2048, 2, 2, 1.3e-3), (1024, 1, 0, 0.2), (100, 5, 3, 0.5),
])
def test_kernel_legendre_column_vs_oracle(lmax, s, m, theta):
    """The GPU kernels' seeds, tables, recurrence and rescaling, run on the
    host, against the oracle's Wigner d (eq. Ylm)."""
    lp, lm = legendre_column(lmax, s, m, theta)
    l = np.arange(lmax + 1)
    nrm = np.sqrt((2 * l + 1) / (4 * math.pi))
    op = nrm * oracle.wigner_d(lmax, m, -s, theta)
    om = nrm * oracle.wigner_d(lmax, m, s, theta)
    for got, ref in ((lp, op), (lm, om)):
        scale = max(np.max(np.abs(ref)), 1e-300)
        assert np.max(np.abs(got - ref)) <= 5e-12 * scale


def test_kernel_legendre_deep_polar_rescaling():
    """Seeds far below the double range (sin(theta/2)^(2m) ~ 1e-2000) are
    carried with an exponent and come back to the right values."""
    lmax, s, theta = 4096, 2, 0.05
    for m in (150, 190, 200):   # lmax sin(theta) ~ 205: the values near l = lmax are O(1e-3 .. 1)
        lp, lm = legendre_column(lmax, s, m, theta)
        l = np.arange(lmax + 1)
        nrm = np.sqrt((2 * l + 1) / (4 * math.pi))
        op = nrm * oracle.wigner_d(lmax, m, -s, theta)
        om = nrm * oracle.wigner_d(lmax, m, s, theta)
        assert np.max(np.abs(op)) > 1e-6
        for got, ref in ((lp, op), (lm, om)):
            assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def _table1():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "table1_predicted.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, ts, lmax, spin, pred = line.split()
        rows.append((name, float(ts), int(lmax), int(spin), float(pred)))
    return rows


@pytest.mark.parametrize("name,ts,lmax,spin,pred", _table1())
def test_table1_predicted_speedup(name, ts, lmax, spin, pred):
    """Sec. II.B-C parameter rules + the Sec. II.A estimate reproduce the
    'predicted speed-up' column of Table I (theta* printed rounded)."""
    info, _, _, _ = plan_geometry(lmax, spin, ts * DEG, 1e-7)
    tol = 0.02 if name == "EDFS" else 0.08
    assert abs(info["predicted_speedup"] / pred - 1) < tol


def test_parameter_rules():
    lmax, ts, eps = 2048, 35.3 * DEG, 1e-10
    info, th, w, mm = plan_geometry(lmax, 2, ts, eps)
    eps_apo = math.sqrt(2 * abs(math.log(eps)) / (ts * lmax))
    assert abs(info["alpha"] - abs(math.log(eps)) / math.pi) < 1e-15
    assert abs(info["eps_apo"] - eps_apo) < 1e-14
    assert abs(info["theta_max"] - ts * (1 + eps_apo)) < 1e-14
    lf = lmax * ts / math.pi * (1 + eps_apo) ** 2
    assert info["Lmax"] >= math.ceil(lf - 1e-9) and info["Lmax"] <= 1.06 * lf + 2
    n2 = info["n2"]
    assert n2 == 2 * info["Lmax"] + 1
    for p in (3, 5, 7, 11, 13):
        while n2 % p == 0:
            n2 //= p
    assert n2 == 1
    j = np.arange(info["Lmax"] + 1)
    assert np.allclose(th, 2 * math.pi * j / info["n2"] * info["theta_max"] / math.pi, rtol=1e-15, atol=0)


def test_window_shape():
    info, th, w, _ = plan_geometry(1024, 0, 20 * DEG, 1e-8)
    Theta = th * math.pi / info["theta_max"]
    Theta_star = math.pi / (1 + info["eps_apo"])
    assert np.all(w[Theta <= Theta_star] == 1.0)
    assert np.all(np.diff(w) <= 1e-15)
    assert np.all((w >= 0) & (w <= 1))
    assert w[-1] < 1e-6


def test_full_sky_fallback():
    info, th, w, _ = plan_geometry(256, 2, 150 * DEG, 1e-10)
    assert info["full_sky"] == 1 and info["theta_max"] == math.pi
    assert info["Lmax"] >= 256 and np.all(w == 1.0)


def _sigma_m(info, th, w, lmax, ntheta=600, ms=None):
    """Error of eq. s2m: |sum_j w_j D_j(Theta) e^{i m theta_j} - e^{i m theta}|
    over the doubled circle (rings j and their mirrors -j), theta in [0, theta*]."""
    L, n2, tmax = info["Lmax"], info["n2"], info["theta_max"]
    jj = np.concatenate([np.arange(L + 1), -np.arange(1, L + 1)])
    ww = np.concatenate([w, w[1:]])
    Thj = 2 * math.pi * jj / n2
    thj = Thj * tmax / math.pi
    theta = np.linspace(0, info["theta_star"], ntheta)
    Theta = theta * math.pi / tmax
    d = Theta[:, None] - Thj[None, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        D = np.sin(n2 * d / 2) / (n2 * np.sin(d / 2))
    D[np.abs(np.sin(d / 2)) < 1e-15] = 1.0
    ms = np.arange(lmax + 1) if ms is None else ms
    approx = (D * ww[None, :]) @ np.exp(1j * np.outer(thj, ms))
    return np.abs(approx - np.exp(1j * np.outer(theta, ms)))


@pytest.mark.parametrize("lmax,ts,eps", [(128, 10, 1e-10), (128, 10, 1e-5), (512, 20, 1e-5), (512, 20, 1e-10),
                                         (2048, 35.5, 1e-10)])
def test_error_model_s2m_within_tolerance(lmax, ts, eps):
    """Brute-force eq. s2m with the plan's rings and weights: every wave
    e^{i m theta}, m <= lmax, is reproduced inside the cap to epsilon."""
    info, th, w, _ = plan_geometry(lmax, 0, ts * DEG, eps)
    ms = np.arange(lmax + 1) if lmax <= 512 else np.unique(np.concatenate([np.arange(0, lmax + 1, 7), np.arange(lmax - 64, lmax + 1)]))
    sig = _sigma_m(info, th, w, lmax, ms=ms)
    assert np.max(sig) <= eps


def test_error_model_zero_at_rings():
    """The error of eq. s2m vanishes at the ring positions inside the cap
    (footnote to eq. s2m): the Dirichlet kernel interpolates its nodes."""
    lmax, eps = 256, 1e-8
    info, th, w, _ = plan_geometry(lmax, 0, 15 * DEG, eps)
    L, n2, tmax = info["Lmax"], info["n2"], info["theta_max"]
    jj = np.concatenate([np.arange(L + 1), -np.arange(1, L + 1)])
    ww = np.concatenate([w, w[1:]])
    thj = 2 * math.pi * jj / n2 * tmax / math.pi
    inside = np.nonzero(th <= info["theta_star"])[0]
    ms = np.arange(lmax + 1)
    for k in inside[:: max(1, len(inside) // 8)]:
        d = (th[k] - thj) * math.pi / tmax
        with np.errstate(invalid="ignore", divide="ignore"):
            D = np.sin(n2 * d / 2) / (n2 * np.sin(d / 2))
        D[np.abs(np.sin(d / 2)) < 1e-15] = 1.0
        err = np.abs((D * ww) @ np.exp(1j * np.outer(thj, ms)) - np.exp(1j * th[k] * ms))
        assert np.max(err) < 1e-12


def test_polar_cutoff_is_tight():
    """Orders above mmax_j are below tau = 1e-4 epsilon on ring j for every l,
    and mmax_j itself is not (oracle Wigner d)."""
    lmax, s, eps = 256, 2, 1e-10
    info, th, w, mm = plan_geometry(lmax, s, 20 * DEG, eps)
    tau = 1e-4 * eps
    l = np.arange(lmax + 1)
    nrm = np.sqrt((2 * l + 1) / (4 * math.pi))

    def colmax(m, t):
        return max(np.max(np.abs(nrm * oracle.wigner_d(lmax, m, -s, t))), np.max(np.abs(nrm * oracle.wigner_d(lmax, m, s, t))))

    for j in list(range(1, len(th), max(1, len(th) // 12))) + [len(th) - 1]:
        if mm[j] < lmax:
            assert colmax(mm[j] + 1, th[j]) < tau
        if mm[j] > s:
            assert colmax(mm[j], th[j]) >= tau
    assert mm[0] == s


def test_invalid_arguments():
    for args in [(-1, 0, 0.1, 1e-5), (10, 11, 0.1, 1e-5), (10, 0, 0.1, 0.5), (10, 0, 0.1, 1e-20), (10, 0, 4.0, 1e-5)]:
        with pytest.raises(_lib.PshtError) as e:
            plan_geometry(*args)
        assert e.value.code == _lib.PSHT_ERR_ARG


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14])
@pytest.mark.parametrize("prec", ["auto", "fp64"])
def test_kernel_polynomial_table_accuracy(eps, prec):
    """The inner ES kernel taps are evaluated from polynomials; the plan
    checks them against the kernel formula on a fine grid (both signs of the
    offset) in the arithmetic the kernels use, and reports the largest error,
    which must stay below eps: 1e-3 eps for the FP64 table, and for the float
    table of the FP32 form (eps >= 1e-6 under "auto") the larger of that and
    2e-7, the float evaluation's own level."""
    info = plan_geometry(256, 2, 0.3, eps, prec)[0]
    bound = max(1e-3 * eps, 2e-7 if info["map_is_fp32"] else 1e-14)
    assert bool(info["map_is_fp32"]) == (prec == "auto" and eps >= 1e-6)
    assert 0.0 < info["kernel_poly_err"] <= bound
