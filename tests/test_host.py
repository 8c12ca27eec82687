"""CPU tests of the library's host side: the C ABI exports, the kernels'
own Legendre seeds/tables (evaluated on the host), the plan parameter rules
(Table I, the error model of eq. s2m), the window and the polar cut-offs."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2603_17166_amd import _lib
from paper_2603_17166_amd.plan import great_circle_spectrum, legendre_column, plan_geometry

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


@pytest.mark.parametrize("lmax,s", [(64, 0), (64, 2), (300, 2), (200, 3), (40, 1)])
def test_great_circle_spectrum_vs_oracle(lmax, s):
    """c_m of eq. cm / eq. cms from the library's long-double recurrence at
    theta = pi/2 against the oracle's Wigner d at pi/2, for a non-trivial
    spectrum; negative m uses d^l_{|m|, s}."""
    l = np.arange(lmax + 1)
    cl = np.exp(-0.3 * np.sqrt(l)) * (1 + 0.5 * np.cos(l))
    cm = great_circle_spectrum(lmax, s, cl)
    ref = np.zeros(2 * lmax + 1)
    for m in range(-lmax, lmax + 1):
        d = oracle.wigner_d(lmax, m, -s, math.pi / 2)
        ref[m + lmax] = np.sum(cl * (2 * l + 1) / 2 * d ** 2)
    assert np.max(np.abs(cm - ref)) <= 1e-13 * np.max(ref)


def test_great_circle_spectrum_closed_forms():
    """Sum rule: sum_m |d^l_{m,-s}|^2 = 1 (unitarity), so sum_m c_m =
    sum_l C_l (2l+1)/2.  Single multipole l = L at spin 0: c_0 =
    (2L+1)/2 P_L(0)^2 with P_L(0) = (-1)^(L/2) (L-1)!!/L!! for even L and 0
    for odd L; and c_m = c_-m."""
    lmax = 120
    l = np.arange(lmax + 1)
    for s in (0, 2, 5):
        cl = (l >= s) / (1.0 + l) ** 1.5
        cm = great_circle_spectrum(lmax, s, cl)
        assert abs(cm.sum() / np.sum(cl * (2 * l + 1) / 2) - 1) < 1e-13
    for L in (10, 11, 64, 97):
        cl = np.zeros(lmax + 1)
        cl[L] = 1.0
        cm = great_circle_spectrum(lmax, 0, cl)
        p0 = 0.0 if L % 2 else (-1) ** (L // 2) * math.exp(math.lgamma(L + 1) - L * math.log(2) - 2 * math.lgamma(L // 2 + 1))
        assert abs(cm[lmax] - (2 * L + 1) / 2 * p0 ** 2) < 1e-13
        assert np.allclose(cm, cm[::-1], rtol=0, atol=1e-14)
        assert np.all(cm[: lmax - L] == 0) and np.all(cm[lmax + L + 1:] == 0)


@pytest.mark.parametrize("lmax,ts,eps,s", [(512, 5, 1e-5, 2), (512, 3, 1e-8, 0), (1024, 3, 1e-10, 0)])
def test_tuned_lmax_predicted_error_vs_brute_force(lmax, ts, eps, s):
    """Lmax tuned to a red spectrum C_l = (l+1)^-2 (Sec. II.D): it is at most
    the eq. Lmax2 value, and the field error of eq. st, evaluated by brute
    force (eq. s2m over every m = -lmax..lmax on a fine theta grid with the
    plan's rings and weights), stays below epsilon / 2 of the field's rms and
    agrees with the plan's own (subsampled) prediction."""
    l = np.arange(lmax + 1)
    cl = 1.0 / (1.0 + l) ** 2
    info, th, w, _ = plan_geometry(lmax, s, ts * DEG, eps, cl=cl)
    base = plan_geometry(lmax, s, ts * DEG, eps)[0]
    assert base["predicted_error"] == -1.0 and base["Lmax"] == base["Lmax_rule"]
    assert info["Lmax_rule"] == base["Lmax"] and info["Lmax"] < info["Lmax_rule"]
    assert info["theta_max"] == base["theta_max"]
    cm = great_circle_spectrum(lmax, s, cl)
    ms = np.arange(-lmax, lmax + 1)
    sig = _sigma_m(info, th, w, lmax, ntheta=800, ms=ms)
    brute = math.sqrt(np.max(sig ** 2 @ cm) / cm.sum())
    assert brute <= 0.6 * eps
    assert 0.7 < info["predicted_error"] / brute < 1.3


def test_tuning_arguments():
    for cl in (np.ones(50), -np.ones(129), np.full(129, np.nan)):
        with pytest.raises(_lib.PshtError) as e:
            plan_geometry(128, 0, 0.2, 1e-8, cl=cl)
        assert e.value.code == _lib.PSHT_ERR_ARG
    with pytest.raises(ValueError):
        great_circle_spectrum(128, 0, np.ones(100))
    with pytest.raises(_lib.PshtError):
        great_circle_spectrum(10, 11, np.ones(11))
    # full-sky plans keep Lmax = lmax whatever the spectrum
    info = plan_geometry(128, 0, 0.2, 1e-8, full_sky=True, cl=np.ones(129))[0]
    assert info["Lmax"] >= 128 and info["predicted_error"] == -1.0


def _scipy_bell(kind, alpha, x):
    """The three bells of Sec. II.C on [-1, 1] from scipy's special functions."""
    import scipy.special as sp
    if kind == "es":
        return np.exp(alpha * math.pi * (np.sqrt(1 - x * x) - 1))
    if kind == "kb":
        return sp.i0(alpha * math.pi * np.sqrt(1 - x * x))
    return sp.pro_ang1(0, 0, alpha * math.pi, x)[0]


def test_kaiser_bessel_bell_fourier_closed_form():
    """The Kaiser-Bessel bell I0(pi alpha sqrt(1 - (Theta/pi)^2)) on
    [-pi, pi] has the normalized Fourier transform printed with eq. KB:
    (pi alpha / sinh(pi alpha)) sinh(pi sqrt(alpha^2 - k^2)) / (pi sqrt(alpha^2 - k^2))
    (sin for k > alpha), checked by quadrature."""
    import scipy.integrate as si
    alpha = abs(math.log(1e-8)) / math.pi
    b0 = si.quad(lambda t: _scipy_bell("kb", alpha, t / math.pi), -math.pi, math.pi, epsrel=1e-13)[0]
    for k in (0.0, 1.5, 4.0, alpha - 0.3, alpha + 0.7, 9.0):
        got = si.quad(lambda t: _scipy_bell("kb", alpha, t / math.pi) * math.cos(k * t), -math.pi, math.pi,
                      epsrel=1e-12, epsabs=1e-14 * b0, limit=400)[0] / b0
        q = alpha * alpha - k * k
        shape = (math.sinh(math.pi * math.sqrt(q)) / (math.pi * math.sqrt(q)) if q > 0 else
                 (math.sin(math.pi * math.sqrt(-q)) / (math.pi * math.sqrt(-q)) if q < 0 else 1.0))
        want = math.pi * alpha / math.sinh(math.pi * alpha) * shape
        assert abs(got - want) < 1e-11


@pytest.mark.parametrize("kind", ["es", "kb", "pswf"])
@pytest.mark.parametrize("lmax,ts,eps", [(512, 10, 1e-5), (1024, 20, 1e-10)])
def test_window_bells_vs_scipy(kind, lmax, ts, eps):
    """Ring weights = 1 - the unit-area cumulative integral of the chosen bell
    across the apodization zone (Sec. II.C, Fig. 4), against scipy's bells
    integrated by adaptive quadrature."""
    import scipy.integrate as si
    info, th, w, _ = plan_geometry(lmax, 0, ts * DEG, eps, window=kind)
    assert info["window"] == _lib.WINDOWS[kind]
    a = info["alpha"]
    Ts = math.pi / (1 + info["eps_apo"])
    dT, h = math.pi - Ts, (math.pi + Ts) / 2
    Th = th * math.pi / info["theta_max"]

    def integral(x):
        return si.quad(lambda y: _scipy_bell(kind, a, y), -1, x, epsabs=0, epsrel=1e-13, limit=200)[0]

    norm = integral(1.0)
    for T, wj in zip(Th, w):
        ref = 1.0 if T <= Ts else 1.0 - integral(min(2 * (T - h) / dT, 1.0)) / norm
        assert abs(wj - ref) < 1e-10


@pytest.mark.parametrize("kind", ["kb", "pswf"])
@pytest.mark.parametrize("lmax,ts,eps", [(512, 10, 1e-5), (512, 20, 1e-10), (2048, 35.5, 1e-7)])
def test_error_model_s2m_other_bells(kind, lmax, ts, eps):
    """Eq. s2m by brute force for the Kaiser-Bessel and Slepian windows (same
    alpha, apodization length and Lmax as the ES rule): every wave is
    reproduced inside the cap to epsilon."""
    info, th, w, _ = plan_geometry(lmax, 0, ts * DEG, eps, window=kind)
    ms = np.arange(lmax + 1) if lmax <= 512 else np.unique(np.concatenate([np.arange(0, lmax + 1, 7), np.arange(lmax - 64, lmax + 1)]))
    assert np.max(_sigma_m(info, th, w, lmax, ms=ms)) <= eps


@pytest.mark.parametrize("lmax,ts,eps", [(512, 10, 1e-5), (1024, 20, 1e-10), (2048, 35.3, 1e-7)])
def test_cost_lmax_rule(lmax, ts, eps):
    """The least-work rule (footnote to eq. Lmax2) shortens the apodization
    zone, does no more Legendre work than eq. Lmax2, and keeps the eq. s2m
    error below epsilon."""
    band = plan_geometry(lmax, 2, ts * DEG, eps)[0]
    info, th, w, _ = plan_geometry(lmax, 2, ts * DEG, eps, lmax_rule="cost")
    assert info["eps_apo"] < band["eps_apo"] and info["theta_max"] < band["theta_max"]
    assert info["legendre_triples"] <= band["legendre_triples"]
    ms = np.unique(np.concatenate([np.arange(0, lmax + 1, 5), np.arange(lmax - 64, lmax + 1)]))
    assert np.max(_sigma_m(info, th, w, lmax, ms=ms)) <= eps


def test_option_arguments():
    for kw in ({"window": "es"}, ):
        plan_geometry(128, 0, 0.2, 1e-8, **kw)
    opts = _lib.PlanOptions()
    info = _lib.PlanInfo()
    lib = _lib.load()
    for field, bad in (("window", 3), ("lmax_rule", 2), ("full_sky", 2)):
        opts = _lib.PlanOptions()
        setattr(opts, field, bad)
        st = lib.psht_plan_geometry_ex(128, 0, 0.2, 1e-8, 0, ctypes.byref(opts), ctypes.byref(info), None, None, None, 0)
        assert st == _lib.PSHT_ERR_ARG


def test_rotation_arguments_on_host():
    """Host-side argument checks of the patch-frame calls (no device work)."""
    lib = _lib.load()
    n = ctypes.c_size_t()
    assert lib.psht_rotate_alm_workspace(4096, 2, ctypes.byref(n)) == _lib.PSHT_OK
    assert n.value == 2 * 4097 * 8193 * 16
    for lmax, nc in [(-1, 2), (16384, 1), (10, 3), (10, 0)]:
        assert lib.psht_rotate_alm_workspace(lmax, nc, ctypes.byref(n)) == _lib.PSHT_ERR_ARG
    assert lib.psht_rotate_points(-1, 0.0, 0.0, 0.0, None, None, None, None, None, None) == _lib.PSHT_ERR_ARG
    assert lib.psht_rotate_points(0, 0.0, 0.0, 0.0, None, None, None, None, None, None) == _lib.PSHT_OK
    assert lib.psht_spin_phase(5, 2, 0, 0, None, None, None) == _lib.PSHT_ERR_ARG
    assert lib.psht_spin_phase(0, 2, 1, 0, None, None, None) == _lib.PSHT_OK
