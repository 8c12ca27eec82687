"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: relative L2 <= 10 epsilon against the FP64 direct-sum oracle for
synthesis and adjoint (Sec. I definitions); the dot-product test checks that
the GPU adjoint is the exact transpose of the GPU synthesis; stage tests
check the Legendre step against the oracle's ring coefficients and the FFT
kernel against numpy.fft.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_17166_amd import _lib
from paper_2603_17166_amd import synthetic as syn
from paper_2603_17166_amd.plan import Plan, fft

pytestmark = pytest.mark.gpu
DEG = math.pi / 180


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.as_tensor(x).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def alm_rel(a, b, lmax):
    d = a - b
    return math.sqrt(max(oracle.alm_dot(d, d, lmax), 0.0) / oracle.alm_dot(b, b, lmax))


# ------------------------------------------------------------------ FFT (P13)

# the lengths cover every radix pass, the tiers of the LDS kernel up to 10240
# points (the 160 KB of LDS a gfx950 workgroup may use) and the phi-row lengths
# of the lmax 2048 workload (5880 and its half)
@pytest.mark.parametrize("n", [1, 2, 3, 6, 10, 12, 13, 14, 15, 91, 105, 143, 210, 1155, 2310, 2352, 2940, 4050, 5880,
                               6000, 8192, 7 * 11 * 13 * 4, 8281, 9009, 10240])
@pytest.mark.parametrize("fp32", [False, True])
def test_fft_vs_numpy(n, fp32):
    say("fft n=%d fp32=%s" % (n, fp32))
    r = syn.rng(n)
    x = r.standard_normal((3, n)) + 1j * r.standard_normal((3, n))
    xt = dev(x.astype(np.complex64 if fp32 else np.complex128))
    for sign in (-1, 1):
        y = fft(xt, sign).cpu().numpy()
        ref = np.fft.fft(x, axis=1) if sign == -1 else np.fft.ifft(x, axis=1) * n
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        tol = (3e-6 if fp32 else 2e-15) * max(1.0, math.log2(n))
        assert err < tol, (n, sign, err)


# ------------------------------------------------------------- configurations

def cap_case(lmax, spin, radius_deg, n, eps, precision="fp64", seed=0):
    th, ph = syn.uniform_cap(n, radius_deg * DEG, 7000 + seed)
    a = syn.gaussian_alm(lmax, spin, 7100 + seed)
    return th, ph, a, eps, precision


CASES = [
    # lmax, spin, radius, npoints, eps, precision
    (128, 0, 10.0, 20000, 1e-10, "fp64"),   # the 10-degree-cap workload at full size
    (128, 2, 10.0, 4000, 1e-10, "fp64"),
    (96, 1, 25.0, 3000, 1e-8, "fp64"),
    (64, 3, 40.0, 2000, 1e-12, "fp64"),
    (200, 2, 5.0, 3000, 1e-10, "fp64"),
    (128, 2, 10.0, 4000, 1e-5, "fp32"),
    (256, 0, 20.0, 3000, 1e-5, "fp32"),
    (40, 2, 150.0, 2000, 1e-10, "fp64"),    # patch too large: full-sky fallback
    (1024, 2, 50.0, 3000, 1e-10, "fp64"),   # phi rows of more than 2560 points: two half-length transforms
]


def _ids(c):
    return "l%d-s%d-r%g-n%d-eps%g-%s" % c


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_synth_parity(case):
    lmax, spin, rad, n, eps, prec = case
    say("synth", _ids(case))
    th, ph, a, eps, prec = cap_case(lmax, spin, rad, n, eps, prec)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    f = plan.synth(dev(a)).cpu().numpy().astype(np.complex128)
    ref = oracle.synth(a, th, ph, lmax, spin)
    err = rel_l2(f, ref)
    say("  rel L2 = %.3e (eps %.0e) info Lmax=%d mmax=%d W=%d" % (err, eps, plan.info["Lmax"], plan.info["mmax"],
                                                                 plan.info["nufft_w"]))
    assert err <= 10 * eps


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_adjoint_parity(case):
    lmax, spin, rad, n, eps, prec = case
    say("adjoint", _ids(case))
    th, ph, _, eps, prec = cap_case(lmax, spin, rad, n, eps, prec)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    f = syn.gaussian_map(n, 7200)
    ft = dev(f.astype(np.complex64 if plan.info["map_is_fp32"] else np.complex128))
    if plan.info["map_is_fp32"]:
        f = ft.cpu().numpy().astype(np.complex128)
    at = plan.adjoint(ft).cpu().numpy()
    ref = oracle.adjoint(f, th, ph, lmax, spin)
    err = alm_rel(at, ref, lmax)
    say("  rel L2 = %.3e" % err)
    assert err <= 10 * eps
    m, l = syn.alm_m_l(lmax)
    assert np.all(at[:, l < spin] == 0)
    assert np.all(at[:, m == 0].imag == 0)


@pytest.mark.parametrize("case", CASES[:5] + CASES[5:7], ids=_ids)
def test_dot_product(case):
    """<synth a, f> = <a, adjoint f> for the GPU pair (exact transpose)."""
    lmax, spin, rad, n, eps, prec = case
    say("dot", _ids(case))
    th, ph, a, eps, prec = cap_case(lmax, spin, rad, n, eps, prec, seed=3)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    fp32 = bool(plan.info["map_is_fp32"])
    f = syn.gaussian_map(n, 7300).astype(np.complex64 if fp32 else np.complex128)
    sa = plan.synth(dev(a)).cpu().numpy().astype(np.complex128)
    at = plan.adjoint(dev(f)).cpu().numpy()
    lhs = oracle.map_dot(sa, f.astype(np.complex128))
    rhs = oracle.alm_dot(a, at, lmax)
    scale = np.linalg.norm(sa) * np.linalg.norm(f)
    say("  |lhs-rhs|/scale = %.3e" % (abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= (2e-6 if fp32 else 1e-12) * scale


# --------------------------------------------------------- Legendre stage (P14)

@pytest.mark.parametrize("lmax,spin,rad", [(128, 0, 10.0), (128, 2, 10.0), (300, 2, 30.0), (200, 3, 5.0)])
def test_legendre_stage_vs_oracle(lmax, spin, rad):
    say("legendre stage", lmax, spin, rad)
    th, ph = syn.uniform_cap(500, rad * DEG, 7400)
    plan = Plan(th, ph, lmax, spin, 1e-10, "fp64")
    a = syn.gaussian_alm(lmax, spin, 7500)
    F = plan.legendre_synth(dev(a)).cpu().numpy()
    L, mmax = plan.info["Lmax"], plan.info["mmax"]
    thj = 2 * math.pi * np.arange(L + 1) / plan.info["n2"] * plan.info["theta_max"] / math.pi
    ref = oracle.ring_coeffs(a, thj, lmax, spin, mmax)
    err = np.max(np.abs(F - ref)) / np.max(np.abs(ref))
    say("  max err = %.3e" % err)
    assert err < 1e-12


@pytest.mark.parametrize("lmax,spin", [(128, 0), (128, 2), (200, 1)])
def test_legendre_stage_transpose(lmax, spin):
    """<L a, F'> = <a, L^T F'>: the Legendre adjoint is the transpose of the synthesis."""
    say("legendre transpose", lmax, spin)
    th, ph = syn.uniform_cap(500, 15 * DEG, 7600)
    plan = Plan(th, ph, lmax, spin, 1e-10, "fp64")
    a = syn.gaussian_alm(lmax, spin, 7700)
    F = plan.legendre_synth(dev(a)).cpu().numpy()
    r = syn.rng(7800)
    Fp = r.standard_normal(F.shape) + 1j * r.standard_normal(F.shape)
    at = plan.legendre_adjoint(dev(Fp)).cpu().numpy()
    lhs = float(np.sum((np.conj(F) * Fp).real))
    rhs = oracle.alm_dot(a, at, lmax)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(F) * np.linalg.norm(Fp)


# -------------------------------------------------------------- edge cases

def test_point_order_invariance():
    lmax, spin = 128, 2
    th, ph = syn.uniform_cap(3000, 12 * DEG, 7900)
    a = dev(syn.gaussian_alm(lmax, spin, 8000))
    perm = syn.rng(8100).permutation(th.shape[0])
    f1 = Plan(th, ph, lmax, spin, 1e-10).synth(a).cpu().numpy()
    f2 = Plan(th[perm], ph[perm], lmax, spin, 1e-10).synth(a).cpu().numpy()
    assert np.max(np.abs(f1[perm] - f2)) <= 1e-13 * np.max(np.abs(f1))


def test_pole_and_wrapped_longitudes():
    """Points exactly at the pole, on theta*, and longitudes outside [0, 2 pi)."""
    lmax, spin, eps = 64, 2, 1e-10
    th = np.array([0.0, 0.0, 1e-9, 0.2, 0.2, 0.1, 0.05])
    ph = np.array([0.0, 3.0, -1.0, 2 * math.pi, -7.5, 100.0, 6.283185307179586])
    a = syn.gaussian_alm(lmax, spin, 8200)
    plan = Plan(th, ph, lmax, spin, eps)
    f = plan.synth(dev(a)).cpu().numpy()
    ref = oracle.synth(a, th, ph, lmax, spin)
    assert rel_l2(f, ref) <= 10 * eps


def test_clustered_points():
    """Many points in one NUFFT cell (an odd count, duplicates included) next to
    a sparse background: the tile layout then has one bank class with
    thousands of slots and classes with none."""
    lmax, spin, eps = 96, 2, 1e-10
    th0, ph0 = syn.uniform_cap(600, 15 * DEG, 8250)
    g = syn.rng(8260)
    th1 = 0.1 + 1e-7 * g.random(2001)
    ph1 = 1.3 + 1e-7 * g.random(2001)
    th1[:300] = th1[0]
    ph1[:300] = ph1[0]
    th, ph = np.concatenate([th0, th1]), np.concatenate([ph0, ph1])
    a = syn.gaussian_alm(lmax, spin, 8270)
    plan = Plan(th, ph, lmax, spin, eps)
    f = plan.synth(dev(a)).cpu().numpy()
    assert rel_l2(f, oracle.synth(a, th, ph, lmax, spin)) <= 10 * eps
    y = syn.gaussian_map(th.shape[0], 8280)
    at = plan.adjoint(dev(y)).cpu().numpy()
    assert alm_rel(at, oracle.adjoint(y, th, ph, lmax, spin), lmax) <= 10 * eps


def test_empty_and_single_point():
    lmax, spin = 32, 0
    a = dev(syn.gaussian_alm(lmax, spin, 8300))
    plan0 = Plan(np.zeros(0), np.zeros(0), lmax, spin, 1e-10)
    assert plan0.synth(a).shape == (0,)
    at = plan0.adjoint(torch.zeros(0, dtype=torch.complex128, device="cuda")).cpu().numpy()
    assert np.all(at == 0)
    th, ph = np.array([0.3]), np.array([1.0])
    plan1 = Plan(th, ph, lmax, spin, 1e-10)
    f = plan1.synth(a).cpu().numpy()
    ref = oracle.synth(a.cpu().numpy(), th, ph, lmax, spin)
    assert rel_l2(f, ref) <= 1e-9


def test_lmax_zero_and_spin_equal_lmax():
    for lmax, spin in ((0, 0), (3, 3)):
        th, ph = syn.uniform_cap(50, 20 * DEG, 8400)
        a = syn.gaussian_alm(lmax, spin, 8500)
        f = Plan(th, ph, lmax, spin, 1e-10).synth(dev(a)).cpu().numpy()
        ref = oracle.synth(a, th, ph, lmax, spin)
        assert rel_l2(f, ref) <= 1e-9


def test_batched_maps_match_single():
    lmax, spin = 96, 2
    th, ph = syn.uniform_cap(2000, 10 * DEG, 8600)
    plan = Plan(th, ph, lmax, spin, 1e-10)
    a = torch.stack([dev(syn.gaussian_alm(lmax, spin, 8700 + i)) for i in range(3)])
    fb = plan.synth(a)
    for i in range(3):
        assert torch.equal(fb[i], plan.synth(a[i]))
    ab = plan.adjoint(fb)
    for i in range(3):
        assert torch.allclose(ab[i], plan.adjoint(fb[i]), rtol=0, atol=1e-12 * float(ab[i].abs().max()))


def test_invalid_points_rejected():
    for th in (np.array([0.1, np.nan]), np.array([0.1, 3.5]), np.array([-0.1, 0.2])):
        with pytest.raises(_lib.PshtError) as e:
            Plan(th, np.zeros(2), 16, 0, 1e-8)
        assert e.value.code == _lib.PSHT_ERR_ARG
    with pytest.raises(_lib.PshtError) as e:
        Plan(np.array([0.1, 0.2]), np.array([0.0, np.inf]), 16, 0, 1e-8)
    assert e.value.code == _lib.PSHT_ERR_ARG


def test_workspace_too_small():
    th, ph = syn.uniform_cap(100, 10 * DEG, 8800)
    plan = Plan(th, ph, 32, 0, 1e-8)
    a = dev(syn.gaussian_alm(32, 0, 8900))
    out = torch.empty(100, dtype=torch.complex128, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    code = _lib.load().psht_synth(plan._h, 1, a.data_ptr(), out.data_ptr(), ws.data_ptr(), 16,
                                   torch.cuda.current_stream().cuda_stream)
    assert code == _lib.PSHT_ERR_WORKSPACE


@pytest.mark.parametrize("lmax, radius_deg", [(64, 20), (1024, 50)])
def test_adjoint_overwrites_output(lmax, radius_deg):
    """The adjoint writes every coefficient whatever its output buffer held (it
    accumulates into the output with atomics after clearing it), for a small
    plan and for one with 2 mmax + 1 >= 1024 Theta-stage columns."""
    say("adjoint into a junk-filled output: lmax %d, cap %d deg" % (lmax, radius_deg))
    th, ph = syn.uniform_cap(20000, radius_deg * DEG, 9100 + lmax)
    plan = Plan(th, ph, lmax, 2, 1e-10)
    assert (2 * plan.info["mmax"] + 1 >= 1024) == (lmax == 1024)
    f = dev(syn.gaussian_map(20000, 9200 + lmax))
    ref = plan.adjoint(f, out=torch.zeros((1, 2, syn.nalm(lmax)), dtype=torch.complex128, device="cuda"))
    junk = torch.full_like(ref, complex(float("nan"), 1e300))
    got = plan.adjoint(f, out=junk)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(torch.view_as_real(got)).all())
    d = (got - ref).abs().max().item() / ref.abs().max().item()
    assert d < 1e-12, d


# ------------------------------------------------ segmented Legendre adjoint

@pytest.mark.parametrize("lmax,radius_deg,spin", [(1024, 5.0, 0), (1024, 5.0, 2), (2048, 2.0, 0), (2048, 5.0, 2),
                                                  (2048, 40.0, 2)])
def test_adjoint_segments_vs_oracle(lmax, radius_deg, spin):
    """Served-disc sizes whose adjoint runs in several degree segments per
    order (started from the plan's stored recurrence states, including states
    still scaled below the double range near the pole) and, for a 40-degree
    cap, several waves per item: every coefficient against the oracle for a
    map on 300 points of the patch, and the output written in full over a
    junk-filled buffer."""
    if radius_deg < 30:
        th_all, ph_all = syn.served_patch(radius_deg)
    else:
        th_all, ph_all = syn.uniform_cap(200000, radius_deg * DEG, 9800)
    plan = Plan(th_all, ph_all, lmax, spin, 1e-10, "fp64")
    info = plan.info
    say("segments: lmax %d disc %g deg spin %d: segment %d, waves %d, rings/lane %d, states %d" % (
        lmax, radius_deg, spin, info["adj_segment"], info["adj_waves"], info["adj_rings_per_lane"],
        info["adj_states"]))
    assert info["adj_segment"] < lmax + 1 - info["mmax"] and info["adj_states"] > 0
    if radius_deg >= 30.0:
        assert info["adj_waves"] > 1
    idx = np.sort(syn.rng(9900 + lmax + spin).choice(th_all.shape[0], 300, replace=False))
    g = np.zeros(th_all.shape[0], dtype=np.complex128)
    g[idx] = syn.gaussian_map(300, 9950 + spin)
    junk = torch.full((2, syn.nalm(lmax)), complex(float("nan"), 1e300), dtype=torch.complex128, device="cuda")
    at = plan.adjoint(dev(g), out=junk).cpu().numpy()
    assert np.all(np.isfinite(at.view(np.float64)))
    ref = oracle.adjoint(g[idx], th_all[idx], ph_all[idx], lmax, spin)
    err = alm_rel(at, ref, lmax)
    say("  rel L2 = %.3e" % err)
    assert err <= 10 * 1e-10
    m, l = syn.alm_m_l(lmax)
    assert np.all(at[:, l < spin] == 0)
    assert np.all(at[:, m == 0].imag == 0)
    assert plan.dropped_points() == 0
    plan.close()


@pytest.mark.parametrize("spin,prec,eps", [(2, "fp64", 1e-10), (0, "fp32", 1e-5)])
def test_adjoint_ring_groups_vs_oracle(spin, prec, eps, monkeypatch):
    """Orders cut into ring groups (forced here at 100 rings; plans with more
    rings than an item holds, full sky above lmax ~ 3000, need them): the
    items add into the cleared output.  Against the oracle, over a
    junk-filled output buffer."""
    monkeypatch.setenv("PSHT_ADJ_GROUP", "100")
    lmax = 512
    th, ph = syn.uniform_cap(30000, 30 * DEG, 9960 + spin)
    plan = Plan(th, ph, lmax, spin, eps, prec)
    assert plan.info["Lmax"] + 1 > 100
    idx = np.sort(syn.rng(9970).choice(th.shape[0], 400, replace=False))
    g = np.zeros(th.shape[0], dtype=np.complex64 if plan.info["map_is_fp32"] else np.complex128)
    g[idx] = syn.gaussian_map(400, 9971 + spin)
    junk = torch.full((2, syn.nalm(lmax)), complex(float("nan"), 1e300), dtype=torch.complex128, device="cuda")
    at = plan.adjoint(dev(g), out=junk).cpu().numpy()
    ref = oracle.adjoint(g[idx].astype(np.complex128), th[idx], ph[idx], lmax, spin)
    err = alm_rel(at, ref, lmax)
    say("ring groups spin %d %s: rel L2 %.3e" % (spin, prec, err))
    assert err <= 10 * eps
    m, l = syn.alm_m_l(lmax)
    assert np.all(at[:, l < spin] == 0) and np.all(at[:, m == 0].imag == 0)
    plan.close()
