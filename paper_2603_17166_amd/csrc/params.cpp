// Host side of a plan: the parameter rules of the partial-sky method, the
// rings and window weights, the per-ring m cut-offs, the NUFFT parameters and
// kernel Fourier tables, and the Legendre recurrence tables.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "leg_common.h"
#include "nufft_index.h"
#include "psht_internal.h"

namespace psht {

typedef long double ld;
static const ld kPiL = 3.141592653589793238462643383279502884L;

// ------------------------------------------------------------ FFT lengths

bool is_smooth(int n, const int *primes, int np) {
    if (n < 1) return false;
    for (int i = 0; i < np; ++i)
        while (n % primes[i] == 0) n /= primes[i];
    return n == 1;
}

bool fft_factor(int n, FftFactors &f) {
    static const int order[] = {4, 2, 3, 5, 7, 11, 13};
    f.n = n;
    f.npass = 0;
    int r = n;
    for (int q : order) {
        while (r % q == 0) {
            if (f.npass >= 16) return false;  // the device code holds at most 16 passes (4 bits each)
            f.radix[f.npass++] = q;
            r /= q;
        }
    }
    return r == 1 && n >= 1;
}

// ------------------------------------------------------------ quadrature

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
static void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
    x.assign(n, 0);
    w.assign(n, 0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        ld z = cosl(kPiL * (i + 0.75L) / (n + 0.5L));
        ld pp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p1 = 1, p2 = 0;
            for (int j = 1; j <= n; ++j) {
                ld p3 = p2;
                p2 = p1;
                p1 = ((2 * j - 1) * z * p2 - (j - 1) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1);
            ld dz = p1 / pp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2 / ((1 - z * z) * pp * pp);
    }
}

struct GL {
    std::vector<ld> x, w;
    explicit GL(int n) { gauss_legendre(n, x, w); }
};

// ------------------------------------------------------------------ window

// w(Theta): 1 on |Theta| <= Theta*, then 1 - CDF of the exponential-of-
// semicircle bell b(u) ~ exp(alpha pi (sqrt(1 - (2u/dT)^2) - 1)), |u| <= dT/2,
// dT = pi - Theta*, i.e. the convolution of a top-hat of support 2 pi - dT
// with the unit-area bell (Sec. II.C, eq. KB and Fig. 4).  The bell CDF is
// integrated after u = (dT/2) sin t, which removes the square-root endpoint.
struct Window {
    ld Theta_star, alpha, dT, h, norm;
    const GL *gl;
    Window(ld Ts, ld a, const GL *g) : Theta_star(Ts), alpha(a), gl(g) {
        dT = kPiL - Ts;
        h = (kPiL + Ts) / 2;
        norm = cdf_t(kPiL / 2);
    }
    // integral of exp(alpha pi (cos t - 1)) cos t over [-pi/2, tv]
    ld cdf_t(ld tv) const {
        ld a = -kPiL / 2, half = (tv - a) / 2, s = 0;
        for (size_t i = 0; i < gl->x.size(); ++i) {
            ld t = a + half * (gl->x[i] + 1);
            s += gl->w[i] * expl(alpha * kPiL * (cosl(t) - 1)) * cosl(t);
        }
        return s * half;
    }
    double operator()(ld Theta) const {
        ld T = fabsl(Theta);
        if (T <= Theta_star) return 1.0;
        if (T >= kPiL) return 0.0;
        ld v = T - h;  // in [-dT/2, dT/2]
        ld arg = 2 * v / dT;
        if (arg > 1) arg = 1;
        if (arg < -1) arg = -1;
        return (double)(1 - cdf_t(asinl(arg)) / norm);
    }
};

// Fourier transform of the ES NUFFT kernel psi(x) = exp(beta (sqrt(1 - z^2) - 1)),
// z = 2x/(W h), scaled so that a grid of spacing h spreading with psi has
// unit gain at frequency 0 after division: psihat(k) = (1/h) int psi(x) cos(k x) dx.
static double es_psihat(ld k, int W, ld beta, ld h, const GL &gl) {
    ld s = 0;
    for (size_t i = 0; i < gl.x.size(); ++i) {
        ld t = gl.x[i] * kPiL / 2;
        ld z = sinl(t);
        s += gl.w[i] * expl(beta * (cosl(t) - 1)) * cosl(t) * cosl(k * W * h * z / 2);
    }
    return (double)(s * (kPiL / 2) * W / 2);
}

// ES kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, in long double.
static ld es_psi(ld z, ld beta) {
    ld t = 1 - z * z;
    if (t < 0) t = 0;
    return expl(beta * (sqrtl(t) - 1));
}

// Polynomial form of the inner kernel taps.  For a stencil origin a0 and
// v = 2 (X - a0) - (W - 1) in [-1, 1], tap i has weight g_i(v) = psi(z) with
// z = (v + W - 1 - 2 i) / W; tap W - 1 - i is g_i(-v).  Each inner tap
// i = 1..(W-1)/2 is interpolated at the P + 1 Chebyshev points of [-1, 1]
// (degree P = es_poly_degree: max(W + 1, 12)), converted to powers of v, and checked against psi on a
// fine grid with the device's evaluation order (even and odd parts by Horner
// in v^2).  The two edge taps reach |z| = 1, where sqrt(1 - z^2) has a
// vertical tangent that polynomials resolve slowly; they keep the formula.
// FP32 plans get the table in float, of degree max(W + 2, 10), checked in
// float arithmetic.
static void es_poly_table(Geometry &g) {
    const int W = g.W, P = es_poly_degree(W, g.fp32), NC = (W - 1) / 2, n = P + 1;
    const ld beta = g.beta;
    g.es_poly.assign((size_t)n * NC, 0.0);
    g.es_poly32.assign(g.fp32 ? (size_t)n * NC : 0, 0.0f);
    double worst = 0;
    for (int c = 0; c < NC; ++c) {
        const int i = c + 1;
        auto f = [&](ld v) { return es_psi((v + W - 1 - 2 * i) / (ld)W, beta); };
        std::vector<ld> fx(n), a(n, 0);
        for (int k = 0; k < n; ++k) fx[k] = f(cosl(kPiL * (k + 0.5L) / n));
        for (int j = 0; j < n; ++j) {
            ld sum = 0;
            for (int k = 0; k < n; ++k) sum += fx[k] * cosl(kPiL * j * (k + 0.5L) / n);
            a[j] = sum * 2 / n;
        }
        a[0] /= 2;
        // sum_j a_j T_j(v) in powers of v (T_{j+1} = 2 v T_j - T_{j-1})
        std::vector<ld> mono(n, 0), tm1(n, 0), t0(n, 0), t1(n, 0);
        t0[0] = 1;
        mono[0] += a[0];
        if (n > 1) {
            t1[1] = 1;
            mono[1] += a[1];
        }
        for (int j = 2; j < n; ++j) {
            std::vector<ld> t2(n, 0);
            for (int q = 0; q + 1 < n; ++q) t2[q + 1] += 2 * t1[q];
            for (int q = 0; q < n; ++q) t2[q] -= t0[q];
            for (int q = 0; q < n; ++q) mono[q] += a[j] * t2[q];
            t0 = t1;
            t1 = t2;
        }
        for (int q = 0; q < n; ++q) g.es_poly[(size_t)q * NC + c] = (double)mono[q];
        const int PE = (P % 2 == 0) ? P : P - 1, PO = (P % 2 == 1) ? P : P - 1;
        if (g.fp32) {
            // check in float, in the device's order
            for (int q = 0; q < n; ++q) g.es_poly32[(size_t)q * NC + c] = (float)mono[q];
            const float *C = g.es_poly32.data();
            for (int t = 0; t <= 400; ++t) {
                const float v = -1.0f + t / 200.0f, v2 = v * v;
                float e = C[(size_t)PE * NC + c];
                for (int q = PE - 2; q >= 0; q -= 2) e = std::fma(e, v2, C[(size_t)q * NC + c]);
                float o = C[(size_t)PO * NC + c];
                for (int q = PO - 2; q >= 1; q -= 2) o = std::fma(o, v2, C[(size_t)q * NC + c]);
                o *= v;
                worst = std::max(worst, (double)fabsl((ld)(e + o) - f(v)));
                worst = std::max(worst, (double)fabsl((ld)(e - o) - f(-v)));
            }
            continue;
        }
        // check in double, in the device's order
        for (int t = 0; t <= 400; ++t) {
            const double v = -1.0 + t / 200.0, v2 = v * v;
            double e = g.es_poly[(size_t)PE * NC + c];
            for (int q = PE - 2; q >= 0; q -= 2) e = std::fma(e, v2, g.es_poly[(size_t)q * NC + c]);
            double o = g.es_poly[(size_t)PO * NC + c];
            for (int q = PO - 2; q >= 1; q -= 2) o = std::fma(o, v2, g.es_poly[(size_t)q * NC + c]);
            o *= v;
            worst = std::max(worst, (double)fabsl((ld)(e + o) - f(v)));
            worst = std::max(worst, (double)fabsl((ld)(e - o) - f(-v)));
        }
    }
    g.es_poly_err = worst;
}

// ---------------------------------------------------- polar cut-off search

// Is max over l <= lmax of max(|lambda+_lm(theta)|, |lambda-_lm(theta)|) >= tau?
// Long double recurrence, seeds in log space (independent of the GPU seeds).
static bool leg_significant(int lmax, int s, int m, ld theta, ld tau) {
    int l0 = std::max(m, s);
    if (l0 > lmax) return false;
    ld ch = cosl(theta / 2), sh = sinl(theta / 2), x = cosl(theta);
    ld lnK = 0.5L * logl((2 * l0 + 1) / (4 * kPiL)) +
             0.5L * (lgammal(2 * l0 + 1) - lgammal(m + s + 1) - lgammal(2 * l0 - m - s + 1));
    int dms = std::abs(m - s);
    auto seed = [&](int pc, int ps) -> ld {
        ld lg = lnK;
        if (pc > 0) {
            if (ch == 0) return 0;
            lg += pc * logl(ch);
        }
        if (ps > 0) {
            if (sh == 0) return 0;
            lg += ps * logl(sh);
        }
        if (lg < -11000) return 0;
        return expl(lg);
    };
    ld lp = seed(dms, m + s), lm = seed(m + s, dms);
    if (fabsl(lp) >= tau || fabsl(lm) >= tau) return true;
    if (lp == 0 && lm == 0 && sh != 0) return false;
    ld lpp = 0, lmp = 0;
    ld M = m, S = s;
    for (int l = l0; l < lmax; ++l) {
        ld L = l;
        ld D = sqrtl(((L + 1) * (L + 1) - M * M) * ((L + 1) * (L + 1) - S * S));
        ld a = sqrtl((2 * L + 3) * (2 * L + 1)) * (L + 1) / D;
        ld b = (m * s == 0) ? 0 : a * M * S / (L * (L + 1));
        ld c = (l == l0) ? 0 : sqrtl((2 * L + 3) / (2 * L - 1)) * (L + 1) * sqrtl((L * L - M * M) * (L * L - S * S)) / (L * D);
        ld np = (a * x + b) * lp - c * lpp;
        ld nm = (a * x - b) * lm - c * lmp;
        lpp = lp;
        lp = np;
        lmp = lm;
        lm = nm;
        if (fabsl(lp) >= tau || fabsl(lm) >= tau) return true;
    }
    return false;
}

// Largest m with a significant ring contribution (polar optimization: orders
// well above lmax sin(theta) are irrelevant on the ring, Sec. II.A).
static int ring_cutoff(int lmax, int s, ld theta, ld tau) {
    if (theta == 0) return std::min(s, lmax);
    int lo = (int)floorl(lmax * sinl(theta));
    lo = std::max(0, std::min(lo, lmax));
    while (lo > 0 && !leg_significant(lmax, s, lo, theta, tau)) lo /= 2;
    if (!leg_significant(lmax, s, lo, theta, tau)) return std::min(s, lmax);
    if (leg_significant(lmax, s, lmax, theta, tau)) return lmax;
    int hi = lmax;  // lo significant, hi not
    while (hi - lo > 1) {
        int mid = lo + (hi - lo) / 2;
        if (leg_significant(lmax, s, mid, theta, tau))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- geometry

static int es_width(double eps) {
    int W = (int)std::ceil(std::log10(1.0 / eps)) + 1;
    return std::max(2, std::min(16, W));
}

static double es_beta(int W) {
    double r = 2.30;
    if (W == 2) r = 2.20;
    if (W == 3) r = 2.26;
    if (W == 4) r = 2.38;
    return r * W;
}

bool geometry_compute(Geometry &g, int lmax, int spin, double theta_star, double theta_min, double eps,
                      int precision, bool with_grid, Error &err, bool with_cutoffs, const psht_plan_options *opts) {
    static const int odd_primes[] = {3, 5, 7, 11, 13};
    static const int grid_primes[] = {2, 3, 5, 7};
    if (lmax < 0 || spin < 0 || spin > lmax) {
        err = {PSHT_ERR_ARG, "need lmax >= 0 and 0 <= spin <= lmax"};
        return false;
    }
    if (!(eps >= 1e-14 && eps <= 1e-2)) {
        err = {PSHT_ERR_ARG, "epsilon must lie in [1e-14, 1e-2]"};
        return false;
    }
    if (precision < PSHT_PREC_AUTO || precision > PSHT_PREC_FP64) {
        err = {PSHT_ERR_ARG, "unknown precision"};
        return false;
    }
    if (!(theta_star >= 0 && theta_star <= M_PI) || !(theta_min >= 0 && theta_min <= theta_star)) {
        err = {PSHT_ERR_ARG, "theta range must lie in [0, pi]"};
        return false;
    }
    g = Geometry();
    g.lmax = lmax;
    g.spin = spin;
    g.eps = eps;
    g.fp32 = (precision == PSHT_PREC_FP32) || (precision == PSHT_PREC_AUTO && eps >= 1e-6);
    g.theta_star = theta_star;
    g.theta_min = theta_min;

    // Sec. II.C summary: alpha = |ln eps| / pi, eps_apo = sqrt(2 |ln eps| / (theta* lmax));
    // Sec. II step 2: theta_max = theta* (1 + eps_apo); eq. Lmax2: Lmax = lmax theta*/pi (1 + eps_apo)^2.
    double ln_eps = std::fabs(std::log(eps));
    double ts = std::max(theta_star, 1e-9);
    g.alpha = ln_eps / M_PI;
    double Lf = 0;
    if (lmax > 0) {
        g.eps_apo = std::sqrt(2.0 * ln_eps / (ts * lmax));
        g.theta_max = ts * (1.0 + g.eps_apo);
        Lf = lmax * ts / M_PI * (1.0 + g.eps_apo) * (1.0 + g.eps_apo);
    }
    if (opts && (opts->full_sky != 0 && opts->full_sky != 1)) {
        err = {PSHT_ERR_ARG, "full_sky must be 0 or 1"};
        return false;
    }
    if (opts && opts->window != PSHT_WINDOW_ES) {
        err = {PSHT_ERR_UNSUPPORTED, "window bell not available"};
        return false;
    }
    if (opts && opts->cl) {
        err = {PSHT_ERR_UNSUPPORTED, "spectrum-tuned Lmax not available"};
        return false;
    }
    g.full_sky = (opts && opts->full_sky) || (lmax == 0) || !(g.theta_max < M_PI) || !(Lf < lmax);
    int L;
    if (g.full_sky) {
        // The patch is too large to gain anything: evaluate the map itself on the
        // doubled Fourier sphere (Sec. I.B), exact for Lmax >= lmax.
        g.theta_max = M_PI;
        g.eps_apo = 0.0;
        L = std::max(lmax, 1);
    } else {
        L = std::max(1, (int)std::ceil(Lf - 1e-9));
    }
    while (!is_smooth(2 * L + 1, odd_primes, 5)) ++L;
    g.Lmax = L;
    g.N2 = 2 * L + 1;
    g.nring = L + 1;

    // Rings Theta_j = 2 pi j / N2 (j = 0..Lmax), theta_j = Theta_j theta_max / pi.
    GL gl_win(160);
    ld Theta_star = g.full_sky ? kPiL : kPiL * (ld)ts / (ld)g.theta_max;
    Window win(Theta_star, (ld)g.alpha, &gl_win);
    g.ring_theta.resize(g.nring);
    g.ring_w.resize(g.nring);
    for (int j = 0; j < g.nring; ++j) {
        ld Th = 2 * kPiL * j / g.N2;
        g.ring_theta[j] = (double)(Th * (ld)g.theta_max / kPiL);
        g.ring_w[j] = g.full_sky ? 1.0 : win(Th);
    }

    // Per-ring m cut-offs (without them every ring keeps all m <= lmax).
    g.ring_mmax.assign(g.nring, lmax);
    if (with_cutoffs) {
        ld tau = (ld)(kPolarTauRel * eps);
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                for (int j = (int)t; j < g.nring; j += (int)nt)
                    g.ring_mmax[j] = ring_cutoff(lmax, spin, (ld)g.ring_theta[j], tau);
            });
        for (auto &x : th) x.join();
    }
    g.mmax = 0;
    double triples = 0;
    for (int j = 0; j < g.nring; ++j) {
        g.mmax = std::max(g.mmax, (int)g.ring_mmax[j]);
        for (int m = 0; m <= g.ring_mmax[j]; ++m) triples += lmax + 1 - std::max(m, spin);
    }
    g.legendre_triples = triples;
    g.predicted_speedup = g.full_sky ? 1.0 : 1.0 / ((1.0 + g.eps_apo) * (1.0 - std::cos(g.theta_max)));

    // NUFFT (ES kernel, upsampling 2): W = ceil(log10(1/eps)) + 1, beta = 2.30 W.
    g.W = es_width(eps);
    g.beta = es_beta(g.W);
    g.sigma = 2.0;
    es_poly_table(g);
    if (g.es_poly_err > std::max(1e-3 * eps, g.fp32 ? 2e-7 : 1e-14)) {
        err = {PSHT_ERR_UNSUPPORTED, "kernel polynomial table not accurate enough"};
        return false;
    }
    g.Ntheta = 2 * g.N2;
    while (g.Ntheta < 2 * g.W + 4) g.Ntheta += 2 * g.N2;
    int np = std::max(2 * (2 * g.mmax + 1), 2 * g.W + 4);
    if (np % 2) ++np;
    // Rows longer than the 2560-point tier run as two half-length transforms in
    // workgroups of their own (twice the transforms in flight per CU), rows
    // longer than twice the LDS limit as four (Nphi then a multiple of 4).
    g.phi_parts = np > 2 * kFftMaxLds64 ? 4 : (np > 2560 ? 2 : 1);
    if (const char *e = getenv("PSHT_PHI_PARTS")) {  // tests and tuning runs: 1, 2 or 4 parts
        const int v = atoi(e);
        if ((v == 1 && np <= kFftMaxLds64) || v == 2 || v == 4) g.phi_parts = v;
    }
    while (!is_smooth(np, grid_primes, 4) || np % g.phi_parts) np += 2;
    g.Nphi = np;
    g.sx = g.Ntheta / (2.0 * g.theta_max);
    g.sy = g.Nphi / (2.0 * M_PI);
    double hw = 0.5 * g.W;
    g.row_lo = (int)std::ceil(theta_min * g.sx - hw) - 1;
    int row_hi = (int)std::ceil(theta_star * g.sx - hw) + g.W - 1 + 1;
    g.rows_used = row_hi - g.row_lo + 1;
    if (g.rows_used > g.Ntheta) {
        err = {PSHT_ERR_UNSUPPORTED, "points span more Theta-grid rows than the grid holds"};
        return false;
    }
    if (with_grid) {
        GL gl(128);
        ld hT = 2 * kPiL / g.Ntheta, hP = 2 * kPiL / g.Nphi;
        g.psihat_theta.resize(g.Lmax + 1);
        for (int n = 0; n <= g.Lmax; ++n) g.psihat_theta[n] = es_psihat(n, g.W, g.beta, hT, gl);
        g.psihat_phi.resize(g.mmax + 1);
        for (int m = 0; m <= g.mmax; ++m) g.psihat_phi[m] = es_psihat(m, g.W, g.beta, hP, gl);
    }
    return true;
}

// ---------------------------------------------------------- Legendre tables

LegTable::~LegTable() {
    if (d_coef) (void)hipFree(d_coef);
    if (d_kmant) (void)hipFree(d_kmant);
    if (d_kexp) (void)hipFree(d_kexp);
}

// Wigner-d recurrence coefficients (the three-term recurrence in l for
// d^l_{m,-/+s}) with the normalization sqrt((2l+1)/4pi) folded in, rewritten
// so that the previous term has coefficient one:
//   lambda_{l+1} = (a_l x + b_l) lambda_l - c_l lambda_{l-1},  b = +/- a m s/(l(l+1)),
//   lambda_l = P_l mu_l,  P_{l0} = P_{l0+1} = 1,  P_{l+1} = c_l P_{l-1},
//   mu_{l+1} = (A_l x +/- B_l) mu_l - mu_{l-1},  A = a P_l/P_{l+1},  B = b P_l/P_{l+1}.
// With y = 1 - x = 2 sin^2(theta/2) the step coefficient is (A +/- B) - A y:
// near the pole x = cos(theta) keeps only an absolute 1e-16 of the ring
// position, while y keeps it to full relative precision.  Stored per (l, m):
// {-A, A + B, A - B, P}.  Products are formed in long double.
void leg_table_host(LegTable &t, int lmax, int s) {
    int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    t.lmax = lmax;
    t.spin = s;
    t.h_coef.assign(4 * nalm, 0.0);
    t.h_kmant.assign(lmax + 1, 0.0);
    t.h_kexp.assign(lmax + 1, 0);
    std::vector<ld> a(lmax + 2), b(lmax + 2), c(lmax + 2), P(lmax + 2);
    ld S = s;
    ld binom_mant = 0.5L;  // C(2m, m+s) = binom_mant * 2^binom_exp for the current m >= s
    int binom_exp = 1;
    for (int m = 0; m <= lmax; ++m) {
        int l0 = std::max(m, s);
        if (m > s) {
            int e;
            binom_mant = frexpl(binom_mant * ((ld)(2 * m) * (2 * m - 1) / ((ld)(m + s) * (m - s))), &e);
            binom_exp += e;
        }
        if (l0 > lmax) continue;
        ld M = m;
        for (int l = l0; l <= lmax; ++l) {
            ld L = l;
            ld D = sqrtl(((L + 1) * (L + 1) - M * M) * ((L + 1) * (L + 1) - S * S));
            a[l] = sqrtl((2 * L + 3) * (2 * L + 1)) * (L + 1) / D;
            b[l] = (m * s == 0) ? 0 : a[l] * M * S / (L * (L + 1));
            c[l] = (l == l0) ? 0 : sqrtl((2 * L + 3) / (2 * L - 1)) * (L + 1) * sqrtl((L * L - M * M) * (L * L - S * S)) / (L * D);
        }
        P[l0] = 1;
        if (l0 + 1 <= lmax) P[l0 + 1] = 1;
        for (int l = l0 + 1; l < lmax; ++l) P[l + 1] = c[l] * P[l - 1];
        int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        for (int l = l0; l <= lmax; ++l) {
            double *e = &t.h_coef[4 * (base + l)];
            if (l < lmax) {
                ld A = a[l] * P[l] / P[l + 1], B = b[l] * P[l] / P[l + 1];
                e[0] = (double)(-A);
                e[1] = (double)(A + B);
                e[2] = (double)(A - B);
            }
            e[3] = (double)P[l];
        }
        // K_m = N_l0 sqrt(C(2 l0, m + s))
        int e2;
        ld mant;
        if (m >= s) {
            mant = binom_mant;
            e2 = binom_exp;
        } else {
            mant = frexpl(expl(lgammal(2 * s + 1) - lgammal(s + m + 1) - lgammal(s - m + 1)), &e2);
        }
        if (e2 & 1) {
            mant *= 2;
            e2 -= 1;
        }
        ld K = sqrtl((2 * l0 + 1) / (4 * kPiL)) * sqrtl(mant);
        int e3;
        ld km = frexpl(K, &e3);
        t.h_kmant[m] = (double)km;
        t.h_kexp[m] = e3 + e2 / 2;
    }
}

std::shared_ptr<LegTable> leg_table_get(int lmax, int spin, Error &err) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::weak_ptr<LegTable>> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(lmax * 64 + dev, spin);
    auto it = cache.find(key);
    if (it != cache.end()) {
        auto sp = it->second.lock();
        if (sp) return sp;
    }
    auto t = std::make_shared<LegTable>();
    leg_table_host(*t, lmax, spin);
    size_t nc = t->h_coef.size() * sizeof(double);
    if (hipMalloc(&t->d_coef, nc) != hipSuccess || hipMalloc(&t->d_kmant, (lmax + 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&t->d_kexp, (lmax + 1) * sizeof(int32_t)) != hipSuccess) {
        err = {PSHT_ERR_NOMEM, "device allocation of the Legendre table failed"};
        return nullptr;
    }
    if (hipMemcpy(t->d_coef, t->h_coef.data(), nc, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_kmant, t->h_kmant.data(), (lmax + 1) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_kexp, t->h_kexp.data(), (lmax + 1) * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        err = {PSHT_ERR_DEVICE, "upload of the Legendre table failed"};
        return nullptr;
    }
    t->bytes = nc + (lmax + 1) * (sizeof(double) + sizeof(int32_t));
    t->h_coef.clear();
    t->h_coef.shrink_to_fit();
    cache[key] = t;
    return t;
}

}  // namespace psht
