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

// Bells of the apodization window (Sec. II.C), as functions of x in [-1, 1]
// (x = 2u / dT across the bell's support dT):
//   ES   (eq. KB):     exp(alpha pi (sqrt(1 - x^2) - 1));
//   KB   (Kaiser-Bessel): I0(alpha pi sqrt(1 - x^2)) e^{-alpha pi}, whose Fourier
//        transform over the support is the closed form printed with eq. KB;
//   PSWF (Slepian): the order-0 prolate spheroidal wave function psi_0(c, x)
//        with bandwidth c = alpha pi, the function of support [-1, 1] whose
//        Fourier transform is most concentrated on |k| <= alpha.
// All three are even and positive on (-1, 1); the window uses their unit-area
// cumulative integral.

// I0(z), z >= 0, by its power series sum_k (z^2/4)^k / (k!)^2 (all terms
// positive; z <= 40 here, so about 60 terms reach long-double precision).
static ld bessel_i0(ld z) {
    const ld q = z * z / 4;
    ld term = 1, sum = 1;
    for (int k = 1; k < 400; ++k) {
        term *= q / ((ld)k * k);
        sum += term;
        if (term < sum * 1e-21L) break;
    }
    return sum;
}

// psi_0(c, x) = sum_{k even} b_k Pn_k(x), Pn_k = sqrt(k + 1/2) P_k, from the
// Legendre-basis form of the prolate differential operator
//   L psi = -((1 - x^2) psi')' + c^2 x^2 psi = chi psi:
// in the orthonormal basis Pn_k it is symmetric tridiagonal over k of one
// parity, with diagonal k(k+1) + c^2 (2k^2 + 2k - 1) / ((2k - 1)(2k + 3)) and
// off-diagonal c^2 (k+1)(k+2) / ((2k+3) sqrt((2k+1)(2k+5))) between k and
// k + 2 (from x^2 P_k in P_{k-2}, P_k, P_{k+2}).  psi_0 belongs to the smallest
// eigenvalue chi_0 in (0, c^2/3]: chi_0 by Sturm-count bisection, the vector
// by inverse iteration at a shift just below chi_0.  Coefficients fall off
// faster than geometrically for k beyond c, so k <= 2 c + 80 is ample.
static std::vector<ld> pswf0_coeffs(ld c) {
    const int n = (int)(c + 41);  // k = 0, 2, ..., 2 (n - 1)
    std::vector<ld> d(n), e(n, 0);
    const ld c2 = c * c;
    for (int i = 0; i < n; ++i) {
        const ld k = 2 * i;
        d[i] = k * (k + 1) + c2 * (2 * k * k + 2 * k - 1) / ((2 * k - 1) * (2 * k + 3));
        e[i] = c2 * (k + 1) * (k + 2) / ((2 * k + 3) * sqrtl((2 * k + 1) * (2 * k + 5)));
    }
    auto below = [&](ld lam) {  // eigenvalues < lam = negative pivots of A - lam I
        int cnt = 0;
        ld q = d[0] - lam;
        if (q < 0) ++cnt;
        for (int i = 1; i < n; ++i) {
            if (q == 0) q = 1e-300L;
            q = d[i] - lam - e[i - 1] * e[i - 1] / q;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    ld lo = 0, hi = c2 / 3 + 1;
    for (int it = 0; it < 200; ++it) {
        const ld mid = (lo + hi) / 2;
        if (below(mid) >= 1) hi = mid;
        else lo = mid;
    }
    const ld shift = lo - 1e-9L * (1 + lo);
    std::vector<ld> b(n, 1), cp(n), dp(n);
    for (int it = 0; it < 4; ++it) {  // solve (A - shift) y = b by the Thomas algorithm
        ld den = d[0] - shift;
        cp[0] = e[0] / den;
        dp[0] = b[0] / den;
        for (int i = 1; i < n; ++i) {
            den = d[i] - shift - e[i - 1] * cp[i - 1];
            cp[i] = e[i] / den;
            dp[i] = (b[i] - e[i - 1] * dp[i - 1]) / den;
        }
        b[n - 1] = dp[n - 1];
        for (int i = n - 2; i >= 0; --i) b[i] = dp[i] - cp[i] * b[i + 1];
        ld nrm = 0;
        for (ld v : b) nrm += v * v;
        nrm = sqrtl(nrm);
        for (ld &v : b) v /= nrm;
    }
    // sign: psi_0(0) > 0, with P_k(0) = (-1)^(k/2) (k-1)!!/k!!
    ld p0 = 0, pk = 1;
    for (int i = 0; i < n; ++i) {
        const ld k = 2 * i;
        if (i > 0) pk *= -(k - 1) / k;
        p0 += b[i] * sqrtl(k + 0.5L) * pk;
    }
    if (p0 < 0)
        for (ld &v : b) v = -v;
    return b;
}

// w(Theta): 1 on |Theta| <= Theta*, 0 at Theta = pi, and in between 1 - the
// unit-area cumulative integral of the bell over a support dT = pi - Theta*
// centred at h = (pi + Theta*)/2: the convolution of a top-hat of support
// 2 pi - dT with the bell (Sec. II.C, Fig. 4).  ES and KB cumulative integrals
// are taken by Gauss-Legendre quadrature after x = sin t (which removes the
// square-root endpoint); the PSWF one term by term from
// int_{-1}^{x} P_k = (P_{k+1}(x) - P_{k-1}(x)) / (2k + 1), k >= 1.
struct Window {
    ld Theta_star, alpha, dT, h, norm;
    int kind;
    const GL *gl;
    std::vector<ld> pc;
    Window(ld Ts, ld a, const GL *g, int bell = PSHT_WINDOW_ES) : Theta_star(Ts), alpha(a), kind(bell), gl(g) {
        dT = kPiL - Ts;
        h = (kPiL + Ts) / 2;
        if (kind == PSHT_WINDOW_PSWF) pc = pswf0_coeffs(alpha * kPiL);
        norm = cdf(1);
    }
    ld bell_t(ld t) const {  // bell at x = sin t, times dx/dt = cos t
        const ld ct = cosl(t);
        if (kind == PSHT_WINDOW_KB) return bessel_i0(alpha * kPiL * ct) * expl(-alpha * kPiL) * ct;
        return expl(alpha * kPiL * (ct - 1)) * ct;
    }
    // integral of the bell over [-1, x]
    ld cdf(ld x) const {
        if (x > 1) x = 1;
        if (x < -1) x = -1;
        if (kind == PSHT_WINDOW_PSWF) {
            ld pm = 1, p = x, s = pc[0] * sqrtl(0.5L) * (x + 1);  // P_0, P_1
            for (int k = 1; k < 2 * (int)pc.size(); ++k) {
                const ld pn = ((2 * k + 1) * x * p - k * pm) / (k + 1);  // P_{k+1}
                if ((k & 1) == 0) s += pc[k / 2] * sqrtl(k + 0.5L) * (pn - pm) / (2 * k + 1);
                pm = p;
                p = pn;
            }
            return s;
        }
        const ld a = -kPiL / 2, half = (asinl(x) - a) / 2;
        ld s = 0;
        for (size_t i = 0; i < gl->x.size(); ++i) s += gl->w[i] * bell_t(a + half * (gl->x[i] + 1));
        return s * half;
    }
    double operator()(ld Theta) const {
        ld T = fabsl(Theta);
        if (T <= Theta_star) return 1.0;
        if (T >= kPiL) return 0.0;
        return (double)(1 - cdf(2 * (T - h) / dT) / norm);
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

// Factors of the recurrence coefficients that depend on l alone, shared by
// every order and ring of a cut-off search: (l+1) sqrt((2l+3)(2l+1)),
// (l+1) sqrt((2l+3)/(2l-1)) / l and 1 / (l(l+1)).
struct DegreeRoots {
    std::vector<ld> r1, r2, il;
    explicit DegreeRoots(int lmax) : r1(lmax + 1), r2(lmax + 1), il(lmax + 1) {
        for (int l = 0; l <= lmax; ++l) {
            const ld L = l;
            r1[l] = (L + 1) * sqrtl((2 * L + 3) * (2 * L + 1));
            r2[l] = l > 0 ? (L + 1) * sqrtl((2 * L + 3) / (2 * L - 1)) / L : 0;
            il[l] = l > 0 ? 1 / (L * (L + 1)) : 0;
        }
    }
};

// Is max over l <= lmax of max(|lambda+_lm(theta)|, |lambda-_lm(theta)|) >= tau?
// Long double recurrence, seeds in log space (independent of the GPU seeds).
// The root sqrt((l^2 - m^2)(l^2 - s^2)) of a step's c is the previous step's
// D, so each step takes one square root and one division.
static bool leg_significant(int lmax, int s, int m, ld theta, ld tau, const DegreeRoots &R) {
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
    ld lpp = 0, lmp = 0, Dprev = 0;
    const ld M = m, S = s, MS = M * S;
    for (int l = l0; l < lmax; ++l) {
        const ld L = l;
        const ld D = sqrtl(((L + 1) * (L + 1) - M * M) * ((L + 1) * (L + 1) - S * S));
        const ld iD = 1 / D;
        const ld a = R.r1[l] * iD;
        const ld b = (m * s == 0) ? 0 : a * MS * R.il[l];
        const ld c = (l == l0) ? 0 : R.r2[l] * Dprev * iD;
        Dprev = D;
        const ld np = (a * x + b) * lp - c * lpp;
        const ld nm = (a * x - b) * lm - c * lmp;
        lpp = lp;
        lp = np;
        lmp = lm;
        lm = nm;
        if (fabsl(lp) >= tau || fabsl(lm) >= tau) return true;
    }
    return false;
}

// Largest m with a significant ring contribution (polar optimization: orders
// well above lmax sin(theta) are irrelevant on the ring, Sec. II.A), searched
// from a guess: the neighbouring ring's cut-off, shifted by the change of
// lmax sin(theta), lies within a few orders of the boundary, so a handful of
// tests replace a bisection over [lmax sin(theta), lmax].
static int ring_cutoff(int lmax, int s, ld theta, ld tau, const DegreeRoots &R, int guess) {
    if (theta == 0) return std::min(s, lmax);
    auto sig = [&](int m) { return leg_significant(lmax, s, m, theta, tau, R); };
    // bracket the boundary by steps doubling away from the guess: lo significant
    // (or -1), hi not (or lmax + 1); then bisect
    int lo, hi, g = std::max(0, std::min(guess, lmax));
    if (sig(g)) {
        lo = g;
        for (int step = 1;; step *= 2) {
            const int t = lo + step;
            if (t > lmax) {
                hi = lmax + 1;
                break;
            }
            if (!sig(t)) {
                hi = t;
                break;
            }
            lo = t;
        }
    } else {
        hi = g;
        for (int step = 1;; step *= 2) {
            const int t = hi - step;
            if (t < 0) {
                lo = -1;
                break;
            }
            if (sig(t)) {
                lo = t;
                break;
            }
            hi = t;
        }
    }
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        if (sig(mid))
            lo = mid;
        else
            hi = mid;
    }
    return lo < 0 ? std::min(s, lmax) : lo;
}

// ------------------------------------------- error predictor (Sec. II.D)

// Great-circle spectrum of an isotropic field with power spectrum C_l
// (eq. cm, and eq. cms for spin s with C_l = C^E_l + C^B_l):
//   c_m = sum_{l >= max(|m|, s)} C_l (2l+1)/2 |d^l_{m,-s}(pi/2)|^2,  m = -lmax..lmax,
// with d^l_{-m,-s} = d^l_{m,s} for the negative orders.  (2l+1)/2 d^2 = 2 pi lambda^2
// for the normalized lambda = sqrt((2l+1)/4 pi) d, computed by the three-term
// recurrence in l at theta = pi/2 (cos theta = 0) from the single-term seed,
// in long double.  cm[m + lmax].
void great_circle_spectrum(int lmax, int s, const double *cl, std::vector<double> &cm) {
    cm.assign(2 * (size_t)lmax + 1, 0.0);
    const ld S = s, half = 0.5L;
    for (int m = 0; m <= lmax; ++m) {
        const int l0 = std::max(m, s);
        if (l0 > lmax) continue;
        const ld M = m;
        const ld lnK = 0.5L * logl((2 * l0 + 1) / (4 * kPiL)) +
                       0.5L * (lgammal(2 * l0 + 1) - lgammal(m + s + 1) - lgammal(2 * l0 - m - s + 1));
        // cos(pi/4) = sin(pi/4) = 2^-1/2: both seeds are K 2^{-(|m-s| + m + s)/2}
        const ld seed = expl(lnK - half * (std::abs(m - s) + m + s) * logl(2.0L));
        ld lp = seed, lm = seed, lpp = 0, lmp = 0;
        ld sp = 0, sm = 0;
        for (int l = l0; l <= lmax; ++l) {
            sp += (ld)cl[l] * lp * lp;
            sm += (ld)cl[l] * lm * lm;
            if (l == lmax) break;
            const ld L = l;
            const ld D = sqrtl(((L + 1) * (L + 1) - M * M) * ((L + 1) * (L + 1) - S * S));
            const ld a = sqrtl((2 * L + 3) * (2 * L + 1)) * (L + 1) / D;
            const ld b = (m * s == 0) ? 0 : a * M * S / (L * (L + 1));
            const ld c = (l == l0) ? 0
                                   : sqrtl((2 * L + 3) / (2 * L - 1)) * (L + 1) *
                                         sqrtl((L * L - M * M) * (L * L - S * S)) / (L * D);
            const ld np = b * lp - c * lpp, nm = -b * lm - c * lmp;  // (a x +/- b), x = cos(pi/2) = 0
            lpp = lp;
            lp = np;
            lmp = lm;
            lm = nm;
        }
        cm[lmax + m] = (double)(2 * kPiL * sp);
        if (m > 0) cm[lmax - m] = (double)(2 * kPiL * sm);
    }
}

// Predicted relative error of the weighted, band-limited map (Sec. II.D): for
// the rings Theta_j = 2 pi j / N2, j = -L..L, of this L, with weights w_j and
// theta_j = Theta_j theta_max / pi, the error on the wave e^{i m theta} is
//   sigma_m(theta) = | sum_j w_j D_j(Theta) e^{i m theta_j} - e^{i m theta} |
// (eq. s2m, D the Dirichlet kernel of eq. Dnz), and a field with great-circle
// spectrum c_m has sigma^2(theta) = (1/2pi) sum_m c_m sigma_m^2(theta)
// (eq. st).  Returned: max over theta <= theta* of sigma(theta) / <|f|^2>^(1/2),
// <|f|^2> = (1/2pi) sum_m c_m.  theta is sampled on 33 equidistant points of
// [0, theta*] and half-way between consecutive rings in the last fifth of the
// cap (where the error peaks, between the nodes); the orders with a stride of
// at most lmax / 512 (each sampled order standing for `stride` orders).
template <typename WinFn>
double predicted_error(int lmax, double theta_star, double theta_max, int L, const WinFn &win,
                       const std::vector<double> &cm) {
    const int N2 = 2 * L + 1;
    const double h = 2.0 * theta_max / N2;  // ring spacing in theta
    std::vector<double> thj(N2), wj(N2), Thj(N2);
    for (int k = 0; k < N2; ++k) {
        const int j = k - L;
        Thj[k] = 2.0 * M_PI * j / N2;
        thj[k] = j * h;
        wj[k] = win(std::fabs(Thj[k]));
    }
    std::vector<double> ths;
    for (int k = 0; k <= 32; ++k) ths.push_back(theta_star * k / 32.0);
    for (int j = 0; j < L; ++j) {
        const double mid = (j + 0.5) * h;
        if (mid >= 0.8 * theta_star && mid <= theta_star) ths.push_back(mid);
    }
    const int stride = std::max(1, lmax / 512);
    std::vector<int> ms;
    for (int m = -lmax; m <= lmax; m += stride) ms.push_back(m);
    if (ms.back() != lmax) ms.push_back(lmax);
    double total = 0.0;
    for (int m : ms) total += cm[m + lmax];
    if (!(total > 0)) return 0.0;
    std::vector<double> worst(ths.size(), 0.0);
    auto eval = [&](size_t it) {
        const double th = ths[it], Th = th * M_PI / theta_max;
        std::vector<double> ar(N2);
        for (int k = 0; k < N2; ++k) {
            const double d = Th - Thj[k], sd = std::sin(0.5 * d);
            const double D = std::fabs(sd) < 1e-15 ? 1.0 : std::sin(0.5 * N2 * d) / (N2 * sd);
            ar[k] = wj[k] * D;
        }
        double acc = 0.0;
        for (int m : ms) {
            // sum_k a_k e^{i m theta_k}, theta_k = (k - L) h: phasor rotated step by step
            const double cr = std::cos(m * h), ci = std::sin(m * h);
            double pr = std::cos(-m * h * L), pi = std::sin(-m * h * L);
            double sr = 0, si = 0;
            for (int k = 0; k < N2; ++k) {
                sr += ar[k] * pr;
                si += ar[k] * pi;
                const double t = pr * cr - pi * ci;
                pi = pr * ci + pi * cr;
                pr = t;
            }
            const double er = sr - std::cos(m * th), ei = si - std::sin(m * th);
            acc += cm[m + lmax] * (er * er + ei * ei);
        }
        worst[it] = acc;
    };
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t)
        pool.emplace_back([&, t]() {
            for (size_t it = t; it < ths.size(); it += nt) eval(it);
        });
    for (auto &x : pool) x.join();
    double mx = 0.0;
    for (double v : worst) mx = std::max(mx, v);
    return std::sqrt(mx / total);
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
    if (opts && (opts->window < PSHT_WINDOW_ES || opts->window > PSHT_WINDOW_PSWF)) {
        err = {PSHT_ERR_ARG, "unknown window bell"};
        return false;
    }
    if (opts && (opts->lmax_rule != PSHT_LMAX_RULE_BAND && opts->lmax_rule != PSHT_LMAX_RULE_COST)) {
        err = {PSHT_ERR_ARG, "unknown Lmax rule"};
        return false;
    }
    g.window = opts ? opts->window : PSHT_WINDOW_ES;
    // Sec. II.C, footnote to eq. Lmax2: instead of the smallest Lmax, the
    // apodization length that minimizes the Legendre work with polar
    // optimization.  With Delta l = 2 alpha the band estimate of eq. Lmax for a
    // fractional apodization length x is Lmax(x) = lmax theta*/pi (1 + x)(1 + c/x),
    // c = 2 |ln eps| / (theta* lmax) (its minimum x = sqrt(c) is eq. Lmax2), and
    // the work of the Lmax + 1 rings is sum_j m_j (lmax + 1 - m_j / 2) with
    // m_j = min(lmax, lmax sin theta_j) (the pairs (m, l), m <= m_j, l >= m).
    // x is scanned over [sqrt(c)/4, 2 sqrt(c)] with Lmax rounded to a smooth N2.
    if (opts && opts->lmax_rule == PSHT_LMAX_RULE_COST && lmax > 0 && Lf < lmax && g.theta_max < M_PI) {
        const double c = 2.0 * ln_eps / (ts * lmax), x0 = std::sqrt(c);
        double best = HUGE_VAL, bx = g.eps_apo;
        for (int i = 0; i <= 400; ++i) {
            const double x = x0 * (0.25 + 1.75 * i / 400.0), tm = ts * (1 + x);
            if (!(tm < M_PI)) break;
            int Lc = std::max(1, (int)std::ceil(lmax * ts / M_PI * (1 + x) * (1 + c / x) - 1e-9));
            while (!is_smooth(2 * Lc + 1, odd_primes, 5)) ++Lc;
            double work = 0;
            for (int j = 0; j <= Lc; ++j) {
                const double mj = std::min((double)lmax, lmax * std::sin(2.0 * M_PI * j / (2 * Lc + 1) * tm / M_PI));
                work += mj * (lmax + 1 - 0.5 * mj);
            }
            if (work < best) {
                best = work;
                bx = x;
            }
        }
        g.eps_apo = bx;
        g.theta_max = ts * (1.0 + bx);
        Lf = lmax * ts / M_PI * (1.0 + bx) * (1.0 + c / bx);
    }
    if (opts && opts->cl && opts->cl_lmax < lmax) {
        err = {PSHT_ERR_ARG, "cl must hold C_l for l = 0..lmax (cl_lmax >= lmax)"};
        return false;
    }
    if (opts && opts->cl)
        for (int l = 0; l <= lmax; ++l)
            if (!(opts->cl[l] >= 0.0) || !std::isfinite(opts->cl[l])) {
                err = {PSHT_ERR_ARG, "cl must be finite and non-negative"};
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
    g.Lmax_rule = L;

    // Rings Theta_j = 2 pi j / N2 (j = 0..Lmax), theta_j = Theta_j theta_max / pi.
    GL gl_win(160);
    ld Theta_star = g.full_sky ? kPiL : kPiL * (ld)ts / (ld)g.theta_max;
    Window win(Theta_star, (ld)g.alpha, &gl_win, g.window);

    // Lmax from the predicted error for the caller's spectrum (Sec. II.D): the
    // smallest smooth L <= the eq. Lmax2 value whose predicted relative error
    // stays below epsilon / 2 (the NUFFT takes the other part of the budget),
    // found by bisection over the smooth values (the error falls as L grows).
    g.predicted_error = -1.0;
    if (opts && opts->cl && !g.full_sky) {
        std::vector<double> cm;
        great_circle_spectrum(lmax, spin, opts->cl, cm);
        auto wfun = [&](double T) { return win((ld)T); };
        std::vector<int> cand;
        for (int c = 1; c <= L; ++c)
            if (is_smooth(2 * c + 1, odd_primes, 5)) cand.push_back(c);
        int lo = 0, hi = (int)cand.size() - 1;  // cand[hi] = L meets the target by construction of the rule
        const double target = 0.5 * eps;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (predicted_error(lmax, ts, g.theta_max, cand[mid], wfun, cm) <= target) hi = mid;
            else lo = mid + 1;
        }
        L = cand[hi];
        g.predicted_error = predicted_error(lmax, ts, g.theta_max, L, wfun, cm);
    }
    g.Lmax = L;
    g.N2 = 2 * L + 1;
    g.nring = L + 1;
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
        const DegreeRoots roots(lmax);
        // contiguous runs of rings per thread, each ring seeded with its
        // neighbour's cut-off (the first of a run with lmax sin(theta) plus the
        // usual margin of the transition, about 8 (lmax sin(theta))^(1/3))
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        const int run = (g.nring + (int)nt - 1) / (int)nt;
        auto est = [&](int j) { return (ld)lmax * fabsl(sinl((ld)g.ring_theta[j])); };
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t]() {
                const int j0 = (int)t * run, j1 = std::min(g.nring, j0 + run);
                int prev = -1;
                for (int j = j0; j < j1; ++j) {
                    const ld e = est(j);
                    const int guess = prev < 0 ? (int)(e + 8 * cbrtl(e)) : prev + (int)lroundl(e - est(j - 1));
                    g.ring_mmax[j] = ring_cutoff(lmax, spin, (ld)g.ring_theta[j], tau, roots, guess);
                    prev = g.ring_mmax[j];
                }
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
    // C(2m, m+s) = binom_mant[m] * 2^binom_exp[m] for m >= s, by the running
    // product over m (the one part that is sequential in m)
    std::vector<ld> binom_mant(lmax + 1, 0.5L);
    std::vector<int> binom_exp(lmax + 1, 1);
    {
        ld bm = 0.5L;
        int be = 1;
        for (int m = 0; m <= lmax; ++m) {
            if (m > s) {
                int e;
                bm = frexpl(bm * ((ld)(2 * m) * (2 * m - 1) / ((ld)(m + s) * (m - s))), &e);
                be += e;
            }
            binom_mant[m] = bm;
            binom_exp[m] = be;
        }
    }
    const DegreeRoots R(lmax);
    const ld S = s;
    // one order m: the recurrence coefficients a, b, c (one square root per
    // degree: the root in c is the previous degree's D), the normalisation P
    // and the seed factor K_m
    auto order = [&](int m, std::vector<ld> &a, std::vector<ld> &b, std::vector<ld> &c, std::vector<ld> &P) {
        const int l0 = std::max(m, s);
        if (l0 > lmax) return;
        const ld M = m;
        ld Dprev = 0;
        for (int l = l0; l <= lmax; ++l) {
            const ld L = l;
            const ld D = sqrtl(((L + 1) * (L + 1) - M * M) * ((L + 1) * (L + 1) - S * S));
            const ld iD = 1 / D;
            a[l] = R.r1[l] * iD;
            b[l] = (m * s == 0) ? 0 : a[l] * M * S * R.il[l];
            c[l] = (l == l0) ? 0 : R.r2[l] * Dprev * iD;
            Dprev = D;
        }
        P[l0] = 1;
        if (l0 + 1 <= lmax) P[l0 + 1] = 1;
        for (int l = l0 + 1; l < lmax; ++l) P[l + 1] = c[l] * P[l - 1];
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        for (int l = l0; l <= lmax; ++l) {
            double *e = &t.h_coef[4 * (base + l)];
            if (l < lmax) {
                const ld r = P[l] / P[l + 1];
                const ld A = a[l] * r, B = b[l] * r;
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
            mant = binom_mant[m];
            e2 = binom_exp[m];
        } else {
            mant = frexpl(expl(lgammal(2 * s + 1) - lgammal(s + m + 1) - lgammal(s - m + 1)), &e2);
        }
        if (e2 & 1) {
            mant *= 2;
            e2 -= 1;
        }
        const ld K = sqrtl((2 * l0 + 1) / (4 * kPiL)) * sqrtl(mant);
        int e3;
        const ld km = frexpl(K, &e3);
        t.h_kmant[m] = (double)km;
        t.h_kexp[m] = e3 + e2 / 2;
    };
    // the orders are independent: host threads take them in turn (the work of
    // order m falls with m, so interleaving keeps the threads even)
    const unsigned nt = lmax < 64 ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto worker = [&](unsigned tid) {
        std::vector<ld> a(lmax + 2), b(lmax + 2), c(lmax + 2), P(lmax + 2);
        for (int m = (int)tid; m <= lmax; m += (int)nt) order(m, a, b, c, P);
    };
    if (nt == 1) {
        worker(0);
    } else {
        std::vector<std::thread> th;
        for (unsigned q = 0; q < nt; ++q) th.emplace_back(worker, q);
        for (auto &x : th) x.join();
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
