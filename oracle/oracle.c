/*
 * Oracle for the partial-sky spin-weighted SHT: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, direct-sum evaluation of
 *   - the spin-s synthesis of Sec. I (eq. syn, "Synthesis general"),
 *   - its adjoint of Sec. I ("Adjoint synthesis general"),
 *   - the per-ring azimuthal Fourier coefficients F_m(theta) of the same map,
 * with sYlm built from the Wigner small-d definition of Appendix A (eq. Ylm):
 *   sY_lm(theta, phi) = sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) exp(i m phi).
 *
 * Only the tests, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * may load this library.  It shares no code, header, table or helper with the
 * GPU library; nothing in the product path may call it.
 *
 * Arithmetic: x87 long double internally (64-bit mantissa, exponent range
 * down to ~1e-4951, so no explicit rescaling is needed), double on output.
 *
 * Array conventions (the same ones the C ABI of the GPU library documents):
 *   alm:  complex double, shape [2][nalm] (g first, then c),
 *         nalm = (lmax+1)(lmax+2)/2, index(l,m) = m(2 lmax + 1 - m)/2 + l, m >= 0.
 *   map:  complex double [npts].
 * Entries with l < s do not exist (sY_lm is undefined there) and are ignored
 * on input / written as zero on output.  The imaginary parts of g_l0, c_l0
 * are ignored on input (reality condition a*_lm = (-1)^m a_l,-m of Sec. I).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

static int64_t alm_index(int lmax, int l, int m)
{
    return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

static int iabs_(int x) { return x < 0 ? -x : x; }
static int imax_(int a, int b) { return a > b ? a : b; }

/*
 * Wigner small-d at its lowest degree j = max(|a|,|b|), from the explicit
 * finite-sum formula
 *   d^j_{a b}(t) = sum_k (-1)^(a-b+k) sqrt((j+b)!(j-b)!(j+a)!(j-a)!)
 *                  / ((j+b-k)! k! (j-k-a)! (k-b+a)!)
 *                  cos(t/2)^(2j-2k+b-a) sin(t/2)^(2k+a-b),
 * summed over every k for which all factorial arguments are >= 0 (at the
 * lowest degree only one k survives).  Each term is formed in log space so
 * that sin(t/2)^(2j) cannot underflow before it is summed.
 */
static ld wigner_seed(int j, int a, int b, ld t)
{
    ld c = cosl(0.5L * t), s = sinl(0.5L * t);
    ld sum = 0.0L;
    int kmin = imax_(0, b - a), kmax = j + b < j - a ? j + b : j - a;
    for (int k = kmin; k <= kmax; ++k) {
        int pc = 2 * j - 2 * k + b - a;   /* power of cos(t/2) */
        int ps = 2 * k + a - b;           /* power of sin(t/2) */
        ld logmag = 0.5L * (lgammal(j + b + 1) + lgammal(j - b + 1) + lgammal(j + a + 1) + lgammal(j - a + 1))
                  - lgammal(j + b - k + 1) - lgammal(k + 1) - lgammal(j - k - a + 1) - lgammal(k - b + a + 1);
        int neg = ((a - b + k) & 1) != 0;
        if (pc > 0) {
            if (c == 0.0L) continue;
            logmag += pc * logl(fabsl(c));
            if (c < 0 && (pc & 1)) neg = !neg;
        }
        if (ps > 0) {
            if (s == 0.0L) continue;
            logmag += ps * logl(fabsl(s));
            if (s < 0 && (ps & 1)) neg = !neg;
        }
        if (logmag < -11000.0L) continue;   /* below the long double range */
        ld term = expl(logmag);
        sum += neg ? -term : term;
    }
    return sum;
}

/*
 * d^l_{a b}(t) for l = 0..lmax into out[0..lmax] (zero below j0 = max(|a|,|b|)),
 * by the standard three-term recurrence in the degree:
 *   l sqrt(((l+1)^2 - a^2)((l+1)^2 - b^2)) d^{l+1}
 *     = (2l+1) (l(l+1) cos t - a b) d^l - (l+1) sqrt((l^2 - a^2)(l^2 - b^2)) d^{l-1},
 * started from the explicit value at j0 and d^{j0-1} = 0.  At l = 0 (only
 * reached when a = b = 0) the recurrence is used in the form divided by l,
 * which is the Legendre recurrence (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}.
 */
static void wigner_column(int lmax, int a, int b, ld t, ld *out)
{
    int j0 = imax_(iabs_(a), iabs_(b));
    for (int l = 0; l <= lmax && l < j0; ++l) out[l] = 0.0L;
    if (j0 > lmax) return;
    ld x = cosl(t);
    ld dm1 = 0.0L, d = wigner_seed(j0, a, b, t);
    out[j0] = d;
    for (int l = j0; l < lmax; ++l) {
        ld L = (ld)l, A = (ld)a, B = (ld)b;
        ld dp;
        if (l == 0) {
            dp = x * d;  /* a = b = 0: P_1 = x P_0 */
        } else {
            ld lhs = L * sqrtl(((L + 1) * (L + 1) - A * A) * ((L + 1) * (L + 1) - B * B));
            ld t1 = (2 * L + 1) * (L * (L + 1) * x - A * B) * d;
            ld t2 = (L + 1) * sqrtl((L * L - A * A) * (L * L - B * B)) * dm1;
            dp = (t1 - t2) / lhs;
        }
        out[l + 1] = dp;
        dm1 = d;
        d = dp;
    }
}

/* Exported for the pinning tests: d^l_{a b}(theta), l = 0..lmax. */
void oracle_wigner_d(int lmax, int a, int b, double theta, double *out)
{
    ld *col = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
    wigner_column(lmax, a, b, (ld)theta, col);
    for (int l = 0; l <= lmax; ++l) out[l] = (double)col[l];
    free(col);
}

/* Coefficient a_lm (g or c, selected by comp) for any -l <= m <= l, using the
 * reality condition a_{l,-m} = (-1)^m conj(a_lm) (Sec. I) for negative m; the
 * m = 0 coefficient is real, so its imaginary part is dropped. */
static void coeff(const double *alm, int lmax, int comp, int l, int m, ld *re, ld *im)
{
    int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    int am = iabs_(m);
    const double *z = alm + 2 * (comp * nalm + alm_index(lmax, l, am));
    ld r = z[0], i = z[1];
    if (m == 0) { *re = r; *im = 0.0L; return; }
    if (m > 0) { *re = r; *im = i; return; }
    ld sg = (am & 1) ? -1.0L : 1.0L;
    *re = sg * r;
    *im = -sg * i;
}

/*
 * Azimuthal Fourier coefficient of the synthesized map on the ring theta:
 *   F_m(theta) = - sum_{l >= max(|m|,s)} (g_lm + i c_lm) sqrt((2l+1)/4pi) d^l_{m,-s}(theta),
 * so that f(theta, phi) = sum_m F_m(theta) exp(i m phi) (eq. syn with eq. Ylm).
 * col is scratch of length lmax+1.
 */
static void ring_coeff(const double *alm, int lmax, int s, int m, ld theta, ld *col, ld *Fre, ld *Fim)
{
    wigner_column(lmax, m, -s, theta, col);
    ld re = 0.0L, im = 0.0L;
    int l0 = imax_(iabs_(m), s);
    for (int l = l0; l <= lmax; ++l) {
        ld gr, gi, cr, ci;
        coeff(alm, lmax, 0, l, m, &gr, &gi);
        coeff(alm, lmax, 1, l, m, &cr, &ci);
        ld lam = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L)) * col[l];
        /* (g + i c) lam */
        re += (gr - ci) * lam;
        im += (gi + cr) * lam;
    }
    *Fre = -re;
    *Fim = -im;
}

/*
 * Synthesis general (eq. syn):
 *   f_p = - sum_{l=0}^{lmax} sum_{m=-l}^{l} (g_lm + i c_lm) sY_lm(theta_p, phi_p),
 * evaluated directly point by point (parallel over points).
 */
void oracle_synth(int lmax, int s, const double *alm, int64_t npts,
                  const double *theta, const double *phi, double *map, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        ld *col = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
#pragma omp for schedule(dynamic, 4)
        for (int64_t p = 0; p < npts; ++p) {
            ld re = 0.0L, im = 0.0L;
            for (int m = -lmax; m <= lmax; ++m) {
                ld Fr, Fi;
                ring_coeff(alm, lmax, s, m, (ld)theta[p], col, &Fr, &Fi);
                ld ang = (ld)m * (ld)phi[p];
                ld cr = cosl(ang), ci = sinl(ang);
                re += Fr * cr - Fi * ci;
                im += Fr * ci + Fi * cr;
            }
            map[2 * p] = (double)re;
            map[2 * p + 1] = (double)im;
        }
        free(col);
    }
}

/*
 * F_m(theta_j) for |m| <= mmax on a set of rings, written as complex double
 * F[(m + mmax) * nring + j].  This is the exact result of the Legendre step
 * (the per-ring Fourier coefficients of the map of eq. syn).
 */
void oracle_ring_coeffs(int lmax, int s, const double *alm, int nring, const double *theta,
                        int mmax, double *F, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t nm = 2 * (int64_t)mmax + 1;
#pragma omp parallel
    {
        ld *col = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int64_t mi = 0; mi < nm; ++mi) {
            for (int j = 0; j < nring; ++j) {
                int m = (int)mi - mmax;
                ld Fr = 0.0L, Fi = 0.0L;
                if (iabs_(m) <= lmax) ring_coeff(alm, lmax, s, m, (ld)theta[j], col, &Fr, &Fi);
                F[2 * (mi * nring + j)] = (double)Fr;
                F[2 * (mi * nring + j) + 1] = (double)Fi;
            }
        }
        free(col);
    }
}

/*
 * Adjoint synthesis general (Sec. I), for 0 <= m <= l, l >= s:
 *   g~_lm = -1/2    sum_p [ f_p sY*_lm(p) + (-1)^s conj(f_p) (-s)Y*_lm(p) ]
 *   c~_lm = -1/(2i) sum_p [ f_p sY*_lm(p) - (-1)^s conj(f_p) (-s)Y*_lm(p) ]
 * with sY*_lm = sqrt((2l+1)/4pi) d^l_{m,-s}(theta) exp(-i m phi) and
 * (-s)Y*_lm = sqrt((2l+1)/4pi) d^l_{m,s}(theta) exp(-i m phi).
 * Entries with l < s are written as zero.  Parallel over m, so every output
 * coefficient is summed by one thread in point order.
 */
void oracle_adjoint(int lmax, int s, const double *map, int64_t npts,
                    const double *theta, const double *phi, double *alm, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    memset(alm, 0, sizeof(double) * 4 * (size_t)nalm);
    ld sgn_s = (s & 1) ? -1.0L : 1.0L;
#pragma omp parallel
    {
        ld *dp = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        ld *dm = (ld *)malloc(sizeof(ld) * (size_t)(lmax + 1));
        ld *acc = (ld *)malloc(sizeof(ld) * 4 * (size_t)(lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m <= lmax; ++m) {
            int l0 = imax_(m, s);
            if (l0 > lmax) continue;
            for (int i = 0; i < 4 * (lmax + 1); ++i) acc[i] = 0.0L;
            for (int64_t p = 0; p < npts; ++p) {
                wigner_column(lmax, m, -s, (ld)theta[p], dp);
                wigner_column(lmax, m, s, (ld)theta[p], dm);
                ld ang = -(ld)m * (ld)phi[p];
                ld er = cosl(ang), ei = sinl(ang);   /* exp(-i m phi) */
                ld fr = map[2 * p], fi = map[2 * p + 1];
                /* u = f exp(-i m phi), v = conj(f) exp(-i m phi) */
                ld ur = fr * er - fi * ei, ui = fr * ei + fi * er;
                ld vr = fr * er + fi * ei, vi = fr * ei - fi * er;
                for (int l = l0; l <= lmax; ++l) {
                    ld nl = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
                    ld yp = nl * dp[l], ym = nl * dm[l];
                    acc[4 * l + 0] += ur * yp;   /* X = sum f sY* */
                    acc[4 * l + 1] += ui * yp;
                    acc[4 * l + 2] += vr * ym;   /* Y = sum conj(f) (-s)Y* */
                    acc[4 * l + 3] += vi * ym;
                }
            }
            for (int l = l0; l <= lmax; ++l) {
                ld Xr = acc[4 * l], Xi = acc[4 * l + 1], Yr = acc[4 * l + 2], Yi = acc[4 * l + 3];
                /* g = -(X + (-1)^s Y)/2 ; c = -(X - (-1)^s Y)/(2i) = (i/2)(X - (-1)^s Y) */
                ld gr = -0.5L * (Xr + sgn_s * Yr), gi = -0.5L * (Xi + sgn_s * Yi);
                ld dr = Xr - sgn_s * Yr, di = Xi - sgn_s * Yi;
                ld cr = -0.5L * di, ci = 0.5L * dr;
                int64_t k = alm_index(lmax, l, m);
                alm[2 * k] = (double)gr;
                alm[2 * k + 1] = (double)gi;
                alm[2 * (nalm + k)] = (double)cr;
                alm[2 * (nalm + k) + 1] = (double)ci;
            }
        }
        free(dp);
        free(dm);
        free(acc);
    }
}
