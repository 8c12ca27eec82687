// Rotation of spherical-harmonic coefficients, points and spin bases into the
// patch frame (Sec. II, step 1: coordinates in which the patch centre is the
// north pole).
//
// R = Rz(alpha) Ry(beta) Rz(gamma) (active rotation, z-y-z Euler angles) moves
// a point n to R n and a field f to f o R^-1.  The coefficients of the moved
// field are
//   a'_lm = exp(-i m alpha) sum_{m'=-l..l} d^l_{m m'}(beta) exp(-i m' gamma) a_lm'
// with a_{l,-m'} = (-1)^m' conj(a_lm') (the reality condition of Sec. I; g and
// c of a spin field each obey it) and d^l the Wigner small-d matrix of
// Appendix A.  The cost is O(lmax^3); the kernels below:
//
// k_rot_prep  b_{l m'} = exp(-i m' gamma) a_lm' for every m' = -l..l, stored
//             l-major with the columns in |m'|-major order 0, 1, -1, 2, -2, ...
//             (zero where |m'| > l), so that a wavefront reads one row of
//             consecutive columns per degree.
// k_rot_main  one wavefront per (8 consecutive orders m, 128 consecutive
//             columns): each lane runs the three-term recurrence in l of
//             d^l_{m m'}(beta) for 8 orders x 2 columns, forms the partial sums
//             sum_{m'} d b of the 8 outputs (l, m) per degree, reduces them
//             over the 64 lanes with a transposed butterfly (each exchange
//             round halves the values held per lane), turns them by
//             exp(-i m alpha) and adds them into a'_lm with atomics (the
//             columns of one order are spread over several wavefronts).
// k_rot_points, k_spin_phase  points and the spin basis angle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lane_ops.h"
#include "leg_common.h"
#include "psht_internal.h"

namespace psht {

constexpr int kRotK = 8;                // orders per wavefront
constexpr int kRotP = 2;                // columns per lane
constexpr int kRotCols = 64 * kRotP;    // columns per wavefront

__host__ __device__ inline int rot_mp(int col) { return (col & 1) ? (col + 1) / 2 : -(col / 2); }

__device__ inline int64_t rot_alm_index(int lmax, int l, int m) { return (int64_t)m * (2 * lmax + 1 - m) / 2 + l; }

// exp(-i k x) for an integer k: the product k x is split into hi + lo exactly
// (fma), so that its rounding does not enter the phase.
__device__ inline double2 phase_neg(int k, double x) {
    const double hi = (double)k * x;
    const double lo = fma((double)k, x, -hi);
    double s, c;
    sincos(hi, &s, &c);
    return make_double2(c - s * lo, -(s + c * lo));
}

// Double-double difference a - b (two-sum on the high parts).
__device__ inline double2 dd_sub(double2 a, double2 b) {
    const double s = a.x - b.x;
    const double bb = s - a.x;
    const double e = (a.x - (s - bb)) + (-b.x - bb);
    const double t = e + (a.y - b.y);
    const double hi = s + t;
    return make_double2(hi, t - (hi - s));
}

struct RotArgs {
    const double2 *alm;   // input [nc][nalm]
    double2 *B;           // [nc][lmax + 1][ncol]
    double *out;          // output [nc][nalm] complex, accumulated
    const double2 *lf;    // log2(n!) as double-double, n = 0..2 lmax
    int lmax, ncol;
    int64_t nalm;
    double alpha, gamma, cb, hc, hs;  // cos beta, cos(beta/2), sin(beta/2)
};

__global__ __launch_bounds__(256) void k_rot_prep(RotArgs A, int nc) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    const int c = blockIdx.z;
    if (col >= A.ncol || c >= nc) return;
    const int mp = rot_mp(col), k = mp < 0 ? -mp : mp;
    double2 v = make_double2(0.0, 0.0);
    if (k <= l) {
        double2 a = A.alm[(int64_t)c * A.nalm + rot_alm_index(A.lmax, l, k)];
        if (k == 0) a.y = 0.0;
        if (mp < 0) {
            a.y = -a.y;
            if (k & 1) {
                a.x = -a.x;
                a.y = -a.y;
            }
        }
        const double2 e = phase_neg(mp, A.gamma);
        v = make_double2(e.x * a.x - e.y * a.y, e.x * a.y + e.y * a.x);
    }
    A.B[((int64_t)c * (A.lmax + 1) + l) * A.ncol + col] = v;
}

__global__ __launch_bounds__(256) void k_rot_zero(double *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = 0.0;
}

// Seed d^{l0}_{m m'}(beta), l0 = max(m, |m'|), m >= 0, from the single
// surviving term of the explicit sum at the lowest degree:
//   m >= |m'|:  (-1)^(m-m') sqrt(C(2m, m+m'))  c^(m+m')  s^(m-m')
//   m' > m:                 sqrt(C(2m', m'+m)) c^(m'+m)  s^(m'-m)
//   -m' > m:    (-1)^(m+l0) sqrt(C(2l0, l0+m)) c^(l0-m)  s^(l0+m)
// (c = cos(beta/2), s = sin(beta/2)), returned as stored * 2^(512 k), k <= 0.
// The binomial comes from log2(n!) in double-double, the powers by binary
// powering with a separate exponent.
__device__ inline void rot_seed(const RotArgs &A, int m, int mp, double &stored, int &k) {
    const int am = mp < 0 ? -mp : mp;
    int j, x, pc, ps;
    bool neg;
    if (m >= am) {
        j = m;
        x = mp;
        pc = m + mp;
        ps = m - mp;
        neg = ((m - mp) & 1) != 0;
    } else if (mp > 0) {
        j = mp;
        x = m;
        pc = mp + m;
        ps = mp - m;
        neg = false;
    } else {
        j = am;
        x = m;
        pc = j - m;
        ps = j + m;
        neg = ((m + j) & 1) != 0;
    }
    if ((pc > 0 && A.hc == 0.0) || (ps > 0 && A.hs == 0.0)) {
        stored = 0.0;
        k = 0;
        return;
    }
    if (A.hs < 0.0 && (ps & 1)) neg = !neg;
    const double2 L = dd_sub(dd_sub(A.lf[2 * j], A.lf[j + x]), A.lf[j - x]);
    const double half_hi = 0.5 * L.x, half_lo = 0.5 * L.y;
    const double eb = floor(half_hi);
    const double mb = exp2((half_hi - eb) + half_lo);
    const XDbl pcx = xd_pow(fabs(A.hc), pc), psx = xd_pow(fabs(A.hs), ps);
    int e1;
    const double mant = frexp(mb * pcx.m * psx.m, &e1);
    xd_split(neg ? -mant : mant, (int)eb + pcx.e + psx.e + e1, stored, k);
}

// Renormalisation of a scaled pair (true value = stored * 2^(512 k), k <= 0):
// once the stored value passes 2^200 both values are scaled by 2^-512.
__device__ inline void rot_rescale(double &cur, double &prev, int &k) {
    const bool big = (k < 0) && (fabs(cur) > PSHT_RESCALE_HI);
    const double f = big ? PSHT_RESCALE_FACTOR : 1.0;
    cur *= f;
    prev *= f;
    k += big ? 1 : 0;
}

// Factors of the recurrence that depend on the order only, for the step from
// degree l to l + 1 (A_l(x) = sqrt(l^2 - x^2)):
//   F1 = (2l+1)(l+1) / A_{l+1}(m),  Q = m / (l(l+1)),  F2 = (l+1) A_l(m) / (l A_{l+1}(m)),
// zero where the step does not exist (l + 1 <= m) and Q = F2 = 0 at l = 0.
__device__ inline double4 rot_order_factors(int l, int m) {
    if (l + 1 <= m) return make_double4(0.0, 0.0, 0.0, 0.0);
    const double L = l, M = m;
    const double a1 = sqrt((L + 1) * (L + 1) - M * M);
    const double f1 = (2 * L + 1) * (L + 1) / a1;
    if (l == 0) return make_double4(f1, 0.0, 0.0, 0.0);
    const double a0 = sqrt(L * L - M * M);
    return make_double4(f1, M / (L * (L + 1)), (L + 1) * a0 / (L * a1), 0.0);
}

// Exchange-halves round on n complex values (re[i], im[i]): lanes with the
// given lane bit clear keep values 0..n/2-1, the others n/2..n-1, each summed
// with the partner lane's copy.
template <int N, int BIT>
__device__ inline void rot_halve(double *re, double *im, int lane) {
    constexpr int H = N / 2;
    if (BIT == 32) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            swap32(re[i], re[i + H]);
            re[i] += re[i + H];
            swap32(im[i], im[i + H]);
            im[i] += im[i + H];
        }
    } else if (BIT == 16) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            swap16(re[i], re[i + H]);
            re[i] += re[i + H];
            swap16(im[i], im[i + H]);
            im[i] += im[i + H];
        }
    } else {
        const bool up = (lane & BIT) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double sr = up ? re[i] : re[i + H], si = up ? im[i] : im[i + H];
            const double kr = up ? re[i + H] : re[i], ki = up ? im[i + H] : im[i];
            const double rr = BIT == 8 ? lane_xor8(sr) : lane_xor4(sr);
            const double ri = BIT == 8 ? lane_xor8(si) : lane_xor4(si);
            re[i] = kr + rr;
            im[i] = ki + ri;
        }
    }
}

// Full sum of one complex value over the lanes i ^ b for the remaining bits.
template <int BIT> __device__ inline void rot_allsum(double &re, double &im) {
    if (BIT == 4) {
        re += lane_xor4(re);
        im += lane_xor4(im);
    } else if (BIT == 2) {
        re += quad_xor2(re);
        im += quad_xor2(im);
    } else {
        re += quad_xor1(re);
        im += quad_xor1(im);
    }
}

// Reduce NQ = 8 NC complex values over the wavefront; afterwards lane i holds
// the complete sum of value q = i >> S (S = 2 for NC = 2, 3 for NC = 1).
template <int NC> __device__ inline void rot_reduce(double *re, double *im, int lane) {
    constexpr int NQ = kRotK * NC;
    rot_halve<NQ, 32>(re, im, lane);
    rot_halve<NQ / 2, 16>(re, im, lane);
    rot_halve<NQ / 4, 8>(re, im, lane);
    if (NC == 2) {
        rot_halve<2, 4>(re, im, lane);
    } else {
        rot_allsum<4>(re[0], im[0]);
    }
    rot_allsum<2>(re[0], im[0]);
    rot_allsum<1>(re[0], im[0]);
}

template <int NC> __global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_rot_main(RotArgs A) {
    constexpr int S = (NC == 2) ? 2 : 3;
    __shared__ double4 fac[8][kRotK];
    __shared__ double seed_v[kRotK * kRotP][64];
    __shared__ int seed_k[kRotK * kRotP][64];
    const int lane = threadIdx.x;
    const int m0 = blockIdx.x * kRotK;
    const int col0 = blockIdx.y * kRotCols;
    const int lmax = A.lmax;
    const int mpmin = (col0 + 1) / 2;  // smallest |m'| of the wavefront's columns
    int l = max(m0, mpmin);
    if (l > lmax || m0 > lmax) return;

    int mpv[kRotP], amp[kRotP];
    bool colok[kRotP];
    double aprev[kRotP];  // A_l(m') of the current degree
#pragma unroll
    for (int p = 0; p < kRotP; ++p) {
        const int col = col0 + p * 64 + lane;
        colok[p] = col < A.ncol;
        mpv[p] = colok[p] ? rot_mp(col) : 0;
        // columns past the end never start (their first degree lies past lmax)
        amp[p] = colok[p] ? (mpv[p] < 0 ? -mpv[p] : mpv[p]) : lmax + 1;
        const double d2 = (double)l * l - (double)mpv[p] * mpv[p];
        aprev[p] = d2 > 0.0 ? sqrt(d2) : 0.0;
    }
    // states (order k, column p): value at the current degree, previous value
    // and scale; each starts at degree max(m0 + k, |m'|) from its seed, which
    // waits in LDS
    double d[kRotK][kRotP], dp[kRotK][kRotP];
    int kk[kRotK][kRotP];
#pragma unroll
    for (int k = 0; k < kRotK; ++k)
#pragma unroll
        for (int p = 0; p < kRotP; ++p) {
            d[k][p] = dp[k][p] = 0.0;
            kk[k][p] = 0;
            double sv = 0.0;
            int sk = 0;
            if (max(m0 + k, amp[p]) <= lmax) rot_seed(A, m0 + k, mpv[p], sv, sk);
            seed_v[k * kRotP + p][lane] = sv;
            seed_k[k * kRotP + p][lane] = sk;
        }
    // the lane's output after the reduction: value q = lane >> S = k NC + c
    const int q = lane >> S, qk = q / NC, qc = q - qk * NC;
    const int qm = m0 + qk;
    const bool writer = (lane & ((1 << S) - 1)) == 0 && qm <= lmax;
    const double2 rphase = phase_neg(qm, A.alpha);
    const double2 *Bc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Bc[c] = A.B + (int64_t)c * (lmax + 1) * A.ncol;
    double *outq = A.out + 2 * ((int64_t)qc * A.nalm);

    while (l <= lmax) {
        const int lb = l, nsteps = min(8, lmax + 1 - lb);
        {
            const int u = lane >> 3, k = lane & 7;
            fac[u][k] = rot_order_factors(lb + u, m0 + k);
        }
        __syncthreads();
        bool slow = false;
#pragma unroll
        for (int k = 0; k < kRotK; ++k)
#pragma unroll
            for (int p = 0; p < kRotP; ++p) {
                const int l0 = max(m0 + k, amp[p]);
                slow |= (kk[k][p] < 0) || (l0 >= lb && l0 < lb + nsteps);
            }
        slow = __any(slow);
        for (int u = 0; u < nsteps; ++u) {
            l = lb + u;
            double br[kRotP][NC], bi[kRotP][NC];
#pragma unroll
            for (int p = 0; p < kRotP; ++p)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    br[p][c] = bi[p][c] = 0.0;
                    if (colok[p]) {
                        const double2 v = Bc[c][(int64_t)l * A.ncol + col0 + p * 64 + lane];
                        br[p][c] = v.x;
                        bi[p][c] = v.y;
                    }
                }
            double re[kRotK * NC], im[kRotK * NC];
            if (slow) {
#pragma unroll
                for (int k = 0; k < kRotK; ++k)
#pragma unroll
                    for (int p = 0; p < kRotP; ++p)
                        if (l == max(m0 + k, amp[p])) {
                            d[k][p] = seed_v[k * kRotP + p][lane];
                            dp[k][p] = 0.0;
                            kk[k][p] = seed_k[k * kRotP + p][lane];
                        }
            }
#pragma unroll
            for (int k = 0; k < kRotK; ++k)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double sr = 0.0, si = 0.0;
#pragma unroll
                    for (int p = 0; p < kRotP; ++p) {
                        const double dv = (slow && kk[k][p] < 0) ? 0.0 : d[k][p];
                        sr = fma(dv, br[p][c], sr);
                        si = fma(dv, bi[p][c], si);
                    }
                    re[k * NC + c] = sr;
                    im[k * NC + c] = si;
                }
            rot_reduce<NC>(re, im, lane);
            if (writer && qm <= l) {
                double *dst = outq + 2 * rot_alm_index(lmax, l, qm);
                atomicAdd(dst, rphase.x * re[0] - rphase.y * im[0]);
                atomicAdd(dst + 1, rphase.x * im[0] + rphase.y * re[0]);
            }
            if (l < lmax) {
                double g1[kRotP], g2[kRotP];
#pragma unroll
                for (int p = 0; p < kRotP; ++p) {
                    const double d2 = (double)(l + 1) * (l + 1) - (double)mpv[p] * mpv[p];
                    const double an = d2 > 0.0 ? sqrt(d2) : 0.0;
                    g1[p] = an > 0.0 ? 1.0 / an : 0.0;
                    g2[p] = aprev[p] * g1[p];
                    aprev[p] = an;
                }
#pragma unroll
                for (int k = 0; k < kRotK; ++k) {
                    const double4 f = fac[u][k];
#pragma unroll
                    for (int p = 0; p < kRotP; ++p) {
                        const double t = fma(-f.y, (double)mpv[p], A.cb);
                        const double a = f.x * g1[p] * t, b = f.z * g2[p];
                        const double nv = fma(a, d[k][p], -b * dp[k][p]);
                        dp[k][p] = d[k][p];
                        d[k][p] = nv;
                    }
                }
            }
        }
        if (slow) {
#pragma unroll
            for (int k = 0; k < kRotK; ++k)
#pragma unroll
                for (int p = 0; p < kRotP; ++p) rot_rescale(d[k][p], dp[k][p], kk[k][p]);
        }
        __syncthreads();
        l = lb + nsteps;
    }
}

// Points: n' = R n; psi from the rotated basis vector R e_theta(n) to
// e_theta(n'), towards e_phi(n').
__global__ __launch_bounds__(256) void k_rot_points(int64_t n, RotMatrix R, const double *theta, const double *phi,
                                                    double *theta_out, double *phi_out, double *psi_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double st, ct, sp, cp;
    sincos(theta[i], &st, &ct);
    sincos(phi[i], &sp, &cp);
    const double v[3] = {st * cp, st * sp, ct};
    const double e[3] = {ct * cp, ct * sp, -st};
    double w[3], f[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        w[r] = R.r[r][0] * v[0] + R.r[r][1] * v[1] + R.r[r][2] * v[2];
        f[r] = R.r[r][0] * e[0] + R.r[r][1] * e[1] + R.r[r][2] * e[2];
    }
    const double rho = sqrt(w[0] * w[0] + w[1] * w[1]);
    const double t2 = atan2(rho, w[2]);
    double p2 = atan2(w[1], w[0]);
    if (p2 < 0.0) p2 += 2.0 * M_PI;
    if (p2 >= 2.0 * M_PI) p2 = 0.0;
    double st2, ct2, sp2, cp2;
    sincos(t2, &st2, &ct2);
    sincos(p2, &sp2, &cp2);
    const double along_t = f[0] * ct2 * cp2 + f[1] * ct2 * sp2 - f[2] * st2;
    const double along_p = -f[0] * sp2 + f[1] * cp2;
    theta_out[i] = t2;
    phi_out[i] = p2;
    psi_out[i] = atan2(along_p, along_t);
}

template <typename T>
__global__ __launch_bounds__(256) void k_spin_phase(int64_t n, double ks, const double *psi, T *map) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s, c;
    sincos(ks * psi[i], &s, &c);
    const double xr = map[2 * i], xi = map[2 * i + 1];
    map[2 * i] = (T)(c * xr - s * xi);
    map[2 * i + 1] = (T)(c * xi + s * xr);
}

hipError_t launch_rotate_alm(int lmax, int nc, double alpha, double beta, double gamma, const void *alm_in,
                             void *alm_out, void *ws, const double2 *lf, hipStream_t st) {
    RotArgs A;
    A.alm = (const double2 *)alm_in;
    A.B = (double2 *)ws;
    A.out = (double *)alm_out;
    A.lf = lf;
    A.lmax = lmax;
    A.ncol = 2 * lmax + 1;
    A.nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;
    A.alpha = alpha;
    A.gamma = gamma;
    A.cb = cos(beta);
    A.hc = cos(0.5 * beta);
    A.hs = sin(0.5 * beta);
    const int64_t nout = 2 * (int64_t)nc * A.nalm;
    k_rot_zero<<<dim3((unsigned)((nout + 255) / 256)), 256, 0, st>>>(A.out, nout);
    k_rot_prep<<<dim3((A.ncol + 255) / 256, lmax + 1, nc), 256, 0, st>>>(A, nc);
    const dim3 grid((lmax + kRotK) / kRotK, (A.ncol + kRotCols - 1) / kRotCols);
    if (nc == 2) k_rot_main<2><<<grid, 64, 0, st>>>(A);
    else k_rot_main<1><<<grid, 64, 0, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_rotate_points(int64_t n, const RotMatrix &R, const double *theta, const double *phi,
                                double *theta_out, double *phi_out, double *psi_out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_rot_points<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(n, R, theta, phi, theta_out, phi_out, psi_out);
    return hipGetLastError();
}

hipError_t launch_spin_phase(int64_t n, double ks, int fp32, const double *psi, void *map, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (fp32) k_spin_phase<float><<<grid, 256, 0, st>>>(n, ks, psi, (float *)map);
    else k_spin_phase<double><<<grid, 256, 0, st>>>(n, ks, psi, (double *)map);
    return hipGetLastError();
}

}  // namespace psht
