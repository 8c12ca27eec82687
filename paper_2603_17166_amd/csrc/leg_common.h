// Per-lane arithmetic of the ring Legendre (Wigner-d) recurrence, shared by
// the GPU kernels and a host-side diagnostic entry point.
//
// For a ring at colatitude theta (y = 1 - cos theta = 2 sin^2(theta/2),
// ch = cos(theta/2), sh = sin(theta/2)) and an order m >= 0, the two functions
//   lambda+_l = sqrt((2l+1)/4pi) d^l_{m,-s}(theta)   (sY_lm, Appendix A eq. Ylm)
//   lambda-_l = sqrt((2l+1)/4pi) d^l_{m, s}(theta)   ((-s)Y_lm)
// start at l0 = max(m, s) from the single-term Wigner formula
//   lambda+_{l0} = (-1)^(m+s)              K_m ch^|m-s| sh^(m+s)
//   lambda-_{l0} = (-1)^(m+s) [m >= s]     K_m ch^(m+s) sh^|m-s|
// with K_m = N_{l0} sqrt(C(2 l0, m + s)), and obey the three-term recurrence in
// l written as mu_{l+1} = ((A_l +/- B_l) - A_l y) mu_l - mu_{l-1},
// lambda_l = P_l mu_l (the table of A, B, P is built on the host, see params.cpp).
//
// Near the pole the seeds are far below the double range (sh^(2m) with m in
// the thousands), so each value carries an integer scale k <= 0:
// true value = stored * 2^(512 k).  While k < 0 the value is below 2^-312 and
// contributes nothing; once it grows past 2^200 it is renormalised and k rises.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace psht {

constexpr int kScaleStep = 512;
constexpr int kSeedMinExp = -600;
#define PSHT_RESCALE_HI 1.6069380442589903e60   /* 2^200 */
#define PSHT_RESCALE_FACTOR 7.458340731200207e-155 /* 2^-512 */

struct XDbl {
    double m;  // mantissa in [0.5, 1) or 0
    int e;
};

// b^n for b >= 0, n >= 0 with the exponent carried separately (binary powering).
__host__ __device__ inline XDbl xd_pow(double b, int n) {
    int eb;
    double mb = frexp(b, &eb);
    double rm = 0.5;
    int re = 1;
    while (n > 0) {
        if (n & 1) {
            int t;
            rm = frexp(rm * mb, &t);
            re += eb + t;
        }
        n >>= 1;
        if (n > 0) {
            int t;
            mb = frexp(mb * mb, &t);
            eb = 2 * eb + t;
        }
    }
    XDbl r;
    r.m = rm;
    r.e = re;
    return r;
}

// mantissa * 2^e  ->  stored * 2^(kScaleStep * k)
__host__ __device__ inline void xd_split(double mant, int e, double &stored, int &k) {
    if (mant == 0.0) {
        stored = 0.0;
        k = 0;
        return;
    }
    if (e >= kSeedMinExp) {
        k = 0;
        stored = ldexp(mant, e);
    } else {
        int d = kSeedMinExp - e;
        k = -((d + kScaleStep - 1) / kScaleStep);
        stored = ldexp(mant, e - kScaleStep * k);
    }
}

// Seeds mu_{l0} of lambda+ and lambda- (mu_{l0} = lambda_{l0}); see the header comment.
__host__ __device__ inline void leg_seed(double kmant, int kexp, int m, int s, double ch, double sh,
                                         double &vp, int &kp, double &vm, int &km) {
    int dms = m > s ? m - s : s - m;
    XDbl c1 = xd_pow(ch, dms), s1 = xd_pow(sh, m + s);
    XDbl c2 = xd_pow(ch, m + s), s2 = xd_pow(sh, dms);
    xd_split(kmant * c1.m * s1.m, kexp + c1.e + s1.e, vp, kp);
    xd_split(kmant * c2.m * s2.m, kexp + c2.e + s2.e, vm, km);
    if ((m + s) & 1) {
        vp = -vp;
        if (m >= s) vm = -vm;
    }
}

// If the scaled value has grown past 2^200, renormalise the pair and raise k.
__host__ __device__ inline void leg_rescale(double &cur, double &prev, int &k) {
    if (k < 0 && fabs(cur) > PSHT_RESCALE_HI) {
        cur *= PSHT_RESCALE_FACTOR;
        prev *= PSHT_RESCALE_FACTOR;
        k += 1;
    }
}

}  // namespace psht
