// Ring Legendre (Wigner-d) step of the partial-sky transform on gfx950.
//
// Synthesis: for every order m and every ring j with m <= mmax_j,
//   F_j(+m) = -          sum_l (g_lm + i c_lm)             lambda+_lm(theta_j)
//   F_j(-m) = -(-1)^s    sum_l (conj g_lm + i conj c_lm)   lambda-_lm(theta_j)
// so that f(theta_j, phi) = sum_m F_j(m) e^{i m phi} is the map of eq. syn on
// the ring (reality condition a_{l,-m} = (-1)^m conj(a_lm), Sec. I).  This is
// the step whose cost dominates the method (Sec. II.A); only rings inside the
// apodized cap are evaluated and orders well above lmax sin(theta_j) are
// dropped (polar optimization).
//
// Adjoint: the exact transpose,
//   A_lm = sum_j lambda+_lm(theta_j) F'_j(m),  B_lm = sum_j lambda-_lm(theta_j) conj F'_j(-m),
//   g~_lm = -(A + (-1)^s B)/2,  c~_lm = (i/2)(A - (-1)^s B)   (Sec. I, adjoint).
//
// Work decomposition: one 64-lane wavefront per (m, chunk of 64*R rings); each
// lane owns R rings (registers) and runs the recurrence in l; the coefficient
// table and the alm of order m are wave-uniform and come through the scalar
// cache.  The work items of one m sit on one XCD so they share its L2.
#include "leg_common.h"
#include "psht_internal.h"

namespace psht {

struct LegArgs {
    const LegItem *items;
    int nitems;
    int group;  // items per order m
    const double *coef;
    const double *kmant;
    const int32_t *kexp;
    const double *ring_y, *ring_ch, *ring_sh;
    const int32_t *ring_mmax;
    int nring, lmax, spin, mmax;
    int64_t nalm;
    const double *alm;  // synthesis input, complex [2][nalm]
    double *alm_out;    // adjoint output, complex [2][nalm]
    double *F;          // complex [2 mmax + 1][nring]: synthesis output / adjoint input
};

// Block -> item map: the `group` items of one order m run on the same XCD
// (blocks are dealt round-robin to the 8 XCDs), and every XCD starts with the
// low orders, which carry the most work.
__device__ inline int leg_item_index(int bid, int group) {
    int xcd = bid & 7, k = bid >> 3;
    int q = k / group, i = k - q * group;
    return (xcd + 8 * q) * group + i;
}

template <int R, bool SPIN>
__global__ __launch_bounds__(64) void k_leg_synth(LegArgs a) {
    const int idx = leg_item_index(blockIdx.x, a.group);
    if (idx >= a.nitems) return;
    const LegItem it = a.items[idx];
    if (it.je <= it.jb) return;
    const int m = it.m, s = a.spin, lane = threadIdx.x;
    const int l0 = m > s ? m : s;
    if (l0 > a.lmax) return;

    double y[R], up[R], upp[R], um[R], ump[R];
    double fpr[R], fpi[R], fmr[R], fmi[R];
    int kp[R], km[R];
    bool act[R];
    const double kmant = a.kmant[m];
    const int kexp = a.kexp[m];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int j = it.jb + r * 64 + lane;
        act[r] = (j < it.je) && (a.ring_mmax[j] >= m);
        y[r] = 0.0;
        up[r] = um[r] = upp[r] = ump[r] = 0.0;
        kp[r] = km[r] = 0;
        fpr[r] = fpi[r] = fmr[r] = fmi[r] = 0.0;
        if (act[r]) {
            y[r] = a.ring_y[j];
            leg_seed(kmant, kexp, m, s, a.ring_ch[j], a.ring_sh[j], up[r], kp[r], um[r], km[r]);
            if (!SPIN) { um[r] = up[r]; km[r] = kp[r]; }
        }
    }
    const int64_t base = (int64_t)m * (2 * a.lmax + 1 - m) / 2;
    const double *T = a.coef + 4 * base;
    const double2 *G = reinterpret_cast<const double2 *>(a.alm) + base;
    const double2 *C = reinterpret_cast<const double2 *>(a.alm) + a.nalm + base;
    const bool m0 = (m == 0);

    int l = l0;
    // Phase 1: some active lane still carries a scaled (negligible) value.
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= act[r] && (kp[r] < 0 || km[r] < 0);
    scaled = __any(scaled);
    while (scaled && l <= a.lmax) {
        const double P = T[4 * l + 3];
        double2 g = G[l], c = C[l];
        if (m0) { g.y = 0.0; c.y = 0.0; }
        const double apr = (g.x - c.y) * P, api = (g.y + c.x) * P;
        const double amr = (g.x + c.y) * P, ami = (c.x - g.y) * P;
        const double nA = T[4 * l], ApB = T[4 * l + 1], AmB = T[4 * l + 2];
        bool any_scaled = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double vp = kp[r] == 0 ? up[r] : 0.0;
            fpr[r] = fma(apr, vp, fpr[r]);
            fpi[r] = fma(api, vp, fpi[r]);
            if (SPIN) {
                const double vm = km[r] == 0 ? um[r] : 0.0;
                fmr[r] = fma(amr, vm, fmr[r]);
                fmi[r] = fma(ami, vm, fmi[r]);
            } else {
                fmr[r] = fma(amr, vp, fmr[r]);
                fmi[r] = fma(ami, vp, fmi[r]);
            }
            if (l < a.lmax) {
                double np = fma(fma(nA, y[r], ApB), up[r], -upp[r]);
                upp[r] = up[r];
                up[r] = np;
                leg_rescale(up[r], upp[r], kp[r]);
                if (SPIN) {
                    double nm = fma(fma(nA, y[r], AmB), um[r], -ump[r]);
                    ump[r] = um[r];
                    um[r] = nm;
                    leg_rescale(um[r], ump[r], km[r]);
                }
            }
            any_scaled |= act[r] && (kp[r] < 0 || (SPIN && km[r] < 0));
        }
        ++l;
        scaled = __any(any_scaled);
    }
    // Phase 2: every active lane is at true scale.
#pragma unroll 2
    for (; l <= a.lmax; ++l) {
        const double P = T[4 * l + 3];
        double2 g = G[l], c = C[l];
        if (m0) { g.y = 0.0; c.y = 0.0; }
        const double apr = (g.x - c.y) * P, api = (g.y + c.x) * P;
        const double amr = (g.x + c.y) * P, ami = (c.x - g.y) * P;
        const double nA = T[4 * l], ApB = T[4 * l + 1], AmB = T[4 * l + 2];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            fpr[r] = fma(apr, up[r], fpr[r]);
            fpi[r] = fma(api, up[r], fpi[r]);
            if (SPIN) {
                fmr[r] = fma(amr, um[r], fmr[r]);
                fmi[r] = fma(ami, um[r], fmi[r]);
            } else {
                fmr[r] = fma(amr, up[r], fmr[r]);
                fmi[r] = fma(ami, up[r], fmi[r]);
            }
            double np = fma(fma(nA, y[r], ApB), up[r], -upp[r]);
            upp[r] = up[r];
            up[r] = np;
            if (SPIN) {
                double nm = fma(fma(nA, y[r], AmB), um[r], -ump[r]);
                ump[r] = um[r];
                um[r] = nm;
            }
        }
    }
    const double sgn_neg = (s & 1) ? 1.0 : -1.0;  // -(-1)^s
    double2 *Fp = reinterpret_cast<double2 *>(a.F) + (int64_t)(a.mmax + m) * a.nring;
    double2 *Fm = reinterpret_cast<double2 *>(a.F) + (int64_t)(a.mmax - m) * a.nring;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!act[r]) continue;
        int j = it.jb + r * 64 + lane;
        Fp[j] = make_double2(-fpr[r], -fpi[r]);
        if (!m0) Fm[j] = make_double2(sgn_neg * fmr[r], sgn_neg * fmi[r]);
    }
}

// Number of l per reduction chunk of the adjoint.
constexpr int kAdjChunk = 8;

template <int R, bool SPIN>
__global__ __launch_bounds__(64) void k_leg_adjoint(LegArgs a) {
    __shared__ double red[kAdjChunk][4][65];
    const int idx = leg_item_index(blockIdx.x, a.group);
    if (idx >= a.nitems) return;
    const LegItem it = a.items[idx];
    if (it.je <= it.jb) return;
    const int m = it.m, s = a.spin, lane = threadIdx.x;
    const int l0 = m > s ? m : s;
    if (l0 > a.lmax) return;

    double y[R], up[R], upp[R], um[R], ump[R];
    double fpr[R], fpi[R], fmr[R], fmi[R];
    int kp[R], km[R];
    bool act[R];
    const double kmant = a.kmant[m];
    const int kexp = a.kexp[m];
    const double2 *Fp = reinterpret_cast<const double2 *>(a.F) + (int64_t)(a.mmax + m) * a.nring;
    const double2 *Fm = reinterpret_cast<const double2 *>(a.F) + (int64_t)(a.mmax - m) * a.nring;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int j = it.jb + r * 64 + lane;
        act[r] = (j < it.je) && (a.ring_mmax[j] >= m);
        y[r] = 0.0;
        up[r] = um[r] = upp[r] = ump[r] = 0.0;
        kp[r] = km[r] = 0;
        fpr[r] = fpi[r] = fmr[r] = fmi[r] = 0.0;
        if (act[r]) {
            y[r] = a.ring_y[j];
            leg_seed(kmant, kexp, m, s, a.ring_ch[j], a.ring_sh[j], up[r], kp[r], um[r], km[r]);
            if (!SPIN) { um[r] = up[r]; km[r] = kp[r]; }
            double2 vp = Fp[j], vm = Fm[j];
            fpr[r] = vp.x;
            fpi[r] = vp.y;
            fmr[r] = vm.x;
            fmi[r] = -vm.y;  // conj F'(-m)
        }
    }
    const int64_t base = (int64_t)m * (2 * a.lmax + 1 - m) / 2;
    const double *T = a.coef + 4 * base;
    const double sgn_s = (s & 1) ? -1.0 : 1.0;
    double *out = a.alm_out;

    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= act[r] && (kp[r] < 0 || km[r] < 0);
    scaled = __any(scaled);

    for (int lc = l0; lc <= a.lmax; lc += kAdjChunk) {
        for (int t = 0; t < kAdjChunk; ++t) {
            const int l = lc + t;
            double pa_r = 0.0, pa_i = 0.0, pb_r = 0.0, pb_i = 0.0;
            if (l <= a.lmax) {
                const double nA = T[4 * l], ApB = T[4 * l + 1], AmB = T[4 * l + 2];
                const bool step = l < a.lmax;
                bool any_scaled = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double vp = up[r], vm = SPIN ? um[r] : up[r];
                    if (scaled) {
                        vp = kp[r] == 0 ? vp : 0.0;
                        vm = (SPIN ? km[r] : kp[r]) == 0 ? vm : 0.0;
                    }
                    pa_r = fma(vp, fpr[r], pa_r);
                    pa_i = fma(vp, fpi[r], pa_i);
                    pb_r = fma(vm, fmr[r], pb_r);
                    pb_i = fma(vm, fmi[r], pb_i);
                    if (step) {
                        double np = fma(fma(nA, y[r], ApB), up[r], -upp[r]);
                        upp[r] = up[r];
                        up[r] = np;
                        if (SPIN) {
                            double nm = fma(fma(nA, y[r], AmB), um[r], -ump[r]);
                            ump[r] = um[r];
                            um[r] = nm;
                        }
                        if (scaled) {
                            leg_rescale(up[r], upp[r], kp[r]);
                            if (SPIN) leg_rescale(um[r], ump[r], km[r]);
                            any_scaled |= act[r] && (kp[r] < 0 || (SPIN && km[r] < 0));
                        }
                    }
                }
                if (scaled) scaled = __any(any_scaled);
            }
            red[t][0][lane] = pa_r;
            red[t][1][lane] = pa_i;
            red[t][2][lane] = pb_r;
            red[t][3][lane] = pb_i;
        }
        __syncthreads();
        // lane -> (l offset t, component c, half h); each half sums 32 lanes.
        const int o = lane & 31, h = lane >> 5;
        const int t = o >> 2, c = o & 3;
        double sum = 0.0;
#pragma unroll 8
        for (int i = 0; i < 32; ++i) sum += red[t][c][32 * h + i];
        sum += __shfl_xor(sum, 32);
        const double s0 = __shfl(sum, (lane & ~3) | 0);
        const double s1 = __shfl(sum, (lane & ~3) | 1);
        const double s2 = __shfl(sum, (lane & ~3) | 2);
        const double s3 = __shfl(sum, (lane & ~3) | 3);
        const int l = lc + t;
        if (h == 0 && l <= a.lmax) {
            const double P = T[4 * l + 3];
            double v;
            int64_t k = base + l;
            double *dst;
            if (c == 0) { v = -0.5 * P * (s0 + sgn_s * s2); dst = out + 2 * k; }
            else if (c == 1) { v = -0.5 * P * (s1 + sgn_s * s3); dst = out + 2 * k + 1; }
            else if (c == 2) { v = -0.5 * P * (s1 - sgn_s * s3); dst = out + 2 * (a.nalm + k); }
            else { v = 0.5 * P * (s0 - sgn_s * s2); dst = out + 2 * (a.nalm + k) + 1; }
            // Im g~_l0 and Im c~_l0 vanish exactly (reality condition).
            if (!(m == 0 && (c & 1))) atomicAdd(dst, v);
        }
        __syncthreads();
    }
}

template <int R>
static hipError_t leg_launch(bool adjoint, const psht_plan_s &p, const void *alm, double *F, hipStream_t st) {
    const Geometry &g = p.g;
    LegArgs a;
    a.items = p.d_leg_items;
    a.nitems = p.n_leg_items;
    a.group = (g.nring + 64 * R - 1) / (64 * R);
    a.coef = p.leg->d_coef;
    a.kmant = p.leg->d_kmant;
    a.kexp = p.leg->d_kexp;
    a.ring_y = p.d_ring_y;
    a.ring_ch = p.d_ring_ch;
    a.ring_sh = p.d_ring_sh;
    a.ring_mmax = p.d_ring_mmax;
    a.nring = g.nring;
    a.lmax = g.lmax;
    a.spin = g.spin;
    a.mmax = g.mmax;
    a.nalm = (int64_t)(g.lmax + 1) * (g.lmax + 2) / 2;
    a.alm = static_cast<const double *>(alm);
    a.alm_out = static_cast<double *>(const_cast<void *>(alm));
    a.F = F;
    // the item list is padded to a multiple of 8 * group
    dim3 grid(p.n_leg_items), block(64);
    if (p.n_leg_items == 0) return hipSuccess;
    if (!adjoint) {
        if (g.spin) hipLaunchKernelGGL((k_leg_synth<R, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_leg_synth<R, false>), grid, block, 0, st, a);
    } else {
        if (g.spin) hipLaunchKernelGGL((k_leg_adjoint<R, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_leg_adjoint<R, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

constexpr int kLegR = 4;

hipError_t launch_leg_synth(const psht_plan_s &p, const void *alm, double *F, hipStream_t st) {
    return leg_launch<kLegR>(false, p, alm, F, st);
}

hipError_t launch_leg_adjoint(const psht_plan_s &p, const double *F, void *alm, hipStream_t st) {
    return leg_launch<kLegR>(true, p, alm, const_cast<double *>(F), st);
}

int leg_rings_per_item() { return 64 * kLegR; }

}  // namespace psht
