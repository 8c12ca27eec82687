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
// lane owns R rings (registers) and runs the recurrence in l.  The per-(l, m)
// recurrence coefficients and coefficient combinations are wave-uniform: they
// are staged through LDS one chunk ahead of their use.  The work items of one
// m run on one XCD so they share its L2.
//
// Values below the double range (see leg_common.h) occur only near the start
// of the l range of the rings where m is close to the cut-off; while any lane
// of the wave carries one, the wave runs blocks of 8 steps with masked
// accumulation and renormalises between blocks (8 steps grow a value by far
// less than the 2^800 of headroom above the renormalisation threshold).
#include <cstdlib>

#include "lane_ops.h"
#include "leg_common.h"
#include "psht_internal.h"

namespace psht {

struct LegArgs {
    const LegItem *items;
    int nitems;
    int group;  // items per order m
    const double4 *coef;  // {-A, A + B, A - B, P} per (l, m)
    const double *kmant;
    const int32_t *kexp;
    const double *ring_y, *ring_ch, *ring_sh;
    const int32_t *ring_mmax;
    int nring, lmax, spin, mmax;
    int64_t nalm;
    const double2 *g, *c;  // synthesis input: g_lm and c_lm, complex [nalm] each
    double *alm_out;   // adjoint output, complex [2][nalm]
    double *F;         // complex [2 mmax + 1][nring]: synthesis output / adjoint input
    double mscale;     // extra factor on the inputs (synthesis) or outputs (adjoint) of order m >= 1
};

// Block -> item map: the `group` items of one order m run on the same XCD
// (blocks are dealt round-robin to the 8 XCDs), and every XCD starts with the
// low orders, which carry the most work.
__device__ inline int leg_item_index(int bid, int group) {
    int xcd = bid & 7, k = bid >> 3;
    int q = k / group, i = k - q * group;
    return (xcd + 8 * q) * group + i;
}

// Branch-free renormalisation of a scaled pair (see leg_common.h).
__device__ inline void rescale_sel(double &cur, double &prev, int &k) {
    const bool big = (k < 0) && (fabs(cur) > PSHT_RESCALE_HI);
    const double f = big ? PSHT_RESCALE_FACTOR : 1.0;
    cur *= f;
    prev *= f;
    k += big ? 1 : 0;
}

template <int R, bool SPIN> struct LegState {
    double y[R], up[R], upp[R], um[R], ump[R];
    int kp[R], km[R];
    bool act[R];
};

// Seeds of the R rings of this lane for order m.
template <int R, bool SPIN>
__device__ inline void leg_init(const LegArgs &a, const LegItem &it, int lane, LegState<R, SPIN> &S) {
    const int m = it.m, s = a.spin;
    const double kmant = a.kmant[m];
    const int kexp = a.kexp[m];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = it.jb + r * 64 + lane;
        S.act[r] = (j < it.je) && (a.ring_mmax[j] >= m);
        S.y[r] = 0.0;
        S.up[r] = S.um[r] = S.upp[r] = S.ump[r] = 0.0;
        S.kp[r] = S.km[r] = 0;
        if (S.act[r]) {
            S.y[r] = a.ring_y[j];
            leg_seed(kmant, kexp, m, s, a.ring_ch[j], a.ring_sh[j], S.up[r], S.kp[r], S.um[r], S.km[r]);
            if (!SPIN) {
                S.um[r] = S.up[r];
                S.km[r] = S.kp[r];
            }
        }
    }
}

// The R rings of this lane for order m, rings [jb + 64 r + lane] below je,
// from recurrence states stored at plan time: the state of ring j at index
// soff + (j - jb), {mu+_l, mu+_{l-1}, mu-_l, mu-_{l-1}} and the scales {k+, k-}.
template <int R, bool SPIN>
__device__ inline void leg_init_stored(const LegArgs &a, int m, int jb, int je, int lane, const double4 *st_mu,
                                       const int2 *st_k, int64_t soff, LegState<R, SPIN> &S) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = jb + r * 64 + lane;
        S.act[r] = (j < je) && (a.ring_mmax[j] >= m);
        S.y[r] = 0.0;
        S.up[r] = S.upp[r] = S.um[r] = S.ump[r] = 0.0;
        S.kp[r] = S.km[r] = 0;
        if (S.act[r]) {
            const int64_t q = soff + (j - jb);
            const double4 v = st_mu[q];
            const int2 k = st_k[q];
            S.y[r] = a.ring_y[j];
            S.up[r] = v.x;
            S.upp[r] = v.y;
            S.kp[r] = k.x;
            if (SPIN) {
                S.um[r] = v.z;
                S.ump[r] = v.w;
                S.km[r] = k.y;
            } else {
                S.um[r] = v.x;
                S.km[r] = k.x;
            }
        }
    }
}

template <int R, bool SPIN> __device__ inline bool leg_any_scaled(const LegState<R, SPIN> &S) {
    bool sc = false;
#pragma unroll
    for (int r = 0; r < R; ++r) sc |= S.act[r] && (S.kp[r] < 0 || (SPIN && S.km[r] < 0));
    return __any(sc);
}

// mu_{l+1} = ((A +/- B) - A y) mu_l - mu_{l-1}
template <int R, bool SPIN> __device__ inline void leg_advance(LegState<R, SPIN> &S, const double4 t) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double np = fma(fma(t.x, S.y[r], t.y), S.up[r], -S.upp[r]);
        S.upp[r] = S.up[r];
        S.up[r] = np;
        if (SPIN) {
            const double nm = fma(fma(t.x, S.y[r], t.z), S.um[r], -S.ump[r]);
            S.ump[r] = S.um[r];
            S.um[r] = nm;
        }
    }
}

template <int R, bool SPIN> __device__ inline void leg_renorm(LegState<R, SPIN> &S) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rescale_sel(S.up[r], S.upp[r], S.kp[r]);
        if (SPIN) rescale_sel(S.um[r], S.ump[r], S.km[r]);
    }
}

// The coefficient stream of one order m ({-A, A+B, A-B, P} and, for the
// synthesis, the combinations Q) is staged through LDS in chunks of kStage
// steps: every lane loads one 32-byte entry of the next chunk (coalesced)
// while the current chunk is computed from wave-uniform (broadcast) LDS reads.
constexpr int kStage = 32;

// Entry `lane` of the chunk starting at c: the recurrence table, zero past lmax.
__device__ inline double4 stage_entry(const double4 *T4, int c, int lmax, int lane) {
    const int l = c + (lane & 31);
    return l <= lmax ? T4[l] : make_double4(0.0, 0.0, 0.0, 0.0);
}

// The synthesis multiplies lambda+ by P (g + i c) and lambda- by P (conj g +
// i conj c) (Sec. I, with lambda_l = P_l mu_l): the four real combinations
// P {g_r - c_i, g_i + c_r, g_r + c_i, c_r - g_i} of order m at degree l
// (coefficient index k), with the imaginary parts of the m = 0 coefficients
// dropped and the inputs of order m >= 1 scaled by mscale.
__device__ inline double4 synth_combo(const double2 *g, const double2 *c, const double4 *coef, int64_t k, int m,
                                      double mscale) {
    double2 a = g[k], b = c[k];
    double P = coef[k].w;
    if (m == 0) {
        a.y = 0.0;
        b.y = 0.0;
    } else {
        P *= mscale;
    }
    return make_double4((a.x - b.y) * P, (a.y + b.x) * P, (a.x + b.y) * P, (b.x - a.y) * P);
}

// Synthesis staging: lanes 0..31 read the recurrence table, lanes 32..63 form
// the coefficient combinations of the same 32 degrees.
__device__ inline double4 stage_entry_synth(const LegArgs &a, const double4 *T4, int64_t base, int m, int c,
                                            int lmax, int lane) {
    const int l = c + (lane & 31);
    double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
    if (l <= lmax) {
        if (lane < 32) v = T4[l];
        else v = synth_combo(a.g, a.c, a.coef, base + l, m, a.mscale);
    }
    return v;
}

// Steps t in [t0, t1) of a staged chunk starting at l = c (t1 - t0 <= 8):
// accumulate lambda_l into the ring sums, then advance the recurrence.
template <int R, bool SPIN>
__device__ inline void synth_steps(LegState<R, SPIN> &S, double *fpr, double *fpi, double *fmr, double *fmi,
                                   const double4 *sT, const double4 *sQ, int t0, int t1, int c, int lmax) {
#pragma unroll 2
    for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        if (t < t1) {
            const double4 q = sQ[t];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double vp = S.up[r], vm = SPIN ? S.um[r] : S.up[r];
                fpr[r] = fma(q.x, vp, fpr[r]);
                fpi[r] = fma(q.y, vp, fpi[r]);
                fmr[r] = fma(q.z, vm, fmr[r]);
                fmi[r] = fma(q.w, vm, fmi[r]);
            }
            if (c + t < lmax) leg_advance<R, SPIN>(S, sT[t]);
        }
    }
}

// True when some active ring of the wave holds an unscaled value; otherwise
// every term of the current steps is exactly zero and only the recurrence
// has to run.
template <int R, bool SPIN> __device__ inline bool leg_live(const LegState<R, SPIN> &S) {
    bool lv = false;
#pragma unroll
    for (int r = 0; r < R; ++r) lv |= S.act[r] && (S.kp[r] == 0 || (SPIN && S.km[r] == 0));
    return __any(lv);
}

// Recurrence alone over the steps t in [t0, t1) of a staged chunk; FULL: the
// NS steps from t0 all advance (no guards).
template <int R, bool SPIN, bool FULL, int NS>
__device__ inline void advance_steps(LegState<R, SPIN> &S, const double4 *sT, int t0, int t1, int c, int lmax) {
    if (FULL) {
#pragma unroll 2
        for (int u = 0; u < NS; ++u) leg_advance<R, SPIN>(S, sT[t0 + u]);
    } else {
        for (int t = t0; t < t1; ++t)
            if (c + t < lmax) leg_advance<R, SPIN>(S, sT[t]);
    }
}

// Steps b..b+7 of a staged chunk when all eight advance: fully unrolled, no guards.
template <int R, bool SPIN>
__device__ inline void synth_steps8(LegState<R, SPIN> &S, double *fpr, double *fpi, double *fmr, double *fmi,
                                    const double4 *sT, const double4 *sQ, int b) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double4 q = sQ[b + u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double vp = S.up[r], vm = SPIN ? S.um[r] : S.up[r];
            fpr[r] = fma(q.x, vp, fpr[r]);
            fpi[r] = fma(q.y, vp, fpi[r]);
            fmr[r] = fma(q.z, vm, fmr[r]);
            fmi[r] = fma(q.w, vm, fmi[r]);
        }
        leg_advance<R, SPIN>(S, sT[b + u]);
    }
}

// Scaled values in the synthesis.  The sums of a ring take its stored values
// unmasked; while the ring's scale k is negative those terms are not its true
// (negligible, below 2^-312) ones, so the sums restart when k reaches 0 and
// are cleared at the end if it never does (synth_clear_scaled).
template <int R, bool SPIN>
__device__ inline void synth_renorm(LegState<R, SPIN> &S, double *fpr, double *fpi, double *fmr, double *fmi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kp0 = S.kp[r];
        rescale_sel(S.up[r], S.upp[r], S.kp[r]);
        const bool rp = kp0 < 0 && S.kp[r] == 0;
        fpr[r] = rp ? 0.0 : fpr[r];
        fpi[r] = rp ? 0.0 : fpi[r];
        bool rm = rp;
        if (SPIN) {
            const int km0 = S.km[r];
            rescale_sel(S.um[r], S.ump[r], S.km[r]);
            rm = km0 < 0 && S.km[r] == 0;
        }
        fmr[r] = rm ? 0.0 : fmr[r];
        fmi[r] = rm ? 0.0 : fmi[r];
    }
}

template <int R, bool SPIN>
__device__ inline void synth_clear_scaled(const LegState<R, SPIN> &S, double *fpr, double *fpi, double *fmr,
                                          double *fmi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (S.kp[r] < 0) fpr[r] = fpi[r] = 0.0;
        if ((SPIN ? S.km[r] : S.kp[r]) < 0) fmr[r] = fmi[r] = 0.0;
    }
}

// One work item of the synthesis with R rings per lane (the item holds at
// most 64 R rings): the sums over the degrees l0 .. lend of order m, where the
// recurrence starts from the seed at l0 = max(m, s) (soff < 0) or from the
// states stored for l0 (soff >= 0, see leg_init_stored), written to the F
// layout at Fout.
template <int R, bool SPIN>
__device__ inline void leg_synth_item(const LegArgs &a, const LegItem &it, int l0, int lend, int64_t soff,
                                      const double4 *st_mu, const int2 *st_k, double *Fout,
                                      double4 (*sbuf)[2][kStage + 1]) {
    const int m = it.m, s = a.spin, lane = threadIdx.x;
    if (l0 > lend) return;

    const int64_t base = (int64_t)m * (2 * a.lmax + 1 - m) / 2;
    const double4 *T4 = a.coef + base;
    sbuf[0][lane >> 5][lane & 31] = stage_entry_synth(a, T4, base, m, l0, lend, lane);

    LegState<R, SPIN> S;
    if (soff < 0) leg_init<R, SPIN>(a, it, lane, S);
    else leg_init_stored<R, SPIN>(a, m, it.jb, it.je, lane, st_mu, st_k, soff, S);
    double fpr[R], fpi[R], fmr[R], fmi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) fpr[r] = fpi[r] = fmr[r] = fmi[r] = 0.0;
    bool scaled = leg_any_scaled<R, SPIN>(S);
    __syncthreads();

    int slot = 0;
    for (int c = l0; c <= lend; c += kStage) {
        const bool has_next = c + kStage <= lend;
        double4 nv;
        if (has_next) nv = stage_entry_synth(a, T4, base, m, c + kStage, lend, lane);
        const double4 *sT = sbuf[slot][0], *sQ = sbuf[slot][1];
        const int n = min(kStage, lend + 1 - c);
        if (!scaled && has_next) {
            // Full chunk, every step advances, no lane scaled: no per-step guards.
            // The coefficients of step t + 1 are read while step t computes.
            double4 q = sQ[0], tc = sT[0];
#pragma unroll 4
            for (int t = 0; t < kStage; ++t) {
                double4 qn = sQ[t + 1], tn;
                tn.x = sT[t + 1].x;
                tn.y = sT[t + 1].y;
                tn.z = sT[t + 1].z;
                tn.w = 0.0;
                // keep these loads ahead of the arithmetic of step t
                __builtin_amdgcn_sched_barrier(0);
                // Independent work first, dependent updates last, so that no
                // FMA waits for the one just before it: the step coefficients
                // (A +/- B) - A y of every ring, the accumulation of lambda_l,
                // then the recurrence updates that use both.
                double cpl[R], cmi[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cpl[r] = fma(tc.x, S.y[r], tc.y);
                    if (SPIN) cmi[r] = fma(tc.x, S.y[r], tc.z);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double vm = SPIN ? S.um[r] : S.up[r];
                    fpr[r] = fma(q.x, S.up[r], fpr[r]);
                    fpi[r] = fma(q.y, S.up[r], fpi[r]);
                    fmr[r] = fma(q.z, vm, fmr[r]);
                    fmi[r] = fma(q.w, vm, fmi[r]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double np = fma(cpl[r], S.up[r], -S.upp[r]);
                    S.upp[r] = S.up[r];
                    S.up[r] = np;
                    if (SPIN) {
                        const double nm = fma(cmi[r], S.um[r], -S.ump[r]);
                        S.ump[r] = S.um[r];
                        S.um[r] = nm;
                    }
                }
                q = qn;
                tc = tn;
            }
        } else for (int b = 0; b < n; b += 8) {
            const int e = min(b + 8, n);
            const bool full = c + b + 8 <= lend;  // all eight steps exist and advance
            if (scaled && !leg_live<R, SPIN>(S)) {
                // no active ring in the double range yet: recurrence only
                if (full) advance_steps<R, SPIN, true, 8>(S, sT, b, e, c, lend);
                else advance_steps<R, SPIN, false, 8>(S, sT, b, e, c, lend);
            } else if (full) {
                synth_steps8<R, SPIN>(S, fpr, fpi, fmr, fmi, sT, sQ, b);
            } else {
                synth_steps<R, SPIN>(S, fpr, fpi, fmr, fmi, sT, sQ, b, e, c, lend);
            }
            if (scaled) {
                synth_renorm<R, SPIN>(S, fpr, fpi, fmr, fmi);
                scaled = leg_any_scaled<R, SPIN>(S);
            }
        }
        if (has_next) sbuf[slot ^ 1][lane >> 5][lane & 31] = nv;
        __syncthreads();
        slot ^= 1;
    }

    synth_clear_scaled<R, SPIN>(S, fpr, fpi, fmr, fmi);
    const double sgn_neg = (s & 1) ? 1.0 : -1.0;  // -(-1)^s
    double2 *Fp = reinterpret_cast<double2 *>(Fout) + (int64_t)(a.mmax + m) * a.nring;
    double2 *Fm = reinterpret_cast<double2 *>(Fout) + (int64_t)(a.mmax - m) * a.nring;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!S.act[r]) continue;
        const int j = it.jb + r * 64 + lane;
        Fp[j] = make_double2(-fpr[r], -fpi[r]);
        if (m != 0) Fm[j] = make_double2(sgn_neg * fmr[r], sgn_neg * fmi[r]);
    }
}

// An item with at most 64 rings (the remainder of an order's ring range)
// runs the one-ring-per-lane body, at half the work of the R = 2 body.
template <int R, bool SPIN>
__global__ __launch_bounds__(64) void k_leg_synth(LegArgs a) {
    __shared__ double4 sbuf[2][2][kStage + 1];  // one spare entry: the pipelined loop reads one step ahead
    const int idx = leg_item_index(blockIdx.x, a.group);
    if (idx >= a.nitems) return;
    const LegItem it = a.items[idx];
    if (it.je <= it.jb) return;
    const int l0 = it.m > a.spin ? it.m : a.spin;
    if (R > 1 && it.je - it.jb <= 64)
        leg_synth_item<1, SPIN>(a, it, l0, a.lmax, -1, nullptr, nullptr, a.F, sbuf);
    else
        leg_synth_item<R, SPIN>(a, it, l0, a.lmax, -1, nullptr, nullptr, a.F, sbuf);
}

// Degree-segmented synthesis (plans whose items would not fill the GPU): an
// item sums the degrees [la, lb) of its order, starting from the recurrence
// state stored at plan time for la (every segment start is one of the
// adjoint's), into F (segment 0) or into the partial copy of F of its segment
// (segment k >= 1 at parts + (k - 1) part_stride doubles); k_synth_parts_sum
// then adds the partials into F.
struct SynSegArgs {
    LegArgs a;
    const SynSegItem *items;
    int nitems;
    const double4 *st_mu;
    const int2 *st_k;
    double *parts;
    int64_t part_stride;
};

template <int R, bool SPIN>
__global__ __launch_bounds__(64) void k_leg_synth_seg(SynSegArgs A) {
    __shared__ double4 sbuf[2][2][kStage + 1];
    if ((int)blockIdx.x >= A.nitems) return;
    const SynSegItem q = A.items[blockIdx.x];
    if (q.je <= q.jb) return;
    const LegItem it{q.m, q.jb, q.je};
    double *F = q.part == 0 ? A.a.F : A.parts + (int64_t)(q.part - 1) * A.part_stride;
    if (R > 1 && q.je - q.jb <= 64)
        leg_synth_item<1, SPIN>(A.a, it, q.la, q.lb - 1, q.soff, A.st_mu, A.st_k, F, sbuf);
    else
        leg_synth_item<R, SPIN>(A.a, it, q.la, q.lb - 1, q.soff, A.st_mu, A.st_k, F, sbuf);
}

// F(m)[j] += the partials of segments 1 .. nseg_m - 1 for every written entry
// (|m| <= ring_mmax[j] and order |m| has degrees), nseg_m = ceil((lmax + 1 -
// max(|m|, s)) / S); one thread per entry of F, rings contiguous.
__global__ __launch_bounds__(256) void k_synth_parts_sum(double2 *F, const double2 *parts, int64_t part_stride,
                                                         const int32_t *ring_mmax, int nring, int mmax, int lmax,
                                                         int spin, int S) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)(2 * mmax + 1) * nring;
    if (e >= n) return;
    const int mi = (int)(e / nring), j = (int)(e - (int64_t)mi * nring);
    const int m = mi >= mmax ? mi - mmax : mmax - mi;
    const int l0 = m > spin ? m : spin;
    if (l0 > lmax || ring_mmax[j] < m) return;
    const int nseg = (lmax + 1 - l0 + S - 1) / S;
    if (nseg < 2) return;
    double2 acc = F[e];
    for (int k = 1; k < nseg; ++k) {
        const double2 v = parts[(int64_t)(k - 1) * part_stride + e];
        acc.x += v.x;
        acc.y += v.y;
    }
    F[e] = acc;
}

// ---------------------------------------------------------------- adjoint


// Fold of one l-step's four lane sums c0..c3 (Re and Im of the + and - sums)
// into the transposed reduction, as soon as they are computed: a 32-lane swap
// keeps component c + 2 bit5(i) in lane i, summed over lanes i and i ^ 32; the
// two steps u and u + 1 then share a 16-lane swap that keeps step
// u + bit4(i), summed over {i, i ^ 16, i ^ 32, i ^ 48}; the value of step
// pair u / 2 and component parity c & 1 goes to red[row][2 (u / 2) + (c & 1)][col].
template <int CH>
__device__ inline void adj_fold(int u, double c0, double c1, double c2, double c3, double *w, double (*red)[CH][17],
                                int row, int col) {
    swap32(c0, c2);
    c0 += c2;
    swap32(c1, c3);
    c1 += c3;
    const int p = u >> 1;
    if ((u & 1) == 0) {
        w[0] = c0;
        w[1] = c1;
    } else {
        // the pair's two values are final: to LDS at once, so that only two
        // values per lane are live across the block
        swap16(w[0], c0);
        swap16(w[1], c1);
        red[row][2 * p][col] = w[0] + c0;
        red[row][2 * p + 1][col] = w[1] + c1;
    }
}

// Scaled values in the adjoint.  A ring's map values enter its partial sums
// only while its scale k is 0: they are held at zero while k < 0 and loaded
// when k reaches 0, so the stored (scaled) values need no mask.
template <int R, bool SPIN>
__device__ inline void adj_load_f(const LegState<R, SPIN> &S, const double2 *Fp, const double2 *Fm, int j0,
                                  int lane, double *fpr, double *fpi, double *fmr, double *fmi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        fpr[r] = fpi[r] = fmr[r] = fmi[r] = 0.0;
        if (S.act[r]) {
            const int j = j0 + r * 64 + lane;
            if (S.kp[r] == 0) {
                const double2 vp = Fp[j];
                fpr[r] = vp.x;
                fpi[r] = vp.y;
            }
            if ((SPIN ? S.km[r] : S.kp[r]) == 0) {
                const double2 vm = Fm[j];
                fmr[r] = vm.x;
                fmi[r] = -vm.y;  // conj F'(-m); for m = 0 the same column
            }
        }
    }
}

template <int R, bool SPIN>
__device__ inline void adj_renorm(LegState<R, SPIN> &S, const double2 *Fp, const double2 *Fm, int j0, int lane,
                                  double *fpr, double *fpi, double *fmr, double *fmi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kp0 = S.kp[r], km0 = SPIN ? S.km[r] : 0;
        rescale_sel(S.up[r], S.upp[r], S.kp[r]);
        if (SPIN) rescale_sel(S.um[r], S.ump[r], S.km[r]);
        const int j = j0 + r * 64 + lane;
        if (kp0 < 0 && S.kp[r] == 0) {
            const double2 vp = Fp[j];
            fpr[r] = vp.x;
            fpi[r] = vp.y;
        }
        if (SPIN ? (km0 < 0 && S.km[r] == 0) : (kp0 < 0 && S.kp[r] == 0)) {
            const double2 vm = Fm[j];
            fmr[r] = vm.x;
            fmi[r] = -vm.y;
        }
    }
}

// ------------------------------------------------------- segmented adjoint
//
// Beyond its FMAs, the adjoint pays for reducing every l-step's four partial
// sums over the 64 lanes (adj_fold and the LDS output stage): about 13
// instructions per step and wave, whatever the number of rings a lane holds.
// More rings per lane amortise that, but an order's rings then make few long
// items (one or two per order), and the longest items set the time.  Items
// cut in l restore the balance without repeating any recurrence: the item
// (m, [la, lb)) starts from the recurrence state at l = la that the plan
// stored for every ring and segment start (k_leg_adj_states).  The waves of a
// workgroup hold disjoint rings of the order, fold their partial sums into
// LDS, and wave 0 completes them over the waves and writes each output once
// with a plain store (no atomics, no prior clear of the output).

constexpr int kAdjRedDoubles = 4 * 8 * 17;  // one wave's fold area per 8-step block

struct AdjArgs {
    LegArgs a;
    const AdjItem *items;
    int nitems;
    const double4 *st_mu;
    const int2 *st_k;
    bool accumulate;  // ring groups: add into the (cleared) output instead of storing
};

// Rings [j0 + 64 r + lane] of order m: seeds (first segment) or the stored states.
template <int R, bool SPIN>
__device__ inline void adj_seg_init(const AdjArgs &A, const AdjItem &it, int j0, int lane, LegState<R, SPIN> &S) {
    if (it.soff < 0) {
        const LegItem li{it.m, j0, it.je};
        leg_init<R, SPIN>(A.a, li, lane, S);
        return;
    }
    leg_init_stored<R, SPIN>(A.a, it.m, j0, it.je, lane, A.st_mu, A.st_k, it.soff + (j0 - it.jb), S);
}

// Zero outputs of order m for l in [l_from, l_to) (wave 0's lanes).
__device__ inline void adj_zero_range(const LegArgs &a, int64_t base, int l_from, int l_to, int lane) {
    for (int l = l_from + lane; l < l_to; l += 64) {
        const int64_t kk = base + l;
        reinterpret_cast<double2 *>(a.alm_out)[kk] = make_double2(0.0, 0.0);
        reinterpret_cast<double2 *>(a.alm_out)[a.nalm + kk] = make_double2(0.0, 0.0);
    }
}

// Eight steps from b of a staged chunk, all advancing (steps past the item's
// last degree compute with zero-padded table entries; their folded values are
// never written out): per ring, the step coefficients, the partial sums and
// the recurrence update, folded step by step (adj_fold).
template <int R, bool SPIN>
__device__ inline void adj_seg_block(LegState<R, SPIN> &S, const double4 *sT, int b, const double *fpr,
                                     const double *fpi, const double *fmr, const double *fmi, double (*red)[8][17],
                                     int row, int col) {
    double w[2];
    double3 tn = make_double3(sT[b].x, sT[b].y, sT[b].z);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double3 tc = tn;
        if (u + 1 < 8) tn = make_double3(sT[b + u + 1].x, sT[b + u + 1].y, sT[b + u + 1].z);
        double pa_r = 0.0, pa_i = 0.0, pb_r = 0.0, pb_i = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double vp = S.up[r], vm = SPIN ? S.um[r] : S.up[r];
            pa_r = fma(vp, fpr[r], pa_r);
            pa_i = fma(vp, fpi[r], pa_i);
            pb_r = fma(vm, fmr[r], pb_r);
            pb_i = fma(vm, fmi[r], pb_i);
            const double np = fma(fma(tc.x, S.y[r], tc.y), vp, -S.upp[r]);
            S.upp[r] = vp;
            S.up[r] = np;
            if (SPIN) {
                const double nm = fma(fma(tc.x, S.y[r], tc.z), vm, -S.ump[r]);
                S.ump[r] = vm;
                S.um[r] = nm;
            }
        }
        adj_fold<8>(u, pa_r, pa_i, pb_r, pb_i, w, red, row, col);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Workgroup barrier for LDS data only: waits for this wave's LDS operations,
// not for its outstanding global loads (the next table chunk stays in flight
// across the barrier), then s_barrier.
__device__ inline void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int R, bool SPIN>
__device__ void adj_seg_item(const AdjArgs &A, const AdjItem &it, int G, double4 (*sbuf)[kStage], double *redbase) {
    const LegArgs &a = A.a;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = it.m, s = a.spin, lmax = a.lmax;
    const int l0 = m > s ? m : s;
    const int la = it.la, lhi = it.lb - 1;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double4 *T4 = a.coef + base;
    if (threadIdx.x < 32) sbuf[0][threadIdx.x] = stage_entry(T4, la, lmax, threadIdx.x);
    if (wave == 0 && it.soff < 0) adj_zero_range(a, base, m, l0, lane);  // l < s: no such harmonic

    const int j0 = it.jb + wave * 64 * R;
    LegState<R, SPIN> S;
    adj_seg_init<R, SPIN>(A, it, j0, lane, S);
    double fpr[R], fpi[R], fmr[R], fmi[R];
    const double2 *Fp = reinterpret_cast<const double2 *>(a.F) + (int64_t)(a.mmax + m) * a.nring;
    const double2 *Fm = reinterpret_cast<const double2 *>(a.F) + (int64_t)(a.mmax - m) * a.nring;
    adj_load_f<R, SPIN>(S, Fp, Fm, j0, lane, fpr, fpi, fmr, fmi);
    const double sgn_s = (s & 1) ? -1.0 : 1.0;
    const int row = lane >> 4, col = lane & 15;
    bool scaled = leg_any_scaled<R, SPIN>(S);
    __syncthreads();

    int slot = 0, buf = 0;
    for (int c = la; c <= lhi; c += kStage) {
        const bool has_next = c + kStage <= lhi;
        double4 nv;
        if (has_next && threadIdx.x < 32) nv = stage_entry(T4, c + kStage, lmax, threadIdx.x);
        const double4 *sT = sbuf[slot];
        const int n = min(kStage, lhi + 1 - c);
        for (int b = 0; b < n; b += 8) {
            double(*red)[8][17] = reinterpret_cast<double(*)[8][17]>(redbase + (buf * G + wave) * kAdjRedDoubles);
            if (scaled && !leg_live<R, SPIN>(S)) {
                // every active ring of this wave is below the double range: its
                // partial sums are zero, only the recurrence runs
                advance_steps<R, SPIN, true, 8>(S, sT, b, n, c, lhi);
#pragma unroll
                for (int k = 0; k < 8; ++k) red[row][k][col] = 0.0;
            } else {
                adj_seg_block<R, SPIN>(S, sT, b, fpr, fpi, fmr, fmi, red, row, col);
            }
            if (scaled) {
                adj_renorm<R, SPIN>(S, Fp, Fm, j0, lane, fpr, fpi, fmr, fmi);
                scaled = leg_any_scaled<R, SPIN>(S);
            }
            // The fold areas of this block are double buffered: the next block
            // writes the other one, so one barrier per block suffices.
            lds_barrier();
            if (wave == 0) {
                // Step u, component c of wave g sits in row 2 (c >> 1) + (u & 1),
                // value 2 (u >> 1) + (c & 1) of the wave's fold area.  Lane
                // (u = lane >> 3, x = bit 2, h = lane & 3) adds columns 4h .. 4h + 3
                // of A_x and B_x over the waves, the lane quad completes the sums,
                // and lanes h = 0 and 1 write g~ and c~ of component x.
                const int u = lane >> 3, x = (lane >> 2) & 1, h = lane & 3;
                const int qa = u & 1, kv = 2 * (u >> 1) + x;
                double sa = 0.0, sb = 0.0;
                for (int g = 0; g < G; ++g) {
                    const double(*rg)[8][17] =
                        reinterpret_cast<const double(*)[8][17]>(redbase + (buf * G + g) * kAdjRedDoubles);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        sa += rg[qa][kv][4 * h + j];
                        sb += rg[qa + 2][kv][4 * h + j];
                    }
                }
                sa += quad_xor1(sa);
                sb += quad_xor1(sb);
                sa += quad_xor2(sa);
                sb += quad_xor2(sb);
                const int t = b + u;
                if (h < 2 && t < n) {
                    const int64_t kk = base + c + t;
                    const double hP = (m == 0 ? 0.5 : 0.5 * a.mscale) * sT[t].w;
                    // Im g~_l0 and Im c~_l0 vanish (reality condition)
                    const bool imag = h == 0 ? x == 1 : x == 0;
                    double val;
                    double *dst;
                    if (h == 0) {  // g~ = -hP (A + (-1)^s B), component x
                        val = -hP * (sa + sgn_s * sb);
                        dst = a.alm_out + 2 * kk + x;
                    } else {  // c~ = (i/2) P (A - (-1)^s B): Im from the real parts, Re from the imaginary ones
                        const double d = hP * (sa - sgn_s * sb);
                        val = x == 0 ? d : -d;
                        dst = a.alm_out + 2 * (a.nalm + kk) + (1 - x);
                    }
                    val = (m == 0 && imag) ? 0.0 : val;
                    if (A.accumulate) atomicAdd(dst, val);
                    else *dst = val;
                }
            }
            buf ^= 1;
        }
        if (has_next && threadIdx.x < 32) sbuf[slot ^ 1][threadIdx.x] = nv;
        lds_barrier();
        slot ^= 1;
    }
}

// One workgroup of G = blockDim.x / 64 waves per item (G = 1, 2 or 4, so that
// whole workgroups fill a CU's wave slots); rings per lane chosen per item
// (the waves of an item share it) up to RMAX.  About 34 VGPRs per ring: the
// RMAX = 6 kernel takes 245 (two waves per SIMD), the RMAX = 4 kernel is
// held to three waves per SIMD.
template <bool SPIN, int RMAX>
__device__ inline void adj_seg_dispatch(const AdjArgs &A) {
    __shared__ double4 sbuf[2][kStage];
    extern __shared__ double redbase[];  // fold areas [2][G][4][8][17]
    if ((int)blockIdx.x >= A.nitems) return;
    const AdjItem it = A.items[blockIdx.x];
    const int G = blockDim.x >> 6;
    switch (it.R) {
        case 0:
            // no active ring: the order's outputs are zero
            if (threadIdx.x < 64)
                adj_zero_range(A.a, (int64_t)it.m * (2 * A.a.lmax + 1 - it.m) / 2, it.la, it.lb, threadIdx.x);
            break;
        case 1: adj_seg_item<1, SPIN>(A, it, G, sbuf, redbase); break;
        case 2: adj_seg_item<2, SPIN>(A, it, G, sbuf, redbase); break;
        case 3: adj_seg_item<3, SPIN>(A, it, G, sbuf, redbase); break;
        case 4: adj_seg_item<4, SPIN>(A, it, G, sbuf, redbase); break;
        case 5: if constexpr (RMAX >= 5) adj_seg_item<5, SPIN>(A, it, G, sbuf, redbase); break;
        default: if constexpr (RMAX >= 6) adj_seg_item<6, SPIN>(A, it, G, sbuf, redbase); break;
    }
}

template <bool SPIN>
__global__ __launch_bounds__(256, 2) void k_leg_adj_seg6(AdjArgs A) { adj_seg_dispatch<SPIN, 6>(A); }
template <bool SPIN>
__global__ __launch_bounds__(256, 3) void k_leg_adj_seg4(AdjArgs A) { adj_seg_dispatch<SPIN, 4>(A); }

// Plan time: one lane per ring runs the recurrence of order m from its seed
// and stores (mu_l, mu_{l-1}) and the scales at every segment start
// l = l0 + k S, k >= 1.
template <bool SPIN>
__global__ __launch_bounds__(64) void k_leg_adj_states(LegArgs a, const StateItem *items, int nitems, double4 *st_mu,
                                                       int2 *st_k) {
    if ((int)blockIdx.x >= nitems) return;
    const StateItem it = items[blockIdx.x];
    const int j = it.j0 + (int)threadIdx.x;
    if (j >= it.je) return;
    const int m = it.m, s = a.spin, lmax = a.lmax;
    const int l0 = m > s ? m : s;
    const double y = a.ring_y[j];
    double up, um, upp = 0.0, ump = 0.0;
    int kp, km;
    leg_seed(a.kmant[m], a.kexp[m], m, s, a.ring_ch[j], a.ring_sh[j], up, kp, um, km);
    if (!SPIN) {
        um = up;
        km = kp;
    }
    const double4 *T4 = a.coef + (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int64_t nr = it.je - it.jb;
    const int lend = l0 + (it.nseg - 1) * it.S;
    int k = 1;
    for (int l = l0; l < lend && l < lmax; ++l) {
        const double4 t = T4[l];
        const double np = fma(fma(t.x, y, t.y), up, -upp);
        upp = up;
        up = np;
        leg_rescale(up, upp, kp);
        if (SPIN) {
            const double nm = fma(fma(t.x, y, t.z), um, -ump);
            ump = um;
            um = nm;
            leg_rescale(um, ump, km);
        }
        if (l + 1 == l0 + k * it.S) {
            const int64_t q = it.soff + (int64_t)(k - 1) * nr + (j - it.jb);
            st_mu[q] = SPIN ? make_double4(up, upp, um, ump) : make_double4(up, upp, up, upp);
            st_k[q] = make_int2(kp, SPIN ? km : kp);
            ++k;
        }
    }
}

// ------------------------------------------------------- batched maps (MFMA)
//
// nb <= 8 coefficient sets on one plan.  For one order m and a chunk of 64
// rings, the sums over l are the dense contraction
//   F_b(+m)[j] = -sum_l lambda+_l(theta_j) Z+_b[l],  Z+_b = P (g_b + i c_b),
//   F_b(-m)[j] = -(-1)^s sum_l lambda-_l(theta_j) Z-_b[l],
// i.e. (64 rings x L) times (L x 16 real columns: 8 maps x {Re, Im}) for each
// sign.  The recurrence runs once for all maps (one ring per lane); blocks of
// 4 consecutive l go through LDS to the A operand of v_mfma_f64_16x16x4f64
// (A[i][k] in lane i + 16 k: ring 16 q + i, l + k), the staged columns are the
// B operand (B[k][j] in lane j + 16 k) and D accumulates in registers (D[i][j]
// in lane j + 16 (i mod 4), register i / 4).

typedef double d4v __attribute__((ext_vector_type(4)));

struct LegBatchArgs {
    LegArgs a;           // work list of 64-ring chunks, tables, rings
    const char *alm0;    // coefficients (g, c) of map 0, complex [2][nalm]; map b at alm0 + b * alm_stride
    int64_t alm_stride;  // bytes
    char *F0;            // F of map 0; map b at F0 + b * stride
    int64_t stride;      // bytes between consecutive maps' F (their workspaces)
    int nb;              // maps in this launch, 1..8
};

// Register budget of two waves per SIMD: the accumulators then stay in VGPRs
// (a three-wave budget split them into AGPRs and copied them around every
// block); the compiler needs 162 VGPRs, the LDS (14 KB) allows 11 waves per CU.
template <bool SPIN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_leg_synth_mm(LegBatchArgs bt) {
    const LegArgs &a = bt.a;
    __shared__ double4 sT[2][kStage];
    // one buffer of coefficient columns: the next chunk waits in registers
    // (nz) until the current one is done, which keeps the LDS at 18 KB
    __shared__ double sZ[kStage][2][16];  // [l][sign][column]
    __shared__ double sL[2][4][64];          // [sign][k][ring]
    const int idx = leg_item_index(blockIdx.x, a.group);
    if (idx >= a.nitems) return;
    const LegItem it = a.items[idx];
    if (it.je <= it.jb) return;
    const int m = it.m, s = a.spin, lane = threadIdx.x;
    const int l0 = m > s ? m : s, lmax = a.lmax;
    if (l0 > lmax) return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double4 *T4 = a.coef + base;

    // Staging of a chunk of kStage steps from l = c: lanes 0..31 load the
    // recurrence table, every lane forms 4 (l, map) entries of the columns
    // (l = c + e / 8, map = e % 8) from the coefficients, zero past lmax and
    // past nb.  The loads of
    // the next chunk are issued before the current chunk is computed and
    // written to the other LDS slot after it.
    auto load_z = [&](int c, int e) {
        const int lo = e >> 3, b = e & 7, l = c + lo;
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        if (b < bt.nb && l <= lmax) {
            const double2 *gb = reinterpret_cast<const double2 *>(bt.alm0 + (int64_t)b * bt.alm_stride);
            v = synth_combo(gb, gb + a.nalm, a.coef, base + l, m, a.mscale);
        }
        return v;
    };
    auto store_z = [&](int e, double4 v) {
        const int lo = e >> 3, b = e & 7;
        sZ[lo][0][2 * b] = v.x;
        sZ[lo][0][2 * b + 1] = v.y;
        sZ[lo][1][2 * b] = v.z;
        sZ[lo][1][2 * b + 1] = v.w;
    };
    if (lane < 32) sT[0][lane] = stage_entry(T4, l0, lmax, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) store_z(lane + 64 * i, load_z(l0, lane + 64 * i));

    LegState<1, SPIN> S;
    leg_init<1, SPIN>(a, it, lane, S);
    bool scaled = leg_any_scaled<1, SPIN>(S);
    d4v Dp[4], Dm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) Dp[q] = Dm[q] = d4v{0.0, 0.0, 0.0, 0.0};
    const int kk = lane >> 4, jj = lane & 15;
    __syncthreads();

    int slot = 0;
    for (int c = l0; c <= lmax; c += kStage) {
        const bool has_next = c + kStage <= lmax;
        double4 nt, nz[4];
        if (has_next) {
            if (lane < 32) nt = stage_entry(T4, c + kStage, lmax, lane);
#pragma unroll
            for (int i = 0; i < 4; ++i) nz[i] = load_z(c + kStage, lane + 64 * i);
        }
        const int n = min(kStage, lmax + 1 - c);
        for (int b4 = 0; b4 < n; b4 += 4) {
            double cp = 1.0, cm = 1.0;
            if (scaled) {
                cp = S.kp[0] == 0 ? 1.0 : 0.0;
                cm = (SPIN ? S.km[0] : S.kp[0]) == 0 ? 1.0 : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int t = b4 + k;
                double vp = 0.0, vm = 0.0;
                if (t < n) {
                    vp = S.up[0] * cp;
                    vm = (SPIN ? S.um[0] : S.up[0]) * cm;
                    if (c + t < lmax) leg_advance<1, SPIN>(S, sT[slot][t]);
                }
                sL[0][k][lane] = vp;
                sL[1][k][lane] = vm;
            }
            if (scaled) {
                leg_renorm<1, SPIN>(S);
                scaled = leg_any_scaled<1, SPIN>(S);
            }
            // One wave per workgroup, whose LDS operations run in program order:
            // the barrier only keeps the compiler from moving this block's
            // writes past its reads (and the next block's writes past them).
            __syncthreads();
            // columns of l = c + b4 + kk (zero past lmax)
            const double bp = sZ[b4 + kk][0][jj], bm = sZ[b4 + kk][1][jj];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Dp[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(sL[0][kk][16 * q + jj], bp, Dp[q], 0, 0, 0);
                Dm[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(sL[1][kk][16 * q + jj], bm, Dm[q], 0, 0, 0);
            }
            __syncthreads();
        }
        if (has_next) {
            if (lane < 32) sT[slot ^ 1][lane] = nt;
            __syncthreads();  // the last block's column reads come first
#pragma unroll
            for (int i = 0; i < 4; ++i) store_z(lane + 64 * i, nz[i]);
        }
        __syncthreads();
        slot ^= 1;
    }

    // D[i][j] of block q: ring jb + 16 q + i, column j = 2 map + {Re, Im}
    const double sgn_neg = (s & 1) ? 1.0 : -1.0;  // -(-1)^s
    const int b = jj >> 1, comp = jj & 1;
    if (b >= bt.nb) return;
    double *F = reinterpret_cast<double *>(bt.F0 + (int64_t)b * bt.stride);
    const int64_t op = 2 * ((int64_t)(a.mmax + m) * a.nring) + comp;
    const int64_t om = 2 * ((int64_t)(a.mmax - m) * a.nring) + comp;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = it.jb + 16 * q + kk + 4 * r;
            if (j >= it.je || a.ring_mmax[j] < m) continue;
            F[op + 2 * j] = -Dp[q][r];
            if (m != 0) F[om + 2 * j] = sgn_neg * Dm[q][r];
        }
    }
}

// Arguments over the synthesis work list (64 R rings per item); the adjoint
// replaces items and nitems by its own list.
template <int R>
static LegArgs leg_args(const psht_plan_s &p, const void *alm_in, const void *alm_out, double *F) {
    const Geometry &g = p.g;
    LegArgs a;
    a.items = p.d_leg_items;
    a.nitems = p.n_leg_items;
    a.group = (g.nring + 64 * R - 1) / (64 * R);
    a.coef = reinterpret_cast<const double4 *>(p.leg->d_coef);
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
    a.g = static_cast<const double2 *>(alm_in);
    a.c = a.g ? a.g + a.nalm : nullptr;
    a.alm_out = static_cast<double *>(const_cast<void *>(alm_out));
    a.F = F;
    a.mscale = 1.0;
    return a;
}

static int rings_knob(const char *name, int dflt) {
    const char *e = getenv(name);
    const int v = e ? atoi(e) : dflt;
    return (v >= 1 && v <= 4) || v == 8 ? v : dflt;
}

// Rings per lane of the synthesis: PSHT_LEG_R (1, 2, 3, 4 or 8) fixes it for
// tuning runs; without it 0, and the plan chooses 1 or 2 by the size of its
// work list.
int leg_rings_per_lane() {
    static const int r = rings_knob("PSHT_LEG_R", 0);
    return r;
}

template <int R>
static void leg_synth_r(const psht_plan_s &p, const void *alm, double *F, double mscale, hipStream_t st) {
    LegArgs a = leg_args<R>(p, alm, nullptr, F);
    a.mscale = mscale;
    dim3 grid(p.n_leg_items), block(64);
    if (p.g.spin) hipLaunchKernelGGL((k_leg_synth<R, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_leg_synth<R, false>), grid, block, 0, st, a);
}

hipError_t launch_leg_synth(const psht_plan_s &p, const void *alm, double *F, double mscale, hipStream_t st) {
    if (p.n_leg_items == 0) return hipSuccess;
    switch (p.leg_rings_per_item / 64) {
        case 1: leg_synth_r<1>(p, alm, F, mscale, st); break;
        case 3: leg_synth_r<3>(p, alm, F, mscale, st); break;
        case 2: leg_synth_r<2>(p, alm, F, mscale, st); break;
        case 8: leg_synth_r<8>(p, alm, F, mscale, st); break;
        default: leg_synth_r<4>(p, alm, F, mscale, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_leg_synth_parts(const psht_plan_s &p, const void *alm, double *F, double *parts,
                                  int64_t part_stride, double mscale, hipStream_t st) {
    if (p.syn_seg == 0) return launch_leg_synth(p, alm, F, mscale, st);
    if (p.n_syn_items == 0) return hipSuccess;
    SynSegArgs A;
    A.a = leg_args<1>(p, alm, nullptr, F);
    A.a.mscale = mscale;
    A.items = p.d_syn_items;
    A.nitems = p.n_syn_items;
    A.st_mu = reinterpret_cast<const double4 *>(p.d_adj_mu);
    A.st_k = reinterpret_cast<const int2 *>(p.d_adj_k);
    A.parts = parts;
    A.part_stride = part_stride;
    const dim3 grid(p.n_syn_items), block(64);
    const bool two = p.syn_r == 2;
    if (p.g.spin) {
        if (two) hipLaunchKernelGGL((k_leg_synth_seg<2, true>), grid, block, 0, st, A);
        else hipLaunchKernelGGL((k_leg_synth_seg<1, true>), grid, block, 0, st, A);
    } else {
        if (two) hipLaunchKernelGGL((k_leg_synth_seg<2, false>), grid, block, 0, st, A);
        else hipLaunchKernelGGL((k_leg_synth_seg<1, false>), grid, block, 0, st, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.syn_parts == 0) return e;
    const int64_t n = (int64_t)(2 * p.g.mmax + 1) * p.g.nring;
    hipLaunchKernelGGL(k_synth_parts_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<double2 *>(F), reinterpret_cast<const double2 *>(parts), part_stride / 2,
                       p.d_ring_mmax, p.g.nring, p.g.mmax, p.g.lmax, p.g.spin, p.syn_seg);
    return hipGetLastError();
}

hipError_t launch_leg_synth_batch(const psht_plan_s &p, int nb, const void *alm0, int64_t alm_stride, char *F0,
                                  int64_t ws_stride, double mscale, hipStream_t st) {
    if (nb < 1 || nb > kMaxLegBatch) return hipErrorInvalidValue;
    if (p.n_leg_items64 == 0) return hipSuccess;
    LegBatchArgs bt;
    bt.a = leg_args<1>(p, nullptr, nullptr, nullptr);
    bt.a.items = p.d_leg_items64;
    bt.a.nitems = p.n_leg_items64;
    bt.a.group = (p.g.nring + 63) / 64;
    bt.a.mscale = mscale;
    bt.alm0 = static_cast<const char *>(alm0);
    bt.alm_stride = alm_stride;
    bt.F0 = F0;
    bt.stride = ws_stride;
    bt.nb = nb;
    if (p.g.spin) hipLaunchKernelGGL((k_leg_synth_mm<true>), dim3(p.n_leg_items64), dim3(64), 0, st, bt);
    else hipLaunchKernelGGL((k_leg_synth_mm<false>), dim3(p.n_leg_items64), dim3(64), 0, st, bt);
    return hipGetLastError();
}

hipError_t launch_leg_adj_states(const psht_plan_s &p, const StateItem *items, int nitems, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    LegArgs a = leg_args<1>(p, nullptr, nullptr, nullptr);
    double4 *mu = reinterpret_cast<double4 *>(p.d_adj_mu);
    int2 *k = reinterpret_cast<int2 *>(p.d_adj_k);
    if (p.g.spin) hipLaunchKernelGGL(k_leg_adj_states<true>, dim3(nitems), dim3(64), 0, st, a, items, nitems, mu, k);
    else hipLaunchKernelGGL(k_leg_adj_states<false>, dim3(nitems), dim3(64), 0, st, a, items, nitems, mu, k);
    return hipGetLastError();
}

static hipError_t leg_adjoint_seg(const psht_plan_s &p, const double *F, void *alm, double mscale, hipStream_t st) {
    // orders above mmax have no ring: their outputs (the tail of g and of c) are zero
    const int64_t nalm = (int64_t)(p.g.lmax + 1) * (p.g.lmax + 2) / 2;
    if (p.adj_accumulate) {
        hipError_t e = launch_fill_zero(alm, (size_t)nalm * 2 * 16, st);
        if (e != hipSuccess) return e;
    } else if (p.alm_tail < nalm) {
        double2 *g = static_cast<double2 *>(alm);
        hipError_t e = launch_fill_zero(g + p.alm_tail, (size_t)(nalm - p.alm_tail) * 16, st);
        if (e == hipSuccess) e = launch_fill_zero(g + nalm + p.alm_tail, (size_t)(nalm - p.alm_tail) * 16, st);
        if (e != hipSuccess) return e;
    }
    if (p.n_adj_items == 0) return hipSuccess;
    AdjArgs A;
    A.a = leg_args<1>(p, nullptr, alm, const_cast<double *>(F));
    A.a.mscale = mscale;
    A.items = p.d_adj_items;
    A.nitems = p.n_adj_items;
    A.st_mu = reinterpret_cast<const double4 *>(p.d_adj_mu);
    A.st_k = reinterpret_cast<const int2 *>(p.d_adj_k);
    A.accumulate = p.adj_accumulate;
    const int G = p.adj_waves;
    const size_t lds = sizeof(double) * 2 * G * kAdjRedDoubles;
    const dim3 grid(p.n_adj_items), block(64 * G);
    if (p.adj_rmax <= 4) {
        if (p.g.spin) hipLaunchKernelGGL(k_leg_adj_seg4<true>, grid, block, lds, st, A);
        else hipLaunchKernelGGL(k_leg_adj_seg4<false>, grid, block, lds, st, A);
    } else {
        if (p.g.spin) hipLaunchKernelGGL(k_leg_adj_seg6<true>, grid, block, lds, st, A);
        else hipLaunchKernelGGL(k_leg_adj_seg6<false>, grid, block, lds, st, A);
    }
    return hipGetLastError();
}

hipError_t launch_leg_adjoint(const psht_plan_s &p, const double *F, void *alm, double mscale, hipStream_t st) {
    return leg_adjoint_seg(p, F, alm, mscale, st);
}

}  // namespace psht
