/*
 * psht -- partial-sky spin-weighted spherical harmonic transforms on MI355X.
 *
 * C ABI of libpsht.so.  Plain pointers and sizes only; every device pointer
 * is a HIP device allocation on the current device, every stream a
 * hipStream_t passed as void* (NULL = the legacy default stream).
 *
 * The library computes, for coefficients g_lm, c_lm (l <= lmax) and spin s,
 *
 *   Synthesis general (Carron & Reinecke, Sec. I, eq. syn):
 *     f_p = - sum_{l,m} (g_lm + i c_lm) sY_lm(theta_p, phi_p),
 *   Adjoint synthesis general (Sec. I):
 *     g~_lm = -1/2    sum_p [ f_p sY*_lm + (-1)^s conj(f_p) (-s)Y*_lm ],
 *     c~_lm = -1/(2i) sum_p [ f_p sY*_lm - (-1)^s conj(f_p) (-s)Y*_lm ],
 *
 * with sY_lm = sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi} (Appendix A,
 * eq. Ylm) and the reality condition a*_lm = (-1)^m a_l,-m (Sec. I).  It
 * follows the partial-sky method of Sec. II: rings inside the apodized cap
 * theta <= theta_max = theta*(1 + eps_apo) (steps 1-2), the weighted,
 * stretched map w(Theta) f(Theta theta_max / pi, phi) (step 3), Lmax + 1
 * rings and the Fourier-sphere evaluation at the points (step 4, Sec. I.B),
 * with the window and apodization rules of Sec. II.B-C (summary paragraph).
 *
 * Layouts
 *   alm  : complex, [nmaps][2][nalm], g first then c; nalm = (lmax+1)(lmax+2)/2,
 *          index(l, m) = m (2 lmax + 1 - m) / 2 + l for 0 <= m <= l.  Always
 *          complex128 (double).  Entries with l < s are ignored by synthesis
 *          and written as zero by the adjoint; Im(g_l0), Im(c_l0) are ignored
 *          by synthesis and written as zero by the adjoint.
 *   map  : complex, [nmaps][npoints] in the caller's point order; complex128
 *          for FP64 plans, complex64 for FP32 plans (info.map_is_fp32).
 *   theta, phi : double [npoints] device arrays, colatitude in [0, pi] and
 *          longitude (any real, reduced mod 2 pi), in the patch frame, i.e.
 *          with the patch centre at the north pole (Sec. II, step 1).
 *
 * Inner products under which psht_adjoint is the exact adjoint of
 * psht_synth (up to rounding): maps  <f, f'> = sum_p Re(conj(f_p) f'_p);
 * coefficients <a, a'> = sum_l (g_l0 g'_l0 + c_l0 c'_l0)
 *                         + 2 sum_{l, m >= 1} Re(conj(g_lm) g'_lm + conj(c_lm) c'_lm).
 *
 * Errors: every argument is validated before anything is launched; on a
 * non-OK status nothing has been written to the outputs (except for
 * PSHT_ERR_DEVICE raised by the runtime after launches).  psht_last_error()
 * returns a thread-local message for the last non-OK status of the calling
 * thread.  No C++ exception crosses this interface.
 */
#ifndef PSHT_H
#define PSHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psht_plan_s *psht_plan;

typedef enum {
    PSHT_OK = 0,
    PSHT_ERR_ARG = 1,          /* invalid argument (value, null pointer, point out of range) */
    PSHT_ERR_NOMEM = 2,        /* device or host allocation failed */
    PSHT_ERR_DEVICE = 3,       /* a HIP runtime call failed */
    PSHT_ERR_UNSUPPORTED = 4,  /* size outside what the kernels handle */
    PSHT_ERR_WORKSPACE = 5     /* workspace missing or smaller than required */
} psht_status;

typedef enum {
    PSHT_PREC_AUTO = 0,  /* FP32 grid/NUFFT when epsilon >= 1e-6, else FP64 */
    PSHT_PREC_FP32 = 1,
    PSHT_PREC_FP64 = 2
} psht_precision;

/* Everything a plan derives from (lmax, spin, points, epsilon).  Names follow
 * the paper: Lmax is the band limit of the stretched map (eq. Lmax2), eps_apo
 * the fractional apodization length, alpha the bell shape parameter (summary
 * of Sec. II.C), theta_max = theta_star (1 + eps_apo) (Sec. II, step 2). */
typedef struct {
    int32_t lmax, spin;
    int32_t Lmax;            /* band limit in Theta; rings j = 0..Lmax */
    int32_t n2;              /* samples on the doubled circle, 2 Lmax + 1 */
    int32_t mmax;            /* largest m kept on any ring (polar optimization) */
    int32_t nufft_w;         /* ES kernel width in grid cells */
    int32_t ntheta_grid;     /* oversampled NUFFT grid size along Theta */
    int32_t nphi_grid;       /* oversampled NUFFT grid size along phi */
    int32_t row_lo;          /* first Theta-grid row touched by any point */
    int32_t rows_used;       /* number of Theta-grid rows touched by the points */
    int32_t map_is_fp32;     /* 1: map buffers are complex64 */
    int32_t full_sky;        /* 1: patch too large, theta_max = pi, w = 1, Lmax >= lmax */
    double epsilon;
    double theta_star, theta_min, theta_max, eps_apo, alpha;
    double nufft_beta, nufft_sigma;
    double predicted_speedup; /* 1 / ((1 + eps_apo)(1 - cos theta_max)), Sec. II.A */
    double legendre_triples;  /* sum over rings of (l, m) pairs kept: algorithmic work */
    int64_t npoints;
    size_t resident_bytes;          /* device memory the plan holds */
    size_t workspace_bytes_per_map; /* workspace psht_synth/psht_adjoint need per map */
    double kernel_poly_err;  /* largest error of the polynomial ES kernel taps (inner taps) */
    /* Legendre adjoint work decomposition: degree segments of adj_segment
     * degrees per order, adj_waves wavefronts per work item (together holding
     * every active ring of the order, at most adj_rings_per_lane rings per
     * lane); adj_states recurrence states (40 bytes each) stored by the plan
     * for the segment starts. */
    int32_t adj_segment, adj_waves, adj_rings_per_lane;
    int64_t adj_states;
    /* Lmax_rule: Lmax from eq. Lmax2; Lmax differs from it when the plan was
     * tuned to a power spectrum (psht_plan_options.cl), and predicted_error is
     * then the predicted relative error of the band-limited weighted map for
     * fields of that spectrum (Sec. II.D, eq. st); -1 when not tuned. */
    int32_t Lmax_rule;
    double predicted_error;
    int32_t window;     /* PSHT_WINDOW_* of the plan */
    /* part of resident_bytes shared with every other plan of the same
     * (lmax, spin): the Legendre recurrence table, freed with the last such
     * plan (0 for psht_plan_geometry) */
    size_t shared_bytes;
    /* Legendre synthesis work decomposition: 0, or (for plans whose per-order
     * work items would leave most of the GPU idle) segments of syn_segment
     * degrees per order, started from the adjoint's stored states, with
     * syn_parts partial copies of the ring coefficients in the workspace */
    int32_t syn_segment, syn_parts;
} psht_plan_info;

/* Options of psht_plan_create_ex / psht_plan_geometry_ex (NULL: all defaults,
 * the behaviour of psht_plan_create).
 *   full_sky : 1 selects the full-sky mode: rings over the whole sphere,
 *              theta_max = pi, window w = 1, Lmax = lmax rounded up to a
 *              smooth 2 Lmax + 1 (the Fourier-sphere synthesis of Sec. I.B
 *              without the partial-sky steps of Sec. II); exact up to the
 *              NUFFT error for any point set.  0: partial sky (the mode falls
 *              back to the full sky only when the patch is too large to gain).
 *   window   : apodization bell of Sec. II.C, all three with shape parameter
 *              alpha = |ln epsilon| / pi: PSHT_WINDOW_ES (0, the
 *              exponential-of-semicircle bell of eq. KB), PSHT_WINDOW_KB (1,
 *              the Kaiser-Bessel bell I0(pi alpha sqrt(1 - x^2)), whose Fourier
 *              transform is the closed form given with eq. KB) or
 *              PSHT_WINDOW_PSWF (2, the order-0 prolate spheroidal (Slepian)
 *              function of bandwidth c = pi alpha).
 *   cl, cl_lmax : optional host array cl[0..cl_lmax] (cl_lmax >= lmax,
 *              finite, >= 0), the power spectrum C_l of the fields to be
 *              transformed (C^E_l + C^B_l for spin > 0); read during the call
 *              only.  When given, Lmax is the smallest smooth value, at most
 *              the rule's, whose predicted relative error of the weighted
 *              band-limited map for such fields (Sec. II.D, eqs. s2m, st, cm,
 *              cms) is at most epsilon / 2; theta_max and the window are the
 *              rule's.  NULL: the rule's Lmax.  Ignored in full-sky mode.
 *   lmax_rule : PSHT_LMAX_RULE_BAND (0): theta_max and Lmax from eq. Lmax2
 *              (the smallest band limit); PSHT_LMAX_RULE_COST (1): the
 *              apodization length that minimizes the Legendre work of the
 *              rings with polar optimization (footnote to eq. Lmax2). */
typedef struct {
    int32_t full_sky;
    int32_t window;
    const double *cl;
    int32_t cl_lmax;
    int32_t lmax_rule;
} psht_plan_options;
enum { PSHT_WINDOW_ES = 0, PSHT_WINDOW_KB = 1, PSHT_WINDOW_PSWF = 2 };
enum { PSHT_LMAX_RULE_BAND = 0, PSHT_LMAX_RULE_COST = 1 };

/* Build a plan for npoints points (device arrays theta, phi; read during the
 * call only, not kept).  Validates lmax >= 0, 0 <= spin <= lmax,
 * 1e-14 <= epsilon <= 1e-2, npoints >= 0 and < 2^30, every theta in
 * [0, pi] and every phi finite (checked on the device; one device-to-host
 * synchronisation on `hip_stream`).  Sorts the points into NUFFT tiles and
 * uploads rings, window weights, per-ring m cut-offs and kernel tables; the
 * Legendre recurrence tables are shared by all plans of the same (lmax, spin).
 * On success *out owns device memory until psht_plan_destroy. */
psht_status psht_plan_create(psht_plan *out, int lmax, int spin, int64_t npoints,
                             const double *theta, const double *phi,
                             double epsilon, int precision, void *hip_stream);

/* psht_plan_create with options (see psht_plan_options; opts may be NULL). */
psht_status psht_plan_create_ex(psht_plan *out, int lmax, int spin, int64_t npoints,
                                const double *theta, const double *phi, double epsilon, int precision,
                                const psht_plan_options *opts, void *hip_stream);

/* Copy the plan's parameters into *info. */
psht_status psht_plan_query(psht_plan plan, psht_plan_info *info);

/* Synthesis general (eq. syn) of nmaps coefficient sets into nmaps maps,
 * asynchronously on hip_stream.  alm: device, complex128 [nmaps][2][nalm];
 * map: device, [nmaps][npoints] complex128 or complex64 (plan precision).
 * workspace: device buffer of at least nmaps * workspace_bytes_per_map bytes,
 * caller-owned, not used after the stream reaches the end of the call. */
psht_status psht_synth(psht_plan plan, int nmaps, const void *alm, void *map,
                       void *workspace, size_t ws_bytes, void *hip_stream);

/* Adjoint synthesis general (Sec. I) of nmaps maps into nmaps coefficient
 * sets; same layouts and workspace rule as psht_synth.  alm is overwritten.
 * The spreading kernel adds its tile subgrids into the workspace, and plans
 * whose orders hold more rings than one adjoint work item (ring groups, full
 * sky at large lmax) add into alm, with device-scope floating-point atomic
 * adds: workspace and alm must be ordinary (coarse-grained) device memory,
 * as hipMalloc and torch's CUDA allocator return, not fine-grained, host or
 * managed memory. */
psht_status psht_adjoint(psht_plan plan, int nmaps, const void *map, void *alm,
                         void *workspace, size_t ws_bytes, void *hip_stream);

/* Gradient forms for automatic differentiation of a real loss L.  Gradients
 * of complex quantities follow the convention dL/dRe z + i dL/dIm z.
 *
 * psht_adjoint_grad: given map_grad = dL/df for f = psht_synth(alm), writes
 * alm_grad = dL/dalm.  Because synthesis is real-linear in (Re, Im) of every
 * entry and the coefficient inner product above weighs orders m >= 1 twice,
 * this is the adjoint synthesis (Sec. I) with the outputs of every m >= 1
 * doubled; m = 0 entries are real (their imaginary parts do not enter the
 * synthesis) and entries with l < s are zero.
 *
 * psht_synth_grad: given alm_grad = dL/da~ for a~ = psht_adjoint(map),
 * writes map_grad = dL/dmap: the synthesis (eq. syn) of alm_grad with every
 * order m >= 1 halved (Im of the m = 0 entries is ignored, as in synthesis).
 *
 * Same layouts, workspace rule, precision and errors as psht_synth /
 * psht_adjoint; the two cost what the plain transforms cost. */
psht_status psht_adjoint_grad(psht_plan plan, int nmaps, const void *map_grad, void *alm_grad,
                              void *workspace, size_t ws_bytes, void *hip_stream);
psht_status psht_synth_grad(psht_plan plan, int nmaps, const void *alm_grad, void *map_grad,
                            void *workspace, size_t ws_bytes, void *hip_stream);

/* Synthesis without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same operation, layouts, stream semantics and errors as
 * psht_synth, but the workspace is a static device array of
 * PSHT_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends; the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  A plan whose
 * nmaps * workspace_bytes_per_map exceeds that size is rejected with
 * PSHT_ERR_WORKSPACE before anything is launched.  All calls on one GPU share
 * the array: calls that overlap on one GPU (different streams or threads)
 * race; the caller serialises them (one stream, or stream ordering). */
#define PSHT_NOALLOC_SCRATCH_BYTES (64u << 20)
psht_status psht_synth_noalloc(psht_plan plan, int nmaps, const void *alm, void *map, void *hip_stream);

/* Free the plan's device memory.  The caller must synchronise every stream
 * that still runs work of this plan first.  NULL is a no-op. */
void psht_plan_destroy(psht_plan plan);

/* Great-circle spectrum of an isotropic spin-s field with power spectrum
 * C_l (Sec. II.D, eq. cm; eq. cms with C_l = C^E_l + C^B_l for s > 0):
 *   c_m = sum_{l >= max(|m|, s)} C_l (2l+1)/2 |d^l_{m,-s}(pi/2)|^2,
 * so that the field along a great circle through the poles has the
 * one-dimensional correlation (1/2pi) sum_m c_m e^{i m (theta - theta')}.
 * cl: host array cl[0..lmax]; cm: host array of 2 lmax + 1 doubles receiving
 * c_m at cm[m + lmax], m = -lmax..lmax (host computation, long double). */
psht_status psht_great_circle_spectrum(int lmax, int spin, const double *cl, double *cm);

/* ---- Patch frame (Sec. II, step 1) -----------------------------------------
 * The method works in coordinates in which the patch centre is the north
 * pole.  These calls move coefficients, points and spin bases from another
 * frame (e.g. equatorial) into that frame.  R = Rz(alpha) Ry(beta) Rz(gamma)
 * is an active rotation with z-y-z Euler angles; for a patch centred at
 * colatitude theta_c and longitude phi_c, (alpha, beta, gamma) =
 * (psi_0, -theta_c, -phi_c) takes the centre to the pole (any psi_0 turns the
 * patch about its centre).  With coefficients a' from psht_rotate_alm and
 * points n' = R n from psht_rotate_points, the spin-s synthesis satisfies
 *   f'(n') = exp(i s psi) f(n),
 * psi being the angle psht_rotate_points returns; psht_spin_phase applies or
 * removes that factor.  The adjoint of a rotation is the rotation by
 * (-gamma, -beta, -alpha). */

/* Workspace bytes psht_rotate_alm needs: ncomp (lmax + 1)(2 lmax + 1) * 16. */
psht_status psht_rotate_alm_workspace(int lmax, int ncomp, size_t *bytes);

/* a'_lm = exp(-i m alpha) sum_{m' = -l..l} d^l_{m m'}(beta) exp(-i m' gamma) a_lm'
 * (Wigner D of Appendix A's d-matrix), with a_{l,-m'} = (-1)^m' conj(a_lm')
 * (reality condition of Sec. I; the imaginary part of a_l0 is ignored), for
 * each of ncomp (1 or 2: g and c of a spin field) coefficient sets.
 * alm_in, alm_out: device complex128 [ncomp][nalm], m-major layout of
 * psht_synth; they must not overlap.  0 <= lmax <= 16383; angles finite.
 * workspace: device memory of at least psht_rotate_alm_workspace bytes,
 * overwritten.  O(lmax^3) work on hip_stream; asynchronous.  The first call
 * for a given lmax on a device builds a small log-factorial table there
 * (kept until the process ends; one synchronous copy).  alm_out is
 * accumulated with device-scope atomic adds, so it must be ordinary device
 * memory. */
psht_status psht_rotate_alm(int lmax, int ncomp, double alpha, double beta, double gamma, const void *alm_in,
                            void *alm_out, void *workspace, size_t ws_bytes, void *hip_stream);

/* n' = R n for npoints points: device double arrays theta, phi in, theta_out
 * in [0, pi], phi_out in [0, 2 pi), psi_out in [-pi, pi] (the angle from R
 * e_theta(n) to e_theta(n'), measured towards e_phi(n')).  Outputs may alias
 * the inputs element for element.  Asynchronous on hip_stream. */
psht_status psht_rotate_points(int64_t npoints, double alpha, double beta, double gamma, const double *theta,
                               const double *phi, double *theta_out, double *phi_out, double *psi_out,
                               void *hip_stream);

/* map[i] *= exp(i sign spin psi[i]) in place; map complex64 (fp32 = 1) or
 * complex128 (fp32 = 0) [npoints] on the device, psi double [npoints];
 * sign +1 or -1.  Asynchronous on hip_stream. */
psht_status psht_spin_phase(int64_t npoints, int spin, int sign, int fp32, const double *psi, void *map,
                            void *hip_stream);

/* Thread-local text for the last non-OK status of this thread ("" if none). */
const char *psht_last_error(void);

/* Integrity counter of a plan: *dropped receives the number of points the
 * interpolation / spreading kernels found outside the NUFFT tile they were
 * sorted into and had to skip since the plan was created.  Plan creation
 * verifies the sort (and fails with PSHT_ERR_DEVICE if any point is outside
 * its tile), so this is 0 unless something is broken.  Synchronises
 * hip_stream (the stream the plan's work ran on) before reading. */
psht_status psht_plan_check(psht_plan plan, int64_t *dropped, void *hip_stream);

/* Host-only evaluation of the plan parameters for a cap of radius theta_star
 * (theta_min = 0), without any device work: the rules of Sec. II.B-C for
 * eps_apo, theta_max, Lmax (eq. Lmax2, rounded up so that 2 Lmax + 1 has only
 * the factors 3, 5, 7, 11, 13), the rings Theta_j = 2 pi j / (2 Lmax + 1),
 * theta_j = Theta_j theta_max / pi (Sec. II.A), the window weights w_j
 * (Sec. II.C) and the per-ring m cut-offs.  ring_theta, ring_weight and
 * ring_mmax are host arrays of `capacity` entries (may be NULL when
 * capacity is 0); they receive min(capacity, Lmax + 1) rings.  The per-ring
 * m cut-off search runs only when capacity > 0; with capacity 0, info->mmax
 * is lmax and info->legendre_triples counts every m on every ring. */
psht_status psht_plan_geometry(int lmax, int spin, double theta_star, double epsilon, int precision,
                               psht_plan_info *info, double *ring_theta, double *ring_weight,
                               int32_t *ring_mmax, int capacity);

/* psht_plan_geometry with options (see psht_plan_options; opts may be NULL). */
psht_status psht_plan_geometry_ex(int lmax, int spin, double theta_star, double epsilon, int precision,
                                  const psht_plan_options *opts, psht_plan_info *info, double *ring_theta,
                                  double *ring_weight, int32_t *ring_mmax, int capacity);

/* ---- Stage-level entry points (diagnostics and stage tests) ----------------
 * Run a single stage of a plan on device buffers.  Layouts:
 *   PSHT_STAGE_LEGENDRE_SYNTH : in = alm complex128 [2][nalm],
 *                               out = F complex128 [2 mmax + 1][Lmax + 1],
 *                               F[(m + mmax)(Lmax+1) + j] = F_m(theta_j), the
 *                               azimuthal Fourier coefficient of the map of
 *                               eq. syn on ring j; zero where m is cut off.
 *   PSHT_STAGE_LEGENDRE_ADJOINT : in = F' (same layout), out = alm [2][nalm];
 *                               the exact transpose of the stage above.
 * Both are asynchronous on hip_stream and allocate nothing. */
enum { PSHT_STAGE_LEGENDRE_SYNTH = 1, PSHT_STAGE_LEGENDRE_ADJOINT = 2 };
psht_status psht_stage(psht_plan plan, int stage, const void *in, void *out, void *hip_stream);

/* psht_stage with a workspace (at least workspace_bytes_per_map bytes,
 * overwritten), for the stages after the Legendre step:
 *   PSHT_STAGE_FOURIER_SYNTH : in = F complex128 [2 mmax + 1][Lmax + 1] (the
 *       layout above), out = map [npoints] in the plan's precision: the
 *       Theta stage (window w_j, doubled circle with the mirror sign
 *       (-1)^(s+m), band limit |n| <= Lmax, Sec. I.B eq. Dnz), the phi stage
 *       and the NUFFT interpolation, i.e. f_p = sum_m e^{i m phi_p}
 *       sum_k D(Theta_p - Theta_k) G_k(m) up to the NUFFT error, with
 *       G_j = w_j F_j, G_{N2-j} = (-1)^(s+m) w_j F_j, and F_j(m) taken as
 *       zero for |m| above ring j's polar cut-off (Sec. II.A; the Legendre
 *       stage writes zeros there).
 *   PSHT_STAGE_FOURIER_ADJOINT : in = map, out = F' [2 mmax + 1][Lmax + 1];
 *       the exact transpose of the stage above (spreading, phi and Theta
 *       adjoints; zero above each ring's cut-off).
 * The Legendre stages accept workspace = NULL and then run as psht_stage;
 * with a workspace, PSHT_STAGE_LEGENDRE_SYNTH runs the work decomposition of
 * psht_synth (degree segments when the plan's syn_segment is non-zero, their
 * partial sums in the workspace).  Asynchronous on hip_stream. */
enum { PSHT_STAGE_FOURIER_SYNTH = 3, PSHT_STAGE_FOURIER_ADJOINT = 4 };
psht_status psht_stage_ex(psht_plan plan, int stage, const void *in, void *out, void *workspace, size_t ws_bytes,
                          void *hip_stream);

/* Batched complex FFT on device data, the kernel the Theta and phi stages use
 * (diagnostics and tests): `batch` transforms of length n (factors 2,3,5,7,11,13,
 * n <= 8192), contiguous rows, in place is allowed.
 * sign = -1: out_k = sum_j in_j e^{-2 pi i jk/n}; sign = +1: e^{+...}; unnormalized.
 * fp32 = 1 selects complex64 data. */
psht_status psht_fft(int n, int batch, int sign, int fp32, const void *in, void *out, void *hip_stream);

/* ---- Per-stage timing ------------------------------------------------------
 * psht_plan_set_timing(plan, stages): stages = 0 turns timing off; otherwise it
 * is a bitmask of the stages to time (bit PSHT_T_x; PSHT_T_ALL for every
 * stage).  Every later psht_synth / psht_adjoint call on the plan then records
 * a pair of HIP events around each selected stage launch on the call's stream.
 * The call resets the totals and creates the events ahead (for 32 calls), so
 * that timing one stage adds two event records per call and nothing else.
 * psht_plan_timing synchronises the events and returns, per stage, the summed
 * elapsed milliseconds and the number of launches since timing was (re-)set.
 * Not thread-safe: one caller at a time per plan while timing is on. */
enum {
    PSHT_T_LEG_SYNTH = 0, PSHT_T_THETA_SYNTH = 1, PSHT_T_PHI_SYNTH = 2, PSHT_T_INTERP = 3,
    PSHT_T_GRID_ZERO = 4, PSHT_T_SPREAD = 5, PSHT_T_PHI_ADJ = 6, PSHT_T_THETA_ADJ = 7,
    PSHT_T_ALM_ZERO = 8, PSHT_T_LEG_ADJ = 9, PSHT_T_COUNT = 10, PSHT_T_ALL = (1 << 10) - 1
};
psht_status psht_plan_set_timing(psht_plan plan, int stages);
psht_status psht_plan_timing(psht_plan plan, double *ms, int64_t *launches);

/* Host evaluation (diagnostics and tests) of
 *   lambda+_l = sqrt((2l+1)/4pi) d^l_{m,-s}(theta),  lambda-_l = sqrt((2l+1)/4pi) d^l_{m,s}(theta)
 * (Appendix A, eq. Ylm) for l = 0..lmax into lam_plus / lam_minus (host arrays
 * of lmax + 1 doubles), by exactly the seeds, recurrence tables and rescaling
 * the GPU Legendre kernels use.  Values still below the double range are 0. */
psht_status psht_legendre_column(int lmax, int spin, int m, double theta, double *lam_plus, double *lam_minus);

#ifdef __cplusplus
}
#endif
#endif /* PSHT_H */
