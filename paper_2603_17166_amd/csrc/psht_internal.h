// Internal declarations of libpsht: plan geometry (host), device tables and
// the stage launchers.  Not part of the public interface (include/psht.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/psht.h"

namespace psht {

// Error carried from the internals to the C ABI.
struct Error {
    psht_status code = PSHT_OK;
    std::string msg;
};

// ---------------------------------------------------------------- geometry

// Everything that follows from (lmax, spin, theta range, epsilon, precision):
// the parameter rules of Sec. II.B-C, the rings of Sec. II.A, the window of
// Sec. II.C, the per-ring m cut-offs (polar optimization, Sec. II.A) and the
// parameters of the exponential-of-semicircle NUFFT.
struct Geometry {
    int lmax = 0, spin = 0;
    double eps = 0;
    bool fp32 = false;
    bool full_sky = false;
    double theta_star = 0, theta_min = 0;
    double alpha = 0, eps_apo = 0, theta_max = 0;
    int Lmax = 0, N2 = 0, nring = 0;
    std::vector<double> ring_theta;   // theta_j (patch colatitude)
    std::vector<double> ring_w;       // w(Theta_j)
    std::vector<int32_t> ring_mmax;   // largest m kept on ring j
    int mmax = 0;
    // NUFFT
    int W = 0;
    double beta = 0, sigma = 2.0;
    int Ntheta = 0, Nphi = 0;
    int phi_parts = 1;  // phi transforms as phi_parts transforms of Nphi / phi_parts points (1, 2 or 4)
    int row_lo = 0, rows_used = 0;
    double sx = 0, sy = 0;           // grid coordinate = theta*sx (rows), phi*sy (cols)
    std::vector<double> psihat_theta; // n = 0..Lmax
    std::vector<double> psihat_phi;   // m = 0..mmax
    // ES kernel on the inner taps 1..(W-1)/2 as polynomials of degree
    // P = max(W + 1, 12) in v = 2 (X - a0) - (W - 1), [P + 1][(W - 1) / 2]
    // (power-major); the mirror taps follow from v -> -v.  es_poly_err:
    // largest error on a test grid.
    std::vector<double> es_poly;
    std::vector<float> es_poly32;  // FP32 plans: the table in float (degree es_poly_degree(W, true))
    double es_poly_err = 0;
    double predicted_speedup = 0;
    double legendre_triples = 0;
    int window = PSHT_WINDOW_ES;   // apodization bell
    int Lmax_rule = 0;             // Lmax from eq. Lmax2 (before any spectrum tuning)
    double predicted_error = -1;   // predicted relative error for the caller's C_l (Sec. II.D); -1: not tuned
};

// Great-circle spectrum c_m, m = -lmax..lmax, of an isotropic field with power
// spectrum cl[0..lmax] (Sec. II.D, eq. cm / eq. cms); cm[m + lmax].
void great_circle_spectrum(int lmax, int spin, const double *cl, std::vector<double> &cm);

// m cut-off threshold relative to epsilon.
constexpr double kPolarTauRel = 1e-4;

bool geometry_compute(Geometry &g, int lmax, int spin, double theta_star, double theta_min,
                      double eps, int precision, bool with_grid, Error &err, bool with_cutoffs = true,
                      const psht_plan_options *opts = nullptr);

// Factorization of an FFT length into radices 4, 2, 3, 5, 7, 11, 13.
struct FftFactors {
    int n = 0, npass = 0;
    int radix[16];
};
bool fft_factor(int n, FftFactors &f);
bool is_smooth(int n, const int *primes, int np);

// ------------------------------------------------ Legendre recurrence tables

// Per (m, l): {-A_l, A_l + B_l, A_l - B_l, P_l} of the normalized recurrence
//   mu_{l+1} = ((A_l +/- B_l) - A_l y) mu_l - mu_{l-1},  y = 1 - cos(theta),
//   lambda_l = P_l mu_l,
// for l from l0 = max(m, s) (see leg_common.h), stored at the coefficient
// index of (l, m).  Seed prefactors K_m = N_l0 sqrt(C(2 l0, m + s)) as
// (mantissa, exponent).
struct LegTable {
    int lmax = 0, spin = 0;
    double *d_coef = nullptr;   // [nalm][4]
    double *d_kmant = nullptr;  // [lmax+1]
    int32_t *d_kexp = nullptr;  // [lmax+1]
    size_t bytes = 0;
    std::vector<double> h_coef, h_kmant;
    std::vector<int32_t> h_kexp;
    ~LegTable();
};
void leg_table_host(LegTable &t, int lmax, int spin);
std::shared_ptr<LegTable> leg_table_get(int lmax, int spin, Error &err);

struct LegItem {
    int32_t m, jb, je;  // rings [jb, je) for this m
};

// Work item of the segmented Legendre adjoint: one workgroup of `waves`
// wavefronts computes the outputs l in [la, lb) of order m from the active
// rings [jb, je) of m (every ring of m, or one ring group of an order with
// more rings than an item holds).  Wave w holds the 64 R consecutive rings
// from jb + 64 R w, R per lane.  An item that does not start at the seed l0 = max(m, s) starts from the
// recurrence state stored at plan time for l = la (index soff of the item's
// first ring; -1 for the first segment).  R = 0: the order has no active ring
// and its outputs are zero.
struct AdjItem {
    int32_t m, jb, je;
    int32_t la, lb;
    int32_t R;
    int64_t soff;
};

// Plan-time recurrence states of the segmented adjoint: one lane per ring of
// the 64 rings from j0 of order m (rings [jb, je) of the order), storing the
// state at the nseg - 1 segment starts l0 + k S, k = 1..nseg-1, at
// soff + (k - 1) (je - jb) + (j - jb).
struct StateItem {
    int32_t m, j0, jb, je, nseg, S;
    int64_t soff;
};

// Work item of the degree-segmented synthesis: rings [jb, je) of order m
// (at most 64 R), degrees [la, lb), starting from the seed (soff = -1, la =
// max(m, s)) or from the adjoint's stored state of the item's first ring at
// index soff; written to F (part 0) or to the partial copy `part` of F.
struct SynSegItem {
    int32_t m, jb, je;
    int32_t la, lb;
    int32_t part;
    int64_t soff;
};

// ------------------------------------------------------------------- plan

struct FftTable {
    int n = 0;
    FftFactors f;
    double *d_tw = nullptr;  // e^{-2 pi i k / n}, k = 0..n-1, interleaved (re, im)
};

}  // namespace psht

struct psht_plan_s {
    psht::Geometry g;
    int64_t npts = 0;
    // rings
    double *d_ring_y = nullptr, *d_ring_ch = nullptr, *d_ring_sh = nullptr, *d_ring_w = nullptr;
    int32_t *d_ring_mmax = nullptr;
    // Legendre work lists: synthesis (blocks of ring chunks per m)
    psht::LegItem *d_leg_items = nullptr;
    int n_leg_items = 0;
    int leg_rings_per_item = 0;
    // segmented adjoint: items, waves per workgroup, segment length, stored states
    psht::AdjItem *d_adj_items = nullptr;
    int n_adj_items = 0;
    int adj_waves = 1;
    int adj_rmax = 6;  // largest rings per lane of any item (selects the kernel instantiation)
    bool adj_accumulate = false;  // ring groups: items add into a cleared output instead of storing
    int adj_seg = 0;
    double *d_adj_mu = nullptr;    // [state] {mu+_l, mu+_{l-1}, mu-_l, mu-_{l-1}}
    int32_t *d_adj_k = nullptr;    // [state] {k+, k-}
    int64_t n_adj_states = 0;
    int64_t alm_tail = 0;          // first coefficient index of order mmax + 1 (outputs zero from there)
    // degree-segmented synthesis (plans whose synthesis items would not fill
    // the GPU): items, segment length and number of partial copies of F
    psht::SynSegItem *d_syn_items = nullptr;
    int n_syn_items = 0;
    int syn_seg = 0;    // 0: not segmented
    int syn_parts = 0;  // partial copies of F (segments beyond the first of the longest order)
    int syn_r = 2;      // rings per lane of the segmented items (1 or 2)
    psht::LegItem *d_leg_items64 = nullptr;  // 64-ring chunks (batched-maps kernel)
    int n_leg_items64 = 0;
    std::shared_ptr<psht::LegTable> leg;
    // NUFFT tables
    double *d_psihat_t = nullptr, *d_psihat_p = nullptr;
    double *d_es_poly = nullptr;
    float *d_es_poly32 = nullptr;
    psht::FftTable fft_n2, fft_nt, fft_np, fft_np_part;
    bool theta_split = false;  // Theta grid transform as two N2-point transforms (NT = 2 N2 above the LDS limit)
    // points, sorted by tile
    int tile_x = 16, tile_y = 32, ntx = 0, nty = 0, ntiles = 0;
    double *d_px = nullptr, *d_py = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_tile_start = nullptr;  // ntiles + 1, in entries (2 per slot)
    int64_t n_entries = 0;            // slot entries of all tiles (points + dummies)
    unsigned long long *d_dropped = nullptr;  // points the NUFFT kernels had to skip (expected 0)
    // workspace layout (bytes, per map)
    size_t ws_F = 0, ws_V = 0, ws_U = 0, ws_per_map = 0;
    size_t resident = 0;
    std::vector<void *> allocations;
    // per-stage HIP-event timing (PSHT_T_* indices)
    unsigned timing = 0;  // bitmask of the stages to time
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> event_pool;
    double t_ms[PSHT_T_COUNT] = {0};
    int64_t t_launches[PSHT_T_COUNT] = {0};
};

namespace psht {

// Stage launchers (defined in the .hip files).  All asynchronous on `st`.
// `mscale` multiplies the coefficients (synthesis) or the outputs (adjoint) of
// every order m >= 1; 1 for the plain transforms.
hipError_t launch_leg_synth(const psht_plan_s &p, const void *alm, double *F, double mscale, hipStream_t st);
// The same through the degree-segmented work list when the plan has one
// (syn_seg > 0), with the partial copies of F at `parts` (syn_parts copies of
// 2 mmax + 1 by nring complex values, `part_stride` doubles apart); otherwise
// launch_leg_synth.
hipError_t launch_leg_synth_parts(const psht_plan_s &p, const void *alm, double *F, double *parts,
                                  int64_t part_stride, double mscale, hipStream_t st);
hipError_t launch_leg_adjoint(const psht_plan_s &p, const double *F, void *alm, double mscale, hipStream_t st);
constexpr int kAdjMaxWavesHost = 4;  // waves per workgroup of the segmented adjoint
constexpr int kAdjMaxRings = 6;      // rings per lane of the segmented adjoint
// Plan time: the recurrence states of the segmented adjoint.
hipError_t launch_leg_adj_states(const psht_plan_s &p, const StateItem *items, int nitems, hipStream_t st);

// Legendre synthesis of nb <= kMaxLegBatch maps in one pass (MFMA): map b reads
// its coefficients at alm0 + b alm_stride and writes F at F0 + b ws_stride
// (its own workspace).
constexpr int kMaxLegBatch = 8;
hipError_t launch_leg_synth_batch(const psht_plan_s &p, int nb, const void *alm0, int64_t alm_stride, char *F0,
                                  int64_t ws_stride, double mscale, hipStream_t st);
hipError_t launch_theta_synth(const psht_plan_s &p, const double *F, void *V, hipStream_t st);
hipError_t launch_theta_adjoint(const psht_plan_s &p, const void *V, double *F, hipStream_t st);
hipError_t launch_phi_synth(const psht_plan_s &p, const void *V, void *U, hipStream_t st);
hipError_t launch_phi_adjoint(const psht_plan_s &p, const void *U, void *V, hipStream_t st);
hipError_t launch_interp(const psht_plan_s &p, const void *U, void *map, hipStream_t st);
hipError_t launch_spread(const psht_plan_s &p, const void *map, void *U, hipStream_t st);
hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t st);

// Patch-frame rotation (k_rotate.hip): R = Rz(alpha) Ry(beta) Rz(gamma).
struct RotMatrix {
    double r[3][3];
};
// Coefficients: workspace ws of nc (lmax + 1)(2 lmax + 1) complex doubles; lf:
// device table of log2(n!) as double-double, n = 0..2 lmax.
hipError_t launch_rotate_alm(int lmax, int nc, double alpha, double beta, double gamma, const void *alm_in,
                             void *alm_out, void *ws, const double2 *lf, hipStream_t st);
hipError_t launch_rotate_points(int64_t n, const RotMatrix &R, const double *theta, const double *phi,
                                double *theta_out, double *phi_out, double *psi_out, hipStream_t st);
hipError_t launch_spin_phase(int64_t n, double ks, int fp32, const double *psi, void *map, hipStream_t st);
hipError_t launch_fft_rows(const FftTable &t, int batch, int sign, bool fp32, const void *in, void *out,
                           hipStream_t st);

// Synthesis driver behind psht_synth / psht_synth_grad (mscale 1 / 0.5): validates
// the arguments and the workspace size, then issues every stage on hip_stream.
psht_status synth_run(psht_plan plan, int nmaps, const void *alm, void *map, void *workspace, size_t ws_bytes,
                      double mscale, void *hip_stream);
// Sets the calling thread's error text (psht_last_error) and returns code.
psht_status set_error(psht_status code, const char *msg);

// Plan-time point kernels.
hipError_t launch_point_stats(const double *theta, const double *phi, int64_t n, double *d_stats,
                              hipStream_t st);
// Bucket sort of the points into NUFFT tiles in two launches: the first
// counts and scatters the points into tiles (tpx, tpy, tperm, tile ranges
// d_pstart) and writes p.d_tile_start in entries (2 per slot, see k_nufft.hip);
// the caller then sizes p.d_px/d_py/d_perm to p.d_tile_start[ntiles] entries
// and the second launch writes the slot layout.
hipError_t launch_point_sort_count(psht_plan_s &p, const double *theta, const double *phi, int32_t *d_keys,
                                   int32_t *d_cursor, int32_t *d_pstart, double *tpx, double *tpy, int32_t *tperm,
                                   hipStream_t st);
// It also counts into *d_bad the entries whose stencil origin lies outside their
// tile (the plan fails if there are any).
hipError_t launch_point_sort_order(psht_plan_s &p, int32_t *d_keys, const int32_t *d_pstart, const double *tpx,
                                   const double *tpy, const int32_t *tperm, unsigned long long *d_bad,
                                   hipStream_t st);
struct TileGeom;
TileGeom tile_geom(const psht_plan_s &p);

// Rings per lane of the Legendre synthesis kernel (a work item covers 64 x
// this many rings); 0 leaves the choice to the plan.
int leg_rings_per_lane();

// Largest FFT length one workgroup transforms in LDS (160 KB on gfx950).
constexpr int kFftMaxLds64 = 10240;
constexpr int kFftMaxLds32 = 10240;

}  // namespace psht
