// C ABI of libpsht (declared in include/psht.h): argument validation, plan
// construction (point statistics, geometry, tables, point sort), workspace
// layout and the stage sequences of synthesis and adjoint synthesis.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>
#include <new>
#include <string>

#include "leg_common.h"
#include "psht_internal.h"

namespace {

thread_local std::string g_last_error;

psht_status fail(psht_status code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

psht_status fail(const psht::Error &e) { return fail(e.code, e.msg); }

psht_status device_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? PSHT_ERR_NOMEM : PSHT_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T> bool dalloc(psht_plan_s &p, T *&ptr, size_t count) {
    void *raw = nullptr;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (hipMalloc(&raw, bytes) != hipSuccess) return false;
    p.allocations.push_back(raw);
    p.resident += bytes;
    ptr = static_cast<T *>(raw);
    return true;
}

// Synchronous upload: the host vectors are temporaries of plan creation.
template <typename T> bool upload(psht_plan_s &p, T *&ptr, const std::vector<T> &host, hipStream_t) {
    if (!dalloc(p, ptr, host.size())) return false;
    if (host.empty()) return true;
    return hipMemcpy(ptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

void free_plan(psht_plan_s *p) {
    if (!p) return;
    for (auto &e : p->pending) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    for (void *a : p->allocations) (void)hipFree(a);
    delete p;
}

hipEvent_t take_event(psht_plan_s &p) {
    if (!p.event_pool.empty()) {
        hipEvent_t e = p.event_pool.back();
        p.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one stage launch, bracketed by timing events when timing is on.
template <typename Fn> hipError_t timed(psht_plan_s &p, int stage, hipStream_t st, Fn fn) {
    if (!((p.timing >> stage) & 1u)) return fn();
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return fn();
    (void)hipEventRecord(a, st);
    hipError_t e = fn();
    (void)hipEventRecord(b, st);
    p.pending.push_back({stage, {a, b}});
    return e;
}

bool make_fft_table(psht_plan_s &p, psht::FftTable &t, int n, hipStream_t st) {
    if (!psht::fft_factor(n, t.f)) return false;
    t.n = n;
    std::vector<double> tw(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < n; ++k) {
        long double a = 2 * pi * k / n;
        tw[2 * k] = (double)cosl(a);
        tw[2 * k + 1] = (double)(-sinl(a));
    }
    return upload(p, t.d_tw, tw, st);
}

void fill_info(const psht_plan_s &p, psht_plan_info *info) {
    const psht::Geometry &g = p.g;
    std::memset(info, 0, sizeof(*info));
    info->lmax = g.lmax;
    info->spin = g.spin;
    info->Lmax = g.Lmax;
    info->n2 = g.N2;
    info->mmax = g.mmax;
    info->nufft_w = g.W;
    info->ntheta_grid = g.Ntheta;
    info->nphi_grid = g.Nphi;
    info->row_lo = g.row_lo;
    info->rows_used = g.rows_used;
    info->map_is_fp32 = g.fp32 ? 1 : 0;
    info->full_sky = g.full_sky ? 1 : 0;
    info->epsilon = g.eps;
    info->theta_star = g.theta_star;
    info->theta_min = g.theta_min;
    info->theta_max = g.theta_max;
    info->eps_apo = g.eps_apo;
    info->alpha = g.alpha;
    info->nufft_beta = g.beta;
    info->nufft_sigma = g.sigma;
    info->predicted_speedup = g.predicted_speedup;
    info->legendre_triples = g.legendre_triples;
    info->npoints = p.npts;
    info->resident_bytes = p.resident + (p.leg ? p.leg->bytes : 0);
    info->shared_bytes = p.leg ? p.leg->bytes : 0;
    info->workspace_bytes_per_map = p.ws_per_map;
    info->kernel_poly_err = g.es_poly_err;
    info->adj_segment = p.adj_seg;
    info->adj_waves = p.adj_waves;
    info->adj_rings_per_lane = p.adj_rmax;
    info->adj_states = p.n_adj_states;
    info->Lmax_rule = g.Lmax_rule;
    info->predicted_error = g.predicted_error;
    info->window = g.window;
    info->syn_segment = p.syn_seg;
    info->syn_parts = p.syn_parts;
}

struct ScopedDevFree {
    void *p = nullptr;
    ~ScopedDevFree() {
        if (p) (void)hipFree(p);
    }
};

// Degree-segmented synthesis.  The synthesis runs one wave per (order m,
// chunk of 64 R rings) over all degrees of m; a small cap at high lmax has few
// such items (a few hundred orders), each thousands of sequential steps long,
// and leaves most of the GPU idle.  Such a plan cuts the degrees of every order
// into segments of Ssyn = 2^k S degrees, S the adjoint's segment length, so
// that every segment start has a state stored for the adjoint; segment k >= 1
// of an order writes its own partial copy of F, which a second kernel adds in.
// Ssyn is the largest such length for which the longest item costs at most a
// third of the average work per wave slot (two waves per SIMD), as for the
// adjoint, lengthened where needed to at most 33 segments per order (32
// partial copies); a plan whose longest order would get fewer than three
// segments is not segmented.
// The items use two rings per lane (one when PSHT_LEG_R fixes one): with
// the parallelism from the segments, the longer per-step work beats the one
// ring per lane of the plain list of such plans (lmax 4096, 5-degree disc:
// 0.135 against 0.162 ms; equal within 2 us on the smallest plans).
bool build_synth_segments(psht_plan_s &p, int ncu, const std::vector<int> &first, const std::vector<int> &last,
                          const std::vector<int64_t> &soff_m, int S, hipStream_t st) {
    const psht::Geometry &g = p.g;
    const int lmax = g.lmax, s = g.spin, M = g.mmax;
    p.syn_seg = 0;
    p.syn_parts = 0;
    p.n_syn_items = 0;
    const int R = psht::leg_rings_per_lane() == 1 ? 1 : 2, chunk = 64 * R;
    auto steps_cost = [&](int nr) { return (R > 1 && nr <= 64) ? 1.0 / R : 1.0; };
    double total = 0.0;
    for (int m = 0; m <= M; ++m) {
        if (first[m] < 0 || std::max(m, s) > lmax) continue;
        const int steps = lmax + 1 - std::max(m, s);
        for (int jb = first[m]; jb <= last[m]; jb += chunk)
            total += steps * steps_cost(std::min(chunk, last[m] + 1 - jb));
    }
    const double slots = (double)std::max(ncu, 1) * 4 * 2;
    int Ssyn = S;
    while ((double)Ssyn * 2 <= total / slots / 3.0) Ssyn *= 2;
    // at most 32 partial copies of F (a tiny cap at very high lmax would
    // otherwise take hundreds, each as large as F, in the workspace)
    while ((int64_t)33 * Ssyn < (int64_t)lmax + 1 - s) Ssyn *= 2;
    if (const char *e = getenv("PSHT_SYN_SEG")) {  // tuning runs: a power-of-two multiple of S, 0 for none
        const int v = atoi(e);
        if (v == 0) Ssyn = lmax + 1;
        else if (v >= S && v % S == 0 && ((v / S) & (v / S - 1)) == 0) Ssyn = v;
    }
    // at most two segments for the longest order: the plain work list (two
    // measured within the noise of one, and cost the partial-sum launch)
    if (3 * Ssyn > lmax + 1 - s) return true;
    const int q = Ssyn / S;
    std::vector<psht::SynSegItem> items;
    int parts = 0;
    for (int m = 0; m <= M; ++m) {
        const int l0 = std::max(m, s);
        if (first[m] < 0 || l0 > lmax) continue;
        const int nr = last[m] - first[m] + 1;
        const int nseg = (lmax + 1 - l0 + Ssyn - 1) / Ssyn;
        parts = std::max(parts, nseg - 1);
        for (int k = 0; k < nseg; ++k) {
            const int la = l0 + k * Ssyn, lb = std::min(lmax + 1, la + Ssyn);
            for (int jb = first[m]; jb <= last[m]; jb += chunk) {
                const int je = std::min(jb + chunk, last[m] + 1);
                // segment k starts at the adjoint's segment k q >= 1 (stored when nseg_adj > 1)
                const int64_t so = k == 0 ? -1 : soff_m[m] + (int64_t)(k * q - 1) * nr + (jb - first[m]);
                items.push_back(psht::SynSegItem{m, jb, je, la, lb, k, so});
            }
        }
    }
    // longest first (blocks are issued in order and dealt round-robin to the XCDs)
    std::stable_sort(items.begin(), items.end(), [&](const psht::SynSegItem &u, const psht::SynSegItem &v) {
        return (u.lb - u.la) * steps_cost(u.je - u.jb) > (v.lb - v.la) * steps_cost(v.je - v.jb);
    });
    if (!upload(p, p.d_syn_items, items, st)) return false;
    p.n_syn_items = (int)items.size();
    p.syn_seg = Ssyn;
    p.syn_parts = parts;
    p.syn_r = R;
    return true;
}

// Work list and recurrence states of the segmented Legendre adjoint.
//
// Order m has the active rings [first_m, last_m] (ring_mmax >= m) and the
// degrees l0 .. lmax, l0 = max(m, s).  The plan takes the smallest G of 1, 2, 4
// waves per workgroup with 384 G >= rings (at most 6 rings per lane; whole
// workgroups then fill a CU's eight wave slots) and splits each order's ring
// range evenly over them (R_m rings per lane).  The segment length S is the
// largest power of two (at least 64) for which the longest item costs at most
// a third of the average work per wave slot (two waves per SIMD): with
// longest-first placement the last items then finish close together.
// Segments k >= 1 start from stored states (40 bytes per ring and segment).
// An order with more active rings than one item holds (1536 at G = 4: the
// full sky above lmax ~ 3000, the partial sky near lmax 10000) is cut into
// ring groups; their items add into the output, which is cleared first.
bool build_adjoint_segments(psht_plan_s &p, int ncu, hipStream_t st, psht::Error &err) {
    const psht::Geometry &g = p.g;
    const int lmax = g.lmax, s = g.spin, M = g.mmax;
    std::vector<int> first(M + 1, -1), last(M + 1, -1);
    for (int j = 0; j < g.nring; ++j)
        for (int m = 0; m <= std::min(M, (int)g.ring_mmax[j]); ++m) {
            if (first[m] < 0) first[m] = j;
            last[m] = j;
        }
    int nrmax = 1;
    for (int m = 0; m <= M; ++m)
        if (first[m] >= 0) nrmax = std::max(nrmax, last[m] - first[m] + 1);
    int G = 1;
    while (G < psht::kAdjMaxWavesHost && 64 * psht::kAdjMaxRings * G < nrmax) G *= 2;
    if (const char *e = getenv("PSHT_ADJ_WAVES")) {  // tuning runs: 1, 2 or 4, as long as the rings fit
        const int v = atoi(e);
        if ((v == 1 || v == 2 || v == 4) && 64 * psht::kAdjMaxRings * v >= nrmax) G = v;
    }
    auto rings_per_lane = [&](int m) {
        if (first[m] < 0) return 0;
        const int nr = last[m] - first[m] + 1, gm = 64 * psht::kAdjMaxRings * G;
        const int ng = (nr + gm - 1) / gm, gsize = (nr + ng - 1) / ng;
        return (gsize + 64 * G - 1) / (64 * G);
    };
    double total = 0.0;
    int rmax = 1;
    for (int m = 0; m <= M; ++m) {
        const int R = rings_per_lane(m);
        rmax = std::max(rmax, R);
        total += (double)(lmax + 1 - std::max(m, s)) * R * G;
    }
    const double slots = (double)std::max(ncu, 1) * 4 * 2;
    int S = 64;
    while (S * 2 <= lmax + 1 && (double)(S * 2) * rmax <= total / slots / 3.0) S *= 2;
    if (const char *e = getenv("PSHT_ADJ_SEG")) {  // tuning runs
        const int v = atoi(e);
        if (v >= 8 && v <= 1 << 16) S = v;
    }
    // Orders with more rings than one item holds (64 x 6 x G) are cut into
    // ring groups whose items add into a cleared output (see adj_accumulate).
    int group_max = 64 * psht::kAdjMaxRings * G;
    if (const char *e = getenv("PSHT_ADJ_GROUP")) {  // tests and tuning runs: smaller ring groups
        const int v = atoi(e);
        if (v >= 1 && v < group_max) group_max = v;
    }
    bool accumulate = false;
    std::vector<psht::AdjItem> items;
    std::vector<psht::StateItem> sitems;
    std::vector<int64_t> soff_m(M + 1, -1);  // first stored state of order m
    int64_t off = 0;
    for (int m = 0; m <= M; ++m) {
        const int l0 = std::max(m, s);
        if (first[m] < 0) {
            items.push_back(psht::AdjItem{m, 0, 0, m, lmax + 1, 0, -1});
            continue;
        }
        const int jb = first[m], je = last[m] + 1, nr = je - jb;
        const int ng = (nr + group_max - 1) / group_max, gsize = (nr + ng - 1) / ng;
        accumulate |= ng > 1;
        const int nseg = (lmax + 1 - l0 + S - 1) / S;
        for (int k = 0; k < nseg; ++k) {
            const int la = l0 + k * S, lb = std::min(lmax + 1, la + S);
            for (int q = 0; q < ng; ++q) {
                const int gb = jb + q * gsize, ge = std::min(je, gb + gsize);
                const int R = (ge - gb + 64 * G - 1) / (64 * G);
                items.push_back(psht::AdjItem{m, gb, ge, la, lb, R,
                                              k == 0 ? -1 : off + (int64_t)(k - 1) * nr + (gb - jb)});
            }
        }
        if (nseg > 1) {
            for (int j0 = jb; j0 < je; j0 += 64) sitems.push_back(psht::StateItem{m, j0, jb, je, nseg, S, off});
            soff_m[m] = off;
            off += (int64_t)(nseg - 1) * nr;
        }
    }
    // longest first (blocks are issued in order and dealt round-robin to the XCDs)
    std::stable_sort(items.begin(), items.end(), [](const psht::AdjItem &u, const psht::AdjItem &v) {
        return (int64_t)(u.lb - u.la) * std::max(u.R, 1) > (int64_t)(v.lb - v.la) * std::max(v.R, 1);
    });
    p.adj_waves = G;
    p.adj_rmax = rmax;
    p.adj_accumulate = accumulate;
    p.adj_seg = S;
    p.n_adj_states = off;
    p.alm_tail = (int64_t)(M + 1) * (2 * lmax + 1 - (M + 1)) / 2 + (M + 1);  // index(l = M + 1, m = M + 1)
    if (!dalloc(p, p.d_adj_mu, (size_t)std::max<int64_t>(off, 1) * 4) ||
        !dalloc(p, p.d_adj_k, (size_t)std::max<int64_t>(off, 1) * 2)) {
        err = {PSHT_ERR_NOMEM, "allocating the adjoint recurrence states"};
        return false;
    }
    psht::StateItem *d_sitems = nullptr;
    if (!upload(p, p.d_adj_items, items, st) || !upload(p, d_sitems, sitems, st)) {
        err = {PSHT_ERR_NOMEM, "uploading the adjoint work list"};
        return false;
    }
    p.n_adj_items = (int)items.size();
    if (!build_synth_segments(p, ncu, first, last, soff_m, S, st)) {
        err = {PSHT_ERR_NOMEM, "uploading the synthesis work list"};
        return false;
    }
    hipError_t e = psht::launch_leg_adj_states(p, d_sitems, (int)sitems.size(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        err = {PSHT_ERR_DEVICE, std::string("adjoint recurrence states: ") + hipGetErrorString(e)};
        return false;
    }
    return true;
}

psht_status plan_create_impl(psht_plan *out, int lmax, int spin, int64_t npoints, const double *theta,
                             const double *phi, double epsilon, int precision, const psht_plan_options *opts,
                             hipStream_t st) {
    if (!out) return fail(PSHT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (lmax < 0 || spin < 0 || spin > lmax) return fail(PSHT_ERR_ARG, "need lmax >= 0 and 0 <= spin <= lmax");
    if (lmax > 16384) return fail(PSHT_ERR_UNSUPPORTED, "lmax above 16384");
    if (!(epsilon >= 1e-14 && epsilon <= 1e-2)) return fail(PSHT_ERR_ARG, "epsilon must lie in [1e-14, 1e-2]");
    if (precision < PSHT_PREC_AUTO || precision > PSHT_PREC_FP64) return fail(PSHT_ERR_ARG, "unknown precision");
    // the slot layout of the sorted points (at most two entries per point) is indexed in int32
    if (npoints < 0 || npoints >= (int64_t(1) << 30)) return fail(PSHT_ERR_ARG, "npoints must lie in [0, 2^30)");
    if (npoints > 0 && (!theta || !phi)) return fail(PSHT_ERR_ARG, "theta/phi are NULL");

    // theta range and validity (one device-to-host synchronisation)
    double tmin = 0.0, tmax = 0.0;
    if (npoints > 0) {
        ScopedDevFree stats;
        hipError_t e = hipMalloc(&stats.p, sizeof(double) * 3 * 1024);
        if (e != hipSuccess) return device_fail(e, "allocating point statistics");
        e = psht::launch_point_stats(theta, phi, npoints, static_cast<double *>(stats.p), st);
        if (e != hipSuccess) return device_fail(e, "point statistics kernel");
        std::vector<double> h(3 * 1024);
        e = hipMemcpyAsync(h.data(), stats.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "reading point statistics");
        double mn = 1e300, mx = -1e300, bad = 0;
        for (int b = 0; b < 1024; ++b) {
            mn = std::min(mn, h[3 * b]);
            mx = std::max(mx, h[3 * b + 1]);
            bad += h[3 * b + 2];
        }
        if (bad > 0)
            return fail(PSHT_ERR_ARG, "some theta outside [0, pi] or phi not finite (" +
                                          std::to_string((long long)bad) + " points)");
        tmin = mn;
        tmax = mx;
    }

    std::unique_ptr<psht_plan_s, void (*)(psht_plan_s *)> plan(new psht_plan_s(), free_plan);
    psht_plan_s &p = *plan;
    p.npts = npoints;
    psht::Error err;
    if (!psht::geometry_compute(p.g, lmax, spin, tmax, tmin, epsilon, precision, true, err, true, opts))
        return fail(err);
    const psht::Geometry &g = p.g;
    const bool fp32 = g.fp32;
    const int fmax = fp32 ? psht::kFftMaxLds32 : psht::kFftMaxLds64;
    // The Theta grid (NT = 2 N2 points) above the LDS limit runs as two N2-point
    // transforms (even and odd rows); N2 itself must fit.
    if (g.N2 > fmax)
        return fail(PSHT_ERR_UNSUPPORTED, "Theta circle of " + std::to_string(g.N2) + " samples exceeds the LDS FFT limit");
    p.theta_split = g.Ntheta > fmax;
    if (const char *e = getenv("PSHT_THETA_SPLIT"))  // tests and tuning runs: 1 forces the split where possible
        if (atoi(e) == 1 && g.Ntheta == 2 * g.N2) p.theta_split = true;
    if (p.theta_split && g.Ntheta != 2 * g.N2)
        return fail(PSHT_ERR_UNSUPPORTED, "Theta grid above the LDS limit that is not twice the circle");
    // phi rows run as g.phi_parts transforms of Nphi / phi_parts points (see params.cpp)
    if (g.Nphi / g.phi_parts > fmax)
        return fail(PSHT_ERR_UNSUPPORTED, "phi grid of " + std::to_string(g.Nphi) + " exceeds the LDS FFT limit");

    p.leg = psht::leg_table_get(lmax, spin, err);
    if (!p.leg) return fail(err);

    // rings
    std::vector<double> ry(g.nring), rch(g.nring), rsh(g.nring);
    for (int j = 0; j < g.nring; ++j) {
        long double t = g.ring_theta[j], sh = sinl(t / 2);
        ry[j] = (double)(2 * sh * sh);
        rch[j] = (double)cosl(t / 2);
        rsh[j] = (double)sh;
    }
    if (!upload(p, p.d_ring_y, ry, st) || !upload(p, p.d_ring_ch, rch, st) || !upload(p, p.d_ring_sh, rsh, st) ||
        !upload(p, p.d_ring_w, g.ring_w, st) || !upload(p, p.d_ring_mmax, g.ring_mmax, st))
        return fail(PSHT_ERR_NOMEM, "uploading ring tables");

    // Legendre work items: `group` chunks of `chunk` rings per order m, groups
    // padded to a multiple of 8.  One list for the per-map kernels (64 R rings
    // per wave) and one of 64-ring chunks for the batched-maps kernel.
    {
        auto build_items = [&](int chunk, std::vector<psht::LegItem> &items) {
            const int group = (g.nring + chunk - 1) / chunk;
            const int ngroups = ((g.mmax + 1) + 7) / 8 * 8;
            items.assign((size_t)ngroups * group, psht::LegItem{0, 0, 0});
            for (int m = 0; m <= g.mmax; ++m) {
                int first = -1, last = -1;
                for (int j = 0; j < g.nring; ++j)
                    if (g.ring_mmax[j] >= m) {
                        if (first < 0) first = j;
                        last = j;
                    }
                for (int c = 0; c < group; ++c) {
                    psht::LegItem &it = items[(size_t)m * group + c];
                    it.m = m;
                    if (first < 0) continue;
                    int jb = first + c * chunk, je = std::min(first + (c + 1) * chunk, last + 1);
                    if (jb < je) {
                        it.jb = jb;
                        it.je = je;
                    }
                }
            }
        };
        // Synthesis order.  The kernel deals item slot (x + 8 q) group + i to the
        // XCD x, in the order of q and i; the items of each XCD are placed in
        // those slots longest first by their cost in the synthesis, where an
        // item of at most 64 rings runs the one-ring-per-lane body at 1/R of
        // the cost (longest-processing-time-first list scheduling; in the plain
        // order these short remainders sat between the full items of their m).
        auto order_for_synth = [&](std::vector<psht::LegItem> &items, int chunk, int R) {
            const int group = (g.nring + chunk - 1) / chunk;
            const int nq = (int)(items.size() / group) / 8;
            auto cost = [&](const psht::LegItem &it) {
                if (it.je <= it.jb) return 0.0;
                const double steps = lmax + 1 - std::max(it.m, spin);
                return (R > 1 && it.je - it.jb <= 64) ? steps / R : steps;
            };
            for (int x = 0; x < 8; ++x) {
                std::vector<size_t> slots;
                for (int q = 0; q < nq; ++q)
                    for (int i = 0; i < group; ++i) slots.push_back((size_t)(x + 8 * q) * group + i);
                std::vector<psht::LegItem> mine;
                for (size_t sl : slots) mine.push_back(items[sl]);
                std::stable_sort(mine.begin(), mine.end(),
                                 [&](const psht::LegItem &u, const psht::LegItem &v) { return cost(u) > cost(v); });
                for (size_t k = 0; k < slots.size(); ++k) items[slots[k]] = mine[k];
            }
        };
        std::vector<psht::LegItem> items;
        int dev = 0, ncu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        auto nonempty = [](const std::vector<psht::LegItem> &v) {
            size_t n = 0;
            for (const auto &it : v) n += it.je > it.jb;
            return n;
        };
        // Synthesis rings per lane.  Small plans whose two-ring items fill less
        // than 40 % of the GPU's wave slots (four per SIMD) run one ring per lane:
        // twice the items, each step half the work, so the longest items finish
        // sooner (lmax 2048, 10-degree disc: 0.165 -> 0.132 ms).  From about half
        // the slots on, two rings per lane are faster (lmax 4096, 20-degree disc:
        // 0.81 against 0.99 ms).
        int rs = psht::leg_rings_per_lane();
        if (rs == 0) {
            build_items(64 * 2, items);
            rs = (ncu > 0 && (double)nonempty(items) < 0.4 * ncu * 4 * 4) ? 1 : 2;
        }
        const int chunk = 64 * rs;
        build_items(chunk, items);
        order_for_synth(items, chunk, rs);
        p.n_leg_items = (int)items.size();
        p.leg_rings_per_item = chunk;
        if (!upload(p, p.d_leg_items, items, st)) return fail(PSHT_ERR_NOMEM, "uploading Legendre work list");
        build_items(64, items);
        p.n_leg_items64 = (int)items.size();
        if (!upload(p, p.d_leg_items64, items, st)) return fail(PSHT_ERR_NOMEM, "uploading Legendre work list");

        // Segmented adjoint (k_leg_adj_seg): items (m, l-segment), each with every
        // active ring of m in G waves of up to 6 rings per lane, started from
        // recurrence states stored here for every ring and segment start.
        psht::Error e2;
        if (!build_adjoint_segments(p, ncu, st, e2)) return fail(e2);
    }

    // NUFFT tables
    if (!upload(p, p.d_psihat_t, g.psihat_theta, st) || !upload(p, p.d_psihat_p, g.psihat_phi, st) ||
        (!g.es_poly.empty() && !upload(p, p.d_es_poly, g.es_poly, st)) ||
        (!g.es_poly32.empty() && !upload(p, p.d_es_poly32, g.es_poly32, st)))
        return fail(PSHT_ERR_NOMEM, "uploading kernel tables");
    if (!make_fft_table(p, p.fft_n2, g.N2, st) || !make_fft_table(p, p.fft_nt, g.Ntheta, st) ||
        !make_fft_table(p, p.fft_np, g.Nphi, st))
        return fail(PSHT_ERR_NOMEM, "FFT tables");
    if (g.phi_parts > 1 && !make_fft_table(p, p.fft_np_part, g.Nphi / g.phi_parts, st))
        return fail(PSHT_ERR_NOMEM, "FFT tables");

    // points: bucket sort into tiles (PSHT_TILE="<rows>x<cols>" overrides the tile shape for tuning runs)
    if (const char *ts = getenv("PSHT_TILE")) {
        int tx = 0, ty = 0;
        if (sscanf(ts, "%dx%d", &tx, &ty) == 2 && tx >= 4 && ty >= 8 && tx <= 64 && ty <= 128 &&
            (size_t)(tx + g.W - 1) * ((ty + g.W - 1) | 1) * 16 <= 65536) {
            p.tile_x = tx;
            p.tile_y = ty;
        }
    }
    p.ntx = (g.rows_used + p.tile_x - 1) / p.tile_x;
    p.nty = (g.Nphi + p.tile_y - 1) / p.tile_y;
    p.ntiles = p.ntx * p.nty;
    if (!dalloc(p, p.d_tile_start, (size_t)p.ntiles + 1) || !dalloc(p, p.d_dropped, 2))
        return fail(PSHT_ERR_NOMEM, "allocating sorted points");
    if (psht::launch_fill_zero(p.d_dropped, 2 * sizeof(unsigned long long), st) != hipSuccess)
        return fail(PSHT_ERR_DEVICE, "clearing the point counters");
    {
        ScopedDevFree keys, cursor, pstart, tpx, tpy, tperm;
        const size_t nn = (size_t)std::max<int64_t>(npoints, 1);
        hipError_t e = hipMalloc(&keys.p, sizeof(int32_t) * nn);
        if (e == hipSuccess) e = hipMalloc(&cursor.p, sizeof(int32_t) * (size_t)p.ntiles);
        if (e == hipSuccess) e = hipMalloc(&pstart.p, sizeof(int32_t) * ((size_t)p.ntiles + 1));
        if (e == hipSuccess) e = hipMalloc(&tpx.p, sizeof(double) * nn);
        if (e == hipSuccess) e = hipMalloc(&tpy.p, sizeof(double) * nn);
        if (e == hipSuccess) e = hipMalloc(&tperm.p, sizeof(int32_t) * nn);
        if (e != hipSuccess) return device_fail(e, "sort scratch");
        e = psht::launch_point_sort_count(p, theta, phi, static_cast<int32_t *>(keys.p),
                                          static_cast<int32_t *>(cursor.p), static_cast<int32_t *>(pstart.p),
                                          static_cast<double *>(tpx.p), static_cast<double *>(tpy.p),
                                          static_cast<int32_t *>(tperm.p), st);
        int32_t total = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&total, p.d_tile_start + p.ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "point sort");
        p.n_entries = total;
        const size_t ne = (size_t)std::max<int64_t>(p.n_entries, 1);
        if (!dalloc(p, p.d_px, ne) || !dalloc(p, p.d_py, ne) || !dalloc(p, p.d_perm, ne))
            return fail(PSHT_ERR_NOMEM, "allocating sorted points");
        // p.d_dropped[1] counts sorted entries outside their tile
        e = psht::launch_point_sort_order(p, static_cast<int32_t *>(keys.p), static_cast<const int32_t *>(pstart.p),
                                          static_cast<const double *>(tpx.p), static_cast<const double *>(tpy.p),
                                          static_cast<const int32_t *>(tperm.p), p.d_dropped + 1, st);
        unsigned long long bad = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad, p.d_dropped + 1, sizeof(bad), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "point sort");
        if (bad != 0)
            return fail(PSHT_ERR_DEVICE, "internal error: " + std::to_string(bad) +
                                             " sorted points have a stencil outside their NUFFT tile");
    }

    // workspace per map
    const size_t cs = fp32 ? 8 : 16;
    p.ws_F = align256((size_t)(2 * g.mmax + 1) * g.nring * 16);
    p.ws_V = align256((size_t)g.rows_used * (2 * g.mmax + 1) * cs);
    p.ws_U = align256((size_t)g.rows_used * g.Nphi * cs);
    // the synthesis' partial copies of F use the V and U region, which is
    // free until the Legendre stage has added them into F
    p.ws_per_map = p.ws_F + std::max(p.ws_V + p.ws_U, (size_t)p.syn_parts * p.ws_F);
    *out = plan.release();
    return PSHT_OK;
}

// Smallest number of maps that takes the batched Legendre pass: its cost does
// not depend on the number of maps (the MFMA tiles always hold 8), and it
// beats the one-map pass from about 4.6 maps on (PSHT_MM_MIN overrides it
// for tuning runs; a value above 8 disables the batched pass).
int leg_batch_min() {
    static int v = [] {
        const char *e = getenv("PSHT_MM_MIN");
        const int x = e ? atoi(e) : 5;
        return x >= 2 ? x : 5;
    }();
    return v;
}

bool check_ws(const psht_plan_s &p, int nmaps, void *ws, size_t ws_bytes) {
    if (nmaps == 0) return true;
    return ws != nullptr && ws_bytes >= (size_t)nmaps * p.ws_per_map;
}

}  // namespace

psht_status psht::set_error(psht_status code, const char *msg) { return fail(code, msg); }

extern "C" {

psht_status psht_plan_create(psht_plan *out, int lmax, int spin, int64_t npoints, const double *theta,
                             const double *phi, double epsilon, int precision, void *hip_stream) {
    return psht_plan_create_ex(out, lmax, spin, npoints, theta, phi, epsilon, precision, nullptr, hip_stream);
}

psht_status psht_plan_create_ex(psht_plan *out, int lmax, int spin, int64_t npoints, const double *theta,
                                const double *phi, double epsilon, int precision, const psht_plan_options *opts,
                                void *hip_stream) {
    try {
        return plan_create_impl(out, lmax, spin, npoints, theta, phi, epsilon, precision, opts,
                                static_cast<hipStream_t>(hip_stream));
    } catch (const std::bad_alloc &) {
        return fail(PSHT_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(PSHT_ERR_DEVICE, e.what());
    } catch (...) {
        return fail(PSHT_ERR_DEVICE, "unknown error");
    }
}

psht_status psht_plan_query(psht_plan plan, psht_plan_info *info) {
    if (!plan || !info) return fail(PSHT_ERR_ARG, "plan or info is NULL");
    fill_info(*plan, info);
    return PSHT_OK;
}

}  // extern "C"

namespace {

}  // namespace

// Synthesis of nmaps maps with the given workspace (shared by psht_synth,
// psht_synth_grad and the entry point without allocation).
psht_status psht::synth_run(psht_plan plan, int nmaps, const void *alm, void *map, void *workspace, size_t ws_bytes,
                            double mscale, void *hip_stream) {
    if (!plan) return fail(PSHT_ERR_ARG, "plan is NULL");
    if (nmaps < 0) return fail(PSHT_ERR_ARG, "nmaps < 0");
    if (nmaps > 0 && (!alm || (!map && plan->npts > 0))) return fail(PSHT_ERR_ARG, "alm or map is NULL");
    if (!check_ws(*plan, nmaps, workspace, ws_bytes))
        return fail(PSHT_ERR_WORKSPACE, "workspace smaller than nmaps * workspace_bytes_per_map");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const psht::Geometry &g = plan->g;
    const size_t alm_bytes = (size_t)(g.lmax + 1) * (g.lmax + 2) / 2 * 2 * 16;
    const size_t map_bytes = (size_t)plan->npts * (g.fp32 ? 8 : 16);
    psht_plan_s &P = *plan;
    const int batch_min = leg_batch_min();
    for (int i = 0; i < nmaps;) {
        // groups of batch_min..8 maps share one batched (MFMA) Legendre pass
        const int nb = nmaps - i >= batch_min ? std::min(nmaps - i, psht::kMaxLegBatch) : 1;
        char *ws0 = static_cast<char *>(workspace) + (size_t)i * plan->ws_per_map;
        const char *a0 = static_cast<const char *>(alm) + i * alm_bytes;
        hipError_t e;
        if (nb > 1)
            e = timed(P, PSHT_T_LEG_SYNTH, st, [&] {
                return psht::launch_leg_synth_batch(P, nb, a0, (int64_t)alm_bytes, ws0, (int64_t)plan->ws_per_map,
                                                    mscale, st);
            });
        else
            e = timed(P, PSHT_T_LEG_SYNTH, st, [&] {
                return psht::launch_leg_synth_parts(P, a0, reinterpret_cast<double *>(ws0),
                                                    reinterpret_cast<double *>(ws0 + plan->ws_F),
                                                    (int64_t)(plan->ws_F / 8), mscale, st);
            });
        for (int b = 0; b < nb && e == hipSuccess; ++b) {
            char *ws = ws0 + (size_t)b * plan->ws_per_map;
            double *F = reinterpret_cast<double *>(ws);
            void *V = ws + plan->ws_F;
            void *U = ws + plan->ws_F + plan->ws_V;
            void *m = static_cast<char *>(map) + (size_t)(i + b) * map_bytes;
            e = timed(P, PSHT_T_THETA_SYNTH, st, [&] { return psht::launch_theta_synth(P, F, V, st); });
            if (e == hipSuccess) e = timed(P, PSHT_T_PHI_SYNTH, st, [&] { return psht::launch_phi_synth(P, V, U, st); });
            if (e == hipSuccess) e = timed(P, PSHT_T_INTERP, st, [&] { return psht::launch_interp(P, U, m, st); });
        }
        if (e != hipSuccess) return device_fail(e, "synthesis launch");
        i += nb;
    }
    return PSHT_OK;
}

namespace {

psht_status adjoint_impl(psht_plan plan, int nmaps, const void *map, void *alm, void *workspace, size_t ws_bytes,
                         double mscale, void *hip_stream) {
    if (!plan) return fail(PSHT_ERR_ARG, "plan is NULL");
    if (nmaps < 0) return fail(PSHT_ERR_ARG, "nmaps < 0");
    if (nmaps > 0 && (!alm || (!map && plan->npts > 0))) return fail(PSHT_ERR_ARG, "alm or map is NULL");
    if (!check_ws(*plan, nmaps, workspace, ws_bytes))
        return fail(PSHT_ERR_WORKSPACE, "workspace smaller than nmaps * workspace_bytes_per_map");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const psht::Geometry &g = plan->g;
    const size_t alm_bytes = (size_t)(g.lmax + 1) * (g.lmax + 2) / 2 * 2 * 16;
    const size_t map_bytes = (size_t)plan->npts * (g.fp32 ? 8 : 16);
    for (int i = 0; i < nmaps; ++i) {
        char *ws = static_cast<char *>(workspace) + (size_t)i * plan->ws_per_map;
        double *F = reinterpret_cast<double *>(ws);
        void *V = ws + plan->ws_F;
        void *U = ws + plan->ws_F + plan->ws_V;
        void *a = static_cast<char *>(alm) + i * alm_bytes;
        const void *m = static_cast<const char *>(map) + i * map_bytes;
        psht_plan_s &P = *plan;
        hipError_t e = timed(P, PSHT_T_GRID_ZERO, st, [&] { return psht::launch_fill_zero(U, P.ws_U, st); });
        if (e == hipSuccess) e = timed(P, PSHT_T_SPREAD, st, [&] { return psht::launch_spread(P, m, U, st); });
        if (e == hipSuccess) e = timed(P, PSHT_T_PHI_ADJ, st, [&] { return psht::launch_phi_adjoint(P, U, V, st); });
        if (e == hipSuccess) e = timed(P, PSHT_T_THETA_ADJ, st, [&] { return psht::launch_theta_adjoint(P, V, F, st); });

        if (e == hipSuccess) e = timed(P, PSHT_T_LEG_ADJ, st, [&] { return psht::launch_leg_adjoint(P, F, a, mscale, st); });
        if (e != hipSuccess) return device_fail(e, "adjoint launch");
    }
    return PSHT_OK;
}

}  // namespace

extern "C" {

psht_status psht_synth(psht_plan plan, int nmaps, const void *alm, void *map, void *workspace, size_t ws_bytes,
                       void *hip_stream) {
    return psht::synth_run(plan, nmaps, alm, map, workspace, ws_bytes, 1.0, hip_stream);
}

psht_status psht_adjoint(psht_plan plan, int nmaps, const void *map, void *alm, void *workspace, size_t ws_bytes,
                         void *hip_stream) {
    return adjoint_impl(plan, nmaps, map, alm, workspace, ws_bytes, 1.0, hip_stream);
}

psht_status psht_adjoint_grad(psht_plan plan, int nmaps, const void *map_grad, void *alm_grad, void *workspace,
                              size_t ws_bytes, void *hip_stream) {
    return adjoint_impl(plan, nmaps, map_grad, alm_grad, workspace, ws_bytes, 2.0, hip_stream);
}

psht_status psht_synth_grad(psht_plan plan, int nmaps, const void *alm_grad, void *map_grad, void *workspace,
                            size_t ws_bytes, void *hip_stream) {
    return psht::synth_run(plan, nmaps, alm_grad, map_grad, workspace, ws_bytes, 0.5, hip_stream);
}

void psht_plan_destroy(psht_plan plan) { free_plan(plan); }

psht_status psht_plan_set_timing(psht_plan plan, int stages) {
    if (!plan) return fail(PSHT_ERR_ARG, "plan is NULL");
    for (auto &e : plan->pending) {
        (void)hipEventSynchronize(e.second.second);
        plan->event_pool.push_back(e.second.first);
        plan->event_pool.push_back(e.second.second);
    }
    plan->pending.clear();
    for (int i = 0; i < PSHT_T_COUNT; ++i) {
        plan->t_ms[i] = 0;
        plan->t_launches[i] = 0;
    }
    plan->timing = (unsigned)stages & (unsigned)PSHT_T_ALL;
    // events for 32 calls ahead: none is created while timed work is issued
    const int want = 64 * __builtin_popcount(plan->timing);
    while ((int)plan->event_pool.size() < want) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return fail(PSHT_ERR_DEVICE, "creating timing events");
        plan->event_pool.push_back(e);
    }
    return PSHT_OK;
}

psht_status psht_plan_timing(psht_plan plan, double *ms, int64_t *launches) {
    if (!plan || !ms || !launches) return fail(PSHT_ERR_ARG, "NULL argument");
    for (auto &e : plan->pending) {
        hipError_t r = hipEventSynchronize(e.second.second);
        float t = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&t, e.second.first, e.second.second);
        if (r != hipSuccess) return device_fail(r, "timing events");
        plan->t_ms[e.first] += t;
        plan->t_launches[e.first] += 1;
        plan->event_pool.push_back(e.second.first);
        plan->event_pool.push_back(e.second.second);
    }
    plan->pending.clear();
    for (int i = 0; i < PSHT_T_COUNT; ++i) {
        ms[i] = plan->t_ms[i];
        launches[i] = plan->t_launches[i];
    }
    return PSHT_OK;
}

const char *psht_last_error(void) { return g_last_error.c_str(); }

psht_status psht_rotate_alm_workspace(int lmax, int ncomp, size_t *bytes) {
    if (lmax < 0 || lmax > 16383 || (ncomp != 1 && ncomp != 2) || !bytes)
        return fail(PSHT_ERR_ARG, "need 0 <= lmax <= 16383, ncomp 1 or 2, bytes not NULL");
    *bytes = (size_t)ncomp * (size_t)(lmax + 1) * (size_t)(2 * lmax + 1) * 16;
    return PSHT_OK;
}

psht_status psht_rotate_alm(int lmax, int ncomp, double alpha, double beta, double gamma, const void *alm_in,
                            void *alm_out, void *workspace, size_t ws_bytes, void *hip_stream) {
    size_t need = 0;
    if (psht_rotate_alm_workspace(lmax, ncomp, &need) != PSHT_OK) return PSHT_ERR_ARG;
    if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(gamma))
        return fail(PSHT_ERR_ARG, "rotation angles must be finite");
    if (!alm_in || !alm_out || !workspace) return fail(PSHT_ERR_ARG, "NULL array");
    const size_t bytes = (size_t)ncomp * (size_t)(lmax + 1) * (size_t)(lmax + 2) / 2 * 16;
    const char *a = (const char *)alm_in, *b = (const char *)alm_out;
    if (a < b + bytes && b < a + bytes) return fail(PSHT_ERR_ARG, "alm_in and alm_out overlap");
    if (ws_bytes < need) return fail(PSHT_ERR_WORKSPACE, "workspace smaller than psht_rotate_alm_workspace");
    // log2(n!) for n = 0..2 lmax, per (device, lmax), kept for the process lifetime
    static std::mutex mu;
    static std::map<std::pair<int, int>, double2 *> tables;
    double2 *lf = nullptr;
    {
        std::lock_guard<std::mutex> lock(mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        auto key = std::make_pair(dev, lmax);
        auto it = tables.find(key);
        if (it != tables.end()) {
            lf = it->second;
        } else try {
            std::vector<double2> h(2 * (size_t)lmax + 1);
            for (size_t n = 0; n < h.size(); ++n) {
                const long double v = lgammal((long double)n + 1) / logl(2.0L);
                h[n].x = (double)v;
                h[n].y = (double)(v - (long double)h[n].x);
            }
            void *d = nullptr;
            hipError_t e = hipMalloc(&d, h.size() * sizeof(double2));
            if (e != hipSuccess) return device_fail(e, "log-factorial table");
            e = hipMemcpy(d, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(d);
                return device_fail(e, "log-factorial table");
            }
            tables[key] = (double2 *)d;
            lf = (double2 *)d;
        } catch (const std::bad_alloc &) {
            return fail(PSHT_ERR_NOMEM, "host allocation failed");
        }
    }
    hipError_t e = psht::launch_rotate_alm(lmax, ncomp, alpha, beta, gamma, alm_in, alm_out, workspace, lf,
                                           static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? PSHT_OK : device_fail(e, "rotation kernels");
}

psht_status psht_rotate_points(int64_t npoints, double alpha, double beta, double gamma, const double *theta,
                               const double *phi, double *theta_out, double *phi_out, double *psi_out,
                               void *hip_stream) {
    if (npoints < 0) return fail(PSHT_ERR_ARG, "npoints < 0");
    if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(gamma))
        return fail(PSHT_ERR_ARG, "rotation angles must be finite");
    if (npoints > 0 && (!theta || !phi || !theta_out || !phi_out || !psi_out))
        return fail(PSHT_ERR_ARG, "NULL array");
    psht::RotMatrix R;
    const double ca = std::cos(alpha), sa = std::sin(alpha), cb = std::cos(beta), sb = std::sin(beta),
                 cg = std::cos(gamma), sg = std::sin(gamma);
    // Rz(alpha) Ry(beta) Rz(gamma)
    const double Y[3][3] = {{cb * cg, -cb * sg, sb}, {sg, cg, 0.0}, {-sb * cg, sb * sg, cb}};
    for (int c = 0; c < 3; ++c) {
        R.r[0][c] = ca * Y[0][c] - sa * Y[1][c];
        R.r[1][c] = sa * Y[0][c] + ca * Y[1][c];
        R.r[2][c] = Y[2][c];
    }
    hipError_t e = psht::launch_rotate_points(npoints, R, theta, phi, theta_out, phi_out, psi_out,
                                              static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? PSHT_OK : device_fail(e, "point rotation kernel");
}

psht_status psht_spin_phase(int64_t npoints, int spin, int sign, int fp32, const double *psi, void *map,
                            void *hip_stream) {
    if (npoints < 0 || (sign != 1 && sign != -1) || (fp32 != 0 && fp32 != 1))
        return fail(PSHT_ERR_ARG, "need npoints >= 0, sign +-1, fp32 0 or 1");
    if (npoints > 0 && (!psi || !map)) return fail(PSHT_ERR_ARG, "NULL array");
    hipError_t e = psht::launch_spin_phase(npoints, (double)sign * spin, fp32, psi, map,
                                           static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? PSHT_OK : device_fail(e, "spin phase kernel");
}

psht_status psht_great_circle_spectrum(int lmax, int spin, const double *cl, double *cm) {
    if (lmax < 0 || spin < 0 || spin > lmax || !cl || !cm) return fail(PSHT_ERR_ARG, "bad arguments");
    try {
        std::vector<double> v;
        psht::great_circle_spectrum(lmax, spin, cl, v);
        std::copy(v.begin(), v.end(), cm);
        return PSHT_OK;
    } catch (...) {
        return fail(PSHT_ERR_NOMEM, "host allocation failed");
    }
}

psht_status psht_plan_check(psht_plan plan, int64_t *dropped, void *hip_stream) {
    if (!plan || !dropped) return fail(PSHT_ERR_ARG, "plan or dropped is NULL");
    *dropped = 0;
    if (!plan->d_dropped) return PSHT_OK;
    unsigned long long v = 0;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(&v, plan->d_dropped, sizeof(v), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "reading the point counter");
    *dropped = (int64_t)v;
    return PSHT_OK;
}

psht_status psht_plan_geometry(int lmax, int spin, double theta_star, double epsilon, int precision,
                               psht_plan_info *info, double *ring_theta, double *ring_weight, int32_t *ring_mmax,
                               int capacity) {
    return psht_plan_geometry_ex(lmax, spin, theta_star, epsilon, precision, nullptr, info, ring_theta, ring_weight,
                                 ring_mmax, capacity);
}

psht_status psht_plan_geometry_ex(int lmax, int spin, double theta_star, double epsilon, int precision,
                                  const psht_plan_options *opts, psht_plan_info *info, double *ring_theta,
                                  double *ring_weight, int32_t *ring_mmax, int capacity) {
    try {
        if (!info) return fail(PSHT_ERR_ARG, "info is NULL");
        if (capacity < 0 || (capacity > 0 && (!ring_theta || !ring_weight || !ring_mmax)))
            return fail(PSHT_ERR_ARG, "ring arrays are NULL");
        psht_plan_s p;
        psht::Error err;
        if (!psht::geometry_compute(p.g, lmax, spin, theta_star, 0.0, epsilon, precision, false, err, capacity > 0,
                                    opts))
            return fail(err);
        fill_info(p, info);
        info->workspace_bytes_per_map = 0;
        info->resident_bytes = 0;
        int n = std::min(capacity, p.g.nring);
        for (int j = 0; j < n; ++j) {
            ring_theta[j] = p.g.ring_theta[j];
            ring_weight[j] = p.g.ring_w[j];
            ring_mmax[j] = p.g.ring_mmax[j];
        }
        return PSHT_OK;
    } catch (const std::bad_alloc &) {
        return fail(PSHT_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(PSHT_ERR_DEVICE, "unknown error");
    }
}

psht_status psht_stage_ex(psht_plan plan, int stage, const void *in, void *out, void *workspace, size_t ws_bytes,
                          void *hip_stream) {
    if (stage == PSHT_STAGE_LEGENDRE_SYNTH && workspace != nullptr && plan != nullptr && plan->syn_seg > 0) {
        // with a workspace: the work list synth_run uses (degree segments with
        // partial copies of F in the workspace)
        if (!in || !out) return fail(PSHT_ERR_ARG, "in or out is NULL");
        if (!check_ws(*plan, 1, workspace, ws_bytes))
            return fail(PSHT_ERR_WORKSPACE, "workspace smaller than workspace_bytes_per_map");
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        const psht::Geometry &g = plan->g;
        hipError_t e = psht::launch_fill_zero(out, (size_t)(2 * g.mmax + 1) * g.nring * 16, st);
        if (e == hipSuccess)
            e = psht::launch_leg_synth_parts(*plan, in, static_cast<double *>(out), static_cast<double *>(workspace),
                                             (int64_t)(plan->ws_F / 8), 1.0, st);
        if (e != hipSuccess) return device_fail(e, "stage launch");
        return PSHT_OK;
    }
    if (stage == PSHT_STAGE_LEGENDRE_SYNTH || stage == PSHT_STAGE_LEGENDRE_ADJOINT)
        return psht_stage(plan, stage, in, out, hip_stream);
    if (stage != PSHT_STAGE_FOURIER_SYNTH && stage != PSHT_STAGE_FOURIER_ADJOINT)
        return fail(PSHT_ERR_ARG, "unknown stage");
    if (!plan || !in || !out) return fail(PSHT_ERR_ARG, "plan, in or out is NULL");
    if (!check_ws(*plan, 1, workspace, ws_bytes))
        return fail(PSHT_ERR_WORKSPACE, "workspace smaller than workspace_bytes_per_map");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    psht_plan_s &P = *plan;
    char *ws = static_cast<char *>(workspace);
    void *V = ws + P.ws_F;
    void *U = ws + P.ws_F + P.ws_V;
    hipError_t e;
    if (stage == PSHT_STAGE_FOURIER_SYNTH) {
        e = psht::launch_theta_synth(P, static_cast<const double *>(in), V, st);
        if (e == hipSuccess) e = psht::launch_phi_synth(P, V, U, st);
        if (e == hipSuccess) e = psht::launch_interp(P, U, out, st);
    } else {
        e = psht::launch_fill_zero(U, P.ws_U, st);
        if (e == hipSuccess) e = psht::launch_spread(P, in, U, st);
        if (e == hipSuccess) e = psht::launch_phi_adjoint(P, U, V, st);
        if (e == hipSuccess) e = psht::launch_theta_adjoint(P, V, static_cast<double *>(out), st);
    }
    if (e != hipSuccess) return device_fail(e, "stage launch");
    return PSHT_OK;
}

psht_status psht_stage(psht_plan plan, int stage, const void *in, void *out, void *hip_stream) {
    if (!plan || !in || !out) return fail(PSHT_ERR_ARG, "plan, in or out is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const psht::Geometry &g = plan->g;
    hipError_t e;
    if (stage == PSHT_STAGE_LEGENDRE_SYNTH) {
        e = psht::launch_fill_zero(out, (size_t)(2 * g.mmax + 1) * g.nring * 16, st);
        if (e == hipSuccess) e = psht::launch_leg_synth(*plan, in, static_cast<double *>(out), 1.0, st);
    } else if (stage == PSHT_STAGE_LEGENDRE_ADJOINT) {
        e = psht::launch_fill_zero(out, (size_t)(g.lmax + 1) * (g.lmax + 2) / 2 * 2 * 16, st);
        if (e == hipSuccess) e = psht::launch_leg_adjoint(*plan, static_cast<const double *>(in), out, 1.0, st);
    } else {
        return fail(PSHT_ERR_ARG, "unknown stage");
    }
    if (e != hipSuccess) return device_fail(e, "stage launch");
    return PSHT_OK;
}

psht_status psht_fft(int n, int batch, int sign, int fp32, const void *in, void *out, void *hip_stream) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, psht_plan_s *> tables;  // kept for the process lifetime
    if (n < 1 || batch < 0 || (sign != 1 && sign != -1)) return fail(PSHT_ERR_ARG, "bad n, batch or sign");
    if (batch > 0 && (!in || !out)) return fail(PSHT_ERR_ARG, "in or out is NULL");
    if (n > (fp32 ? psht::kFftMaxLds32 : psht::kFftMaxLds64)) return fail(PSHT_ERR_UNSUPPORTED, "n above the LDS limit");
    psht::FftFactors f;
    if (!psht::fft_factor(n, f)) return fail(PSHT_ERR_UNSUPPORTED, "n has a prime factor outside 2,3,5,7,11,13");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    psht_plan_s *holder;
    {
        std::lock_guard<std::mutex> lock(mu);
        int dev = 0;
        (void)hipGetDevice(&dev);
        auto key = std::make_pair(n, dev);
        auto it = tables.find(key);
        if (it == tables.end()) {
            holder = new psht_plan_s();
            if (!make_fft_table(*holder, holder->fft_np, n, st) || hipStreamSynchronize(st) != hipSuccess) {
                free_plan(holder);
                return fail(PSHT_ERR_NOMEM, "FFT table");
            }
            tables[key] = holder;
        } else {
            holder = it->second;
        }
    }
    hipError_t e = psht::launch_fft_rows(holder->fft_np, batch, sign, fp32 != 0, in, out, st);
    if (e != hipSuccess) return device_fail(e, "fft launch");
    return PSHT_OK;
}

// Host evaluation of lambda+-_lm(theta), l = 0..lmax, with the tables, seeds,
// recurrence and rescaling the GPU kernels use (values still scaled below the
// double range are reported as zero).
psht_status psht_legendre_column(int lmax, int spin, int m, double theta, double *lam_plus, double *lam_minus) {
    if (lmax < 0 || spin < 0 || spin > lmax || m < 0 || m > lmax || !lam_plus || !lam_minus)
        return fail(PSHT_ERR_ARG, "bad arguments");
    try {
        psht::LegTable t;
        psht::leg_table_host(t, lmax, spin);
        for (int l = 0; l <= lmax; ++l) lam_plus[l] = lam_minus[l] = 0.0;
        const int l0 = std::max(m, spin);
        double up, um, upp = 0.0, ump = 0.0;
        int kp, km;
        psht::leg_seed(t.h_kmant[m], t.h_kexp[m], m, spin, std::cos(theta / 2), std::sin(theta / 2), up, kp, um, km);
        const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
        const double sh = std::sin(theta / 2), y = 2 * sh * sh;
        for (int l = l0; l <= lmax; ++l) {
            const double *c = &t.h_coef[4 * (base + l)];
            lam_plus[l] = kp == 0 ? c[3] * up : 0.0;
            lam_minus[l] = km == 0 ? c[3] * um : 0.0;
            if (l < lmax) {
                double np = std::fma(std::fma(c[0], y, c[1]), up, -upp);
                upp = up;
                up = np;
                psht::leg_rescale(up, upp, kp);
                double nm = std::fma(std::fma(c[0], y, c[2]), um, -ump);
                ump = um;
                um = nm;
                psht::leg_rescale(um, ump, km);
            }
        }
        return PSHT_OK;
    } catch (...) {
        return fail(PSHT_ERR_NOMEM, "host allocation failed");
    }
}

}  // extern "C"
