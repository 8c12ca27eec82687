// Non-uniform stage of the Fourier-sphere route on gfx950: type-2
// interpolation (synthesis) and type-1 spreading (adjoint) with the
// exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1)),
// plus the plan-time point statistics and the bucket sort of the points into
// grid tiles.
//
// Grid: rows a = row_lo .. row_lo + rows_used - 1 of the oversampled Theta grid
// (spacing 2 pi / Ntheta, Theta = theta pi / theta_max, Sec. II step 3) and all
// Nphi columns (spacing 2 pi / Nphi).  A point with grid coordinates
// (X, Y) = (theta sx, phi sy) touches rows a0 .. a0 + W - 1, a0 = ceil(X - W/2),
// and columns b0 .. b0 + W - 1 (mod Nphi), b0 = ceil(Y - W/2).
//
// Tiles: the points are bucket-sorted by the tile of (a0, b0); a tile covers
// tile_x x tile_y stencil origins, so its points touch a (tile_x + W - 1) x
// (tile_y + W - 1) subgrid.  Inside a tile the points come in slots of two
// sharing their stencil origin (see k_tile_order); spreading gives a thread
// one slot, interpolation one entry.  One workgroup per tile stages that subgrid in
// LDS: interpolation reads it once from HBM; spreading accumulates into it
// (in double) with LDS atomics and flushes it with one global atomic per
// non-zero cell and component.
#include <cstdlib>

#include "nufft_index.h"
#include "psht_internal.h"

namespace psht {

constexpr int kTileThreads = 256;

struct NufftArgs {
    int W;
    double beta;
    int rows_used, Nphi, tile_x, tile_y, ntx, nty;
    int row_lo;
    const double *px, *py;
    const int32_t *perm;
    const int32_t *tile_start;
    const double *poly;    // kernel polynomial table of the inner taps (FP64 plans)
    const float *poly32;   // the same in float (FP32 plans)
    TileGeom geo;
    // points whose stencil left their tile (never expected: the plan verifies
    // the sort; counted, not silently skipped)
    unsigned long long *dropped;
    int xcd_group;  // tiles per XCD group (xcd_tile)
};

// Row stride (in elements) of a tile's subgrid in LDS: odd, so that the
// stencil origins (li, lj) of the slots a wave handles in one instruction
// fall in distinct LDS banks when their classes (li * stride + lj) mod 32
// are distinct, which is how k_tile_order lays the slots out.
__device__ __host__ inline int tile_row_stride(int tile_y, int W) { return (tile_y + W - 1) | 1; }
constexpr int kBankClasses = 32;

// e^x for x in [-40, 0]: x = n ln 2 + r with |r| <= ln(2)/2, the Taylor
// polynomial of degree 10 in r (truncation below 3e-13 relative), times 2^n.
// The kernel exponent beta (sqrt(1 - z^2) - 1) lies in [-beta, 0], beta <= 37.
__device__ inline double es_exp(double x) {
    const double n = rint(x * 1.4426950408889634);  // x / ln 2
    const double r = fma(-n, 0.69314718055994530942, x);
    double p = 1.0 / 3628800.0;  // 1 / 10!
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// ES kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, used for the
// two edge taps (at most about 2e-5 at W = 11, larger for small W, where the
// tolerance is correspondingly looser): the error of the exponential stays
// far below epsilon for every kernel width.
__device__ inline double es_kernel(double z, double beta) {
    double t = fmax(0.0, 1.0 - z * z);
    return es_exp(beta * (sqrt(t) - 1.0));
}
// FP32 form: the hardware square root and base-2 exponential (v_sqrt_f32,
// v_exp_f32, about one ulp each).  The exponent, at most beta log2(e) in
// magnitude, then carries an absolute error of a few ulp of that bound (about
// 3e-6 at W = 6, 1e-5 at W = 16), which is the relative error of the tap.  An
// edge tap weighs at most psi((W - 2)/W), 3 % of the peak at W = 6 and far less
// for wider kernels, so the sum moves by less than 1e-7 relative: below the
// rounding of the FP32 grid itself.
__device__ inline float es_kernel(float z, float beta) {
    const float t = fmaxf(0.0f, 1.0f - z * z);
    return __builtin_amdgcn_exp2f(beta * 1.44269504f * (__builtin_amdgcn_sqrtf(t) - 1.0f));
}

// Kernel weights of the W taps of a point with grid coordinate X and stencil
// origin a0: tap i has psi((X - a0 - i) 2 / W).  With v = 2 (X - a0) - (W - 1)
// in [-1, 1] (formed in double from the point's coordinate, then rounded to T),
// the inner taps 1..(W-1)/2 are polynomials in v of degree
// es_poly_degree(W, T is float) from the plan's table C (power-major) and tap
// W - 1 - i is the same polynomial at -v: even and odd parts by Horner in v^2
// give both.  The two edge taps use the formula.  T = float for the FP32 form
// (weights and their products in float), double otherwise.
// The table is wave-uniform: it is read through the scalar data cache into
// SGPRs (constant address space), so the FMAs take it as scalar operands and
// the LDS stays free for the tile subgrid.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using UniformPtr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ inline UniformPtr<T> uniform_ptr(const T *p) { return (UniformPtr<T>)p; }
#else
template <typename T> using UniformPtr = const T *;
template <typename T> __host__ __device__ inline UniformPtr<T> uniform_ptr(const T *p) { return p; }
#endif

// NS weight sets at once (the coordinates X[s] with origins a0[s] into k[s][]):
// each table coefficient is read once and used by the NS Horner chains, so only
// a few coefficients are live in SGPRs at a time (evaluating the sets one after
// another let the compiler hoist every coefficient and spill SGPRs into VGPR
// lanes, one v_readlane per use).
template <typename T, int W, int NS>
__device__ inline void es_weights_n(const double *X, const int *a0, T beta, UniformPtr<T> C, T (*k)[W]) {
    constexpr int P = es_poly_degree(W, sizeof(T) == 4), NC = (W - 1) / 2;
    constexpr int PE = (P % 2 == 0) ? P : P - 1, PO = (P % 2 == 1) ? P : P - 1;
    T v[NS], v2[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        v[s] = (T)(2.0 * (X[s] - (double)a0[s]) - (double)(W - 1));
        v2[s] = v[s] * v[s];
        k[s][0] = es_kernel((v[s] + (T)(W - 1)) * ((T)1 / (T)W), beta);
        k[s][W - 1] = es_kernel((v[s] - (T)(W - 1)) * ((T)1 / (T)W), beta);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T e[NS], o[NS];
        const T ce = C[PE * NC + c], co = C[PO * NC + c];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            e[s] = ce;
            o[s] = co;
        }
#pragma unroll
        for (int q = PE - 2; q >= 0; q -= 2) {
            const T cq = C[q * NC + c];
#pragma unroll
            for (int s = 0; s < NS; ++s) e[s] = fma(e[s], v2[s], cq);
        }
#pragma unroll
        for (int q = PO - 2; q >= 1; q -= 2) {
            const T cq = C[q * NC + c];
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s] = fma(o[s], v2[s], cq);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const T os = o[s] * v[s];
            k[s][c + 1] = e[s] + os;
            if (W - 2 - c != c + 1) k[s][W - 2 - c] = e[s] - os;
        }
    }
}

// Cell (i, j) = (e / SY, e mod SY) of the flat subgrid index e = threadIdx.x +
// k kTileThreads, advanced by one stride at a time: one division per thread
// instead of one per cell.
struct SubgridWalk {
    int i, j, di, dj;
    __device__ explicit SubgridWalk(int SY) {
        i = (int)threadIdx.x / SY;
        j = (int)threadIdx.x - i * SY;
        di = kTileThreads / SY;
        dj = kTileThreads - di * SY;
    }
    __device__ void next(int SY) {
        i += di;
        j += dj;
        if (j >= SY) {
            j -= SY;
            ++i;
        }
    }
};

// Column c0 + j of a tile's subgrid (c0 < Nphi, j < SY) reduced mod Nphi: the
// subgrid may wrap more than once when Nphi is small.
__device__ inline int wrap_subgrid_col(int c, int Nphi) {
    while (c >= Nphi) c -= Nphi;
    return c;
}

// Block -> tile map for the interpolation and spreading launches (grid of
// xcd_tile_blocks blocks).  Blocks are dealt round-robin to the eight XCDs,
// each with its own L2.  Groups of G consecutive tiles (adjacent in phi) go
// to one XCD and the groups rotate over the XCDs: neighbours inside a group
// share an L2 (their overlapping subgrid halos and the map's cache lines that
// straddle two tiles), while the rotation keeps the XCDs' loads even.  G = 1
// is the plain round-robin.  Returns -1 past the end.
__device__ inline int xcd_tile(int bid, int ntiles, int G) {
    const int x = bid & 7, k = bid >> 3;
    const int q = k / G;
    const int t = (q * 8 + x) * G + (k - q * G);
    return t < ntiles ? t : -1;
}
__host__ inline unsigned xcd_tile_blocks(int ntiles, int G) {
    return 8u * (unsigned)G * (unsigned)((ntiles + 8 * G - 1) / (8 * G));
}
// Tiles per group: the largest power of two up to 64 that leaves at least 64
// groups per XCD (small plans keep the plain round-robin).  lmax 4096, FP32:
// interpolation 0.313 -> 0.299 ms at G = 64, spreading within 2 %.
// PSHT_XCD_GROUP fixes it for tuning runs.
static int xcd_group(int ntiles) {
    static const int forced = [] {
        const char *e = getenv("PSHT_XCD_GROUP");
        const int v = e ? atoi(e) : 0;
        return v >= 1 && v <= 4096 ? v : 0;
    }();
    if (forced) return forced;
    int G = 1;
    while (G < 64 && (int64_t)ntiles >= (int64_t)2 * G * 8 * 64) G *= 2;
    return G;
}

template <typename T> __device__ inline const T *table(const NufftArgs &a);
template <> __device__ inline const double *table<double>(const NufftArgs &a) { return a.poly; }
template <> __device__ inline const float *table<float>(const NufftArgs &a) { return a.poly32; }

template <typename T> struct CplxT;
template <> struct CplxT<double> { typedef double2 type; };
template <> struct CplxT<float> { typedef float2 type; };

// Tile index -> (tx, ty); tiles with no points return immediately.
template <typename T, int W>
__global__ __launch_bounds__(kTileThreads) void k_interp(NufftArgs a, const typename CplxT<T>::type *U,
                                                         typename CplxT<T>::type *map) {
    typedef typename CplxT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *S = reinterpret_cast<C *>(smem);
    const UniformPtr<T> sC = uniform_ptr(table<T>(a));
    const int t = xcd_tile(blockIdx.x, a.ntx * a.nty, a.xcd_group);
    if (t < 0) return;
    const int p0 = a.tile_start[t], p1 = a.tile_start[t + 1];
    if (p0 == p1) return;
    const int tx = t / a.nty, ty = t - tx * a.nty;
    const int SX = a.tile_x + W - 1, SY = a.tile_y + W - 1, SYP = tile_row_stride(a.tile_y, W);
    const int r0 = tx * a.tile_x, c0 = ty * a.tile_y;
    {
        SubgridWalk w(SY);
        for (int e = threadIdx.x; e < SX * SY; e += kTileThreads, w.next(SY)) {
            const int row = r0 + w.i;
            C v;
            v.x = v.y = (T)0;
            if (row < a.rows_used) v = U[(int64_t)row * a.Nphi + wrap_subgrid_col(c0 + w.j, a.Nphi)];
            S[w.i * SYP + w.j] = v;
        }
    }
    __syncthreads();
    // one entry per thread; the two entries of a slot (same cell) sit in
    // neighbouring lanes, whose identical LDS reads are broadcasts
    for (int p = p0 + threadIdx.x; p < p1; p += kTileThreads) {
        const int pm = a.perm[p];
        if (pm < 0) continue;  // dummy entry of an odd cell
        const double X = a.px[p], Y = a.py[p];
        const int a0 = stencil_origin(X, W), b0 = stencil_origin(Y, W);
        int li, lj;
        tile_local(a.geo, X, Y, t, li, lj);
        // The plan verified 0 <= li < tile_x, 0 <= lj < tile_y for every entry;
        // the guard keeps LDS accesses in bounds and counts what it skips.
        if (!in_tile(a.geo, li, lj)) {
            atomicAdd(a.dropped, 1ull);
            continue;
        }
        // weights and sums in T: FP32 for the FP32 form
        T kw[2][W];
        {
            const double xs[2] = {X, Y};
            const int os[2] = {a0, b0};
            es_weights_n<T, W, 2>(xs, os, (T)a.beta, sC, kw);
        }
        const T *kx = kw[0], *ky = kw[1];
        T accr = 0, acci = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const C *Srow = S + (li + i) * SYP + lj;
            T rr = 0, ri = 0;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                C v = Srow[j];
                rr = fma(ky[j], v.x, rr);
                ri = fma(ky[j], v.y, ri);
            }
            accr = fma(kx[i], rr, accr);
            acci = fma(kx[i], ri, acci);
        }
        C out;
        out.x = accr;
        out.y = acci;
        map[pm] = out;
    }
}

template <typename T, int W>
__global__ __launch_bounds__(kTileThreads) void k_spread(NufftArgs a, const typename CplxT<T>::type *map,
                                                         T *U) {
    typedef typename CplxT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = xcd_tile(blockIdx.x, a.ntx * a.nty, a.xcd_group);
    if (t < 0) return;
    const int p0 = a.tile_start[t], p1 = a.tile_start[t + 1];
    if (p0 == p1) return;
    const int tx = t / a.nty, ty = t - tx * a.nty;
    const int SX = a.tile_x + W - 1, SY = a.tile_y + W - 1;
    const int SYP = tile_row_stride(a.tile_y, W);
    // Separate real and imaginary planes, accumulated in double for both map
    // precisions: the FP64 LDS atomic add is a native fast path on gfx950,
    // while FP32 LDS atomic adds measured an order of magnitude slower.
    double *Sre = reinterpret_cast<double *>(smem), *Sim = Sre + SX * SYP;
    const UniformPtr<T> sC = uniform_ptr(table<T>(a));
    const int r0 = tx * a.tile_x, c0 = ty * a.tile_y;
    for (int e = threadIdx.x; e < 2 * SX * SYP; e += kTileThreads) Sre[e] = 0.0;
    __syncthreads();
    // one slot per thread: both points share the stencil cells, so their
    // contributions are summed in registers and each cell gets one LDS update
    for (int q = (p0 >> 1) + threadIdx.x; q < (p1 >> 1); q += kTileThreads) {
        const int p = 2 * q;
        const double X = a.px[p], Y = a.py[p], X2 = a.px[p + 1], Y2 = a.py[p + 1];
        const int a0 = stencil_origin(X, W), b0 = stencil_origin(Y, W);
        int li, lj;
        tile_local(a.geo, X, Y, t, li, lj);
        if (!in_tile(a.geo, li, lj)) {
            atomicAdd(a.dropped, (a.perm[p + 1] >= 0) ? 2ull : 1ull);
            continue;
        }
        // weights and the slot's per-cell sums in T (FP32 for the FP32 form);
        // the subgrid accumulates in double
        T kw[4][W];
        {
            // the partner has the same cell, but its own unwrapped origin: across
            // phi = 0 its b0 differs from this point's by Nphi
            const double xs[4] = {X, Y, X2, Y2};
            const int os[4] = {a0, b0, stencil_origin(X2, W), stencil_origin(Y2, W)};
            es_weights_n<T, W, 4>(xs, os, (T)a.beta, sC, kw);
        }
        const T *kx = kw[0], *ky = kw[1], *kx2 = kw[2], *ky2 = kw[3];
        const C f = map[a.perm[p]];
        const int pm2 = a.perm[p + 1];
        C f2;
        f2.x = f2.y = (T)0;
        if (pm2 >= 0) f2 = map[pm2];
        const T fr = f.x, fi = f.y, fr2 = f2.x, fi2 = f2.y;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            double *Rre = Sre + (li + i) * SYP + lj, *Rim = Sim + (li + i) * SYP + lj;
            const T wr = kx[i] * fr, wi = kx[i] * fi, wr2 = kx2[i] * fr2, wi2 = kx2[i] * fi2;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                atomicAdd(Rre + j, (double)fma(wr, ky[j], wr2 * ky2[j]));
                atomicAdd(Rim + j, (double)fma(wi, ky[j], wi2 * ky2[j]));
            }
        }
    }
    __syncthreads();
    SubgridWalk w(SY);
    for (int e = threadIdx.x; e < SX * SY; e += kTileThreads, w.next(SY)) {
        const int row = r0 + w.i;
        if (row >= a.rows_used) continue;
        const T vr = (T)Sre[w.i * SYP + w.j], vi = (T)Sim[w.i * SYP + w.j];
        if (vr == (T)0 && vi == (T)0) continue;
        T *dst = U + 2 * ((int64_t)row * a.Nphi + wrap_subgrid_col(c0 + w.j, a.Nphi));
        atomicAdd(dst, vr);
        atomicAdd(dst + 1, vi);
    }
}

static NufftArgs nufft_args(const psht_plan_s &p) {
    NufftArgs a;
    a.W = p.g.W;
    a.beta = p.g.beta;
    a.rows_used = p.g.rows_used;
    a.Nphi = p.g.Nphi;
    a.tile_x = p.tile_x;
    a.tile_y = p.tile_y;
    a.ntx = p.ntx;
    a.nty = p.nty;
    a.row_lo = p.g.row_lo;
    a.px = p.d_px;
    a.py = p.d_py;
    a.perm = p.d_perm;
    a.tile_start = p.d_tile_start;
    a.poly = p.d_es_poly;
    a.poly32 = p.d_es_poly32;
    a.geo = tile_geom(p);
    a.dropped = p.d_dropped;
    a.xcd_group = xcd_group(p.ntiles);
    return a;
}

template <typename T, int W>
static hipError_t launch_interp_w(const psht_plan_s &p, const void *U, void *map, hipStream_t st) {
    typedef typename CplxT<T>::type C;
    NufftArgs a = nufft_args(p);
    size_t lds = (size_t)(p.tile_x + W - 1) * tile_row_stride(p.tile_y, W) * sizeof(C);
    hipLaunchKernelGGL((k_interp<T, W>), dim3(xcd_tile_blocks(p.ntiles, a.xcd_group)), dim3(kTileThreads), lds, st, a,
                       static_cast<const C *>(U), static_cast<C *>(map));
    return hipGetLastError();
}

template <typename T, int W>
static hipError_t launch_spread_w(const psht_plan_s &p, const void *map, void *U, hipStream_t st) {
    typedef typename CplxT<T>::type C;
    NufftArgs a = nufft_args(p);
    size_t lds = (size_t)(p.tile_x + W - 1) * tile_row_stride(p.tile_y, W) * 2 * sizeof(double);
    hipLaunchKernelGGL((k_spread<T, W>), dim3(xcd_tile_blocks(p.ntiles, a.xcd_group)), dim3(kTileThreads), lds, st, a,
                       static_cast<const C *>(map), static_cast<T *>(U));
    return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_interp(const psht_plan_s &p, const void *U, void *map, hipStream_t st) {
    switch (p.g.W) {
#define PSHT_W(w) case w: return launch_interp_w<T, w>(p, U, map, st);
        PSHT_W(2) PSHT_W(3) PSHT_W(4) PSHT_W(5) PSHT_W(6) PSHT_W(7) PSHT_W(8) PSHT_W(9)
        PSHT_W(10) PSHT_W(11) PSHT_W(12) PSHT_W(13) PSHT_W(14) PSHT_W(15) PSHT_W(16)
#undef PSHT_W
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t dispatch_spread(const psht_plan_s &p, const void *map, void *U, hipStream_t st) {
    switch (p.g.W) {
#define PSHT_W(w) case w: return launch_spread_w<T, w>(p, map, U, st);
        PSHT_W(2) PSHT_W(3) PSHT_W(4) PSHT_W(5) PSHT_W(6) PSHT_W(7) PSHT_W(8) PSHT_W(9)
        PSHT_W(10) PSHT_W(11) PSHT_W(12) PSHT_W(13) PSHT_W(14) PSHT_W(15) PSHT_W(16)
#undef PSHT_W
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp(const psht_plan_s &p, const void *U, void *map, hipStream_t st) {
    if (p.npts == 0 || p.ntiles == 0) return hipSuccess;
    return p.g.fp32 ? dispatch_interp<float>(p, U, map, st) : dispatch_interp<double>(p, U, map, st);
}

hipError_t launch_spread(const psht_plan_s &p, const void *map, void *U, hipStream_t st) {
    if (p.npts == 0 || p.ntiles == 0) return hipSuccess;
    return p.g.fp32 ? dispatch_spread<float>(p, map, U, st) : dispatch_spread<double>(p, map, U, st);
}

// --------------------------------------------------------------- fill

__global__ void k_fill_zero(uint4 *p, size_t n16) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_fill_zero_bytes(unsigned char *p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    size_t n16 = bytes / 16;
    if (n16) {
        size_t blocks = std::min<size_t>((n16 + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<uint4 *>(ptr), n16);
    }
    size_t rem = bytes - n16 * 16;
    if (rem)
        hipLaunchKernelGGL(k_fill_zero_bytes, dim3(1), dim3(256), 0, st, static_cast<unsigned char *>(ptr) + n16 * 16,
                           rem);
    return hipGetLastError();
}

// ------------------------------------------------------ plan-time points

// Per-block partial statistics: [min theta, max theta, number of invalid points].
constexpr int kStatBlocks = 1024;

__global__ __launch_bounds__(256) void k_point_stats(const double *theta, const double *phi, int64_t n,
                                                     double *out) {
    __shared__ double smin[256], smax[256], sbad[256];
    double mn = 1e300, mx = -1e300, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double t = theta[i], f = phi[i];
        const bool ok = (t >= 0.0) && (t <= M_PI) && isfinite(f);
        if (!ok) bad += 1;
        else {
            mn = fmin(mn, t);
            mx = fmax(mx, t);
        }
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = smin[0];
        out[3 * blockIdx.x + 1] = smax[0];
        out[3 * blockIdx.x + 2] = sbad[0];
    }
}

hipError_t launch_point_stats(const double *theta, const double *phi, int64_t n, double *d_stats, hipStream_t st) {
    hipLaunchKernelGGL(k_point_stats, dim3(kStatBlocks), dim3(256), 0, st, theta, phi, n, d_stats);
    return hipGetLastError();
}

typedef TileGeom SortArgs;

__global__ void k_point_keys(SortArgs a, const double *theta, const double *phi, int64_t n, int32_t *keys,
                             int32_t *count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double X, Y;
    point_grid(a, theta[i], phi[i], X, Y);
    int k = point_tile(a, X, Y);
    keys[i] = k;
    atomicAdd(&count[k], 1);
}

// Exclusive scan of count[0..n) into start[0..n] (start[n] = total), one block.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *count, int n, int32_t *start, int32_t *cursor) {
    __shared__ int32_t part[1024];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(n, b + per);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int i = b; i < e; ++i) {
        const int32_t c = count[i];  // count and cursor may alias
        start[i] = run;
        cursor[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) start[n] = part[1023];
}

__global__ void k_point_scatter(SortArgs a, const double *theta, const double *phi, int64_t n, const int32_t *keys,
                                int32_t *cursor, double *px, double *py, int32_t *perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double X, Y;
    point_grid(a, theta[i], phi[i], X, Y);
    int pos = atomicAdd(&cursor[keys[i]], 1);
    px[pos] = X;
    py[pos] = Y;
    perm[pos] = (int32_t)i;
}

// Order inside a tile.  The points of a tile are laid out in slots of two
// entries: the two points of a slot share their stencil-origin cell (the
// second entry is a dummy with perm = -1 when a cell has an odd count), so a
// thread spreading a slot adds both points' contributions in registers before
// each LDS update, and a thread interpolating a slot reads every subgrid value
// once for both.  A cell (li, lj) has the bank class (li * stride + lj) mod 32
// of its subgrid address (tile_row_stride).  Within a class the slots are
// numbered cell by cell in row-major order (class rank), and the tile's slots
// are laid out by class rank, then class: while all classes still have slots,
// every 32 consecutive slots cover the 32 classes once, so the W x W stencils
// that consecutive lanes update in one instruction fall in distinct LDS banks.
constexpr int kOrderThreads = 256;

// Cell of a point inside tile t (clamped; k_tile_verify checks that no clamp
// is ever needed).
__device__ inline int cell_in_tile(const SortArgs &a, double X, double Y, int t) {
    int li, lj;
    tile_local(a, X, Y, t, li, lj);
    li = min(max(li, 0), a.tile_x - 1);
    lj = min(max(lj, 0), a.tile_y - 1);
    return li * a.tile_y + lj;
}

// Entries whose stencil origin lies outside their tile (plan-time check of the sort).
__global__ void k_tile_verify(SortArgs a, const int32_t *tile_start, int ntiles, const double *px, const double *py,
                              const int32_t *perm, unsigned long long *bad) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const int p0 = tile_start[t], p1 = tile_start[t + 1];
    unsigned long long nbad = 0;
    for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        int li, lj;
        tile_local(a, px[p], py[p], t, li, lj);
        if (perm[p] >= 0 && !in_tile(a, li, lj)) ++nbad;
    }
    if (nbad) atomicAdd(bad, nbad);
}

// Entries (2 per slot) of every tile: sum over cells of 2 ceil(count / 2).
__global__ __launch_bounds__(kOrderThreads) void k_tile_entries(SortArgs a, const int32_t *pstart,
                                                                const double *tpx, const double *tpy,
                                                                int32_t *entries) {
    extern __shared__ int32_t osm[];
    const int C = a.tile_x * a.tile_y;
    int32_t *cnt = osm;
    __shared__ int32_t s_tot;
    const int t = blockIdx.x;
    const int p0 = pstart[t], p1 = pstart[t + 1];
    if (p0 == p1) {
        if (threadIdx.x == 0) entries[t] = 0;
        return;
    }
    for (int c = threadIdx.x; c < C; c += kOrderThreads) cnt[c] = 0;
    if (threadIdx.x == 0) s_tot = 0;
    __syncthreads();
    for (int p = p0 + threadIdx.x; p < p1; p += kOrderThreads)
        atomicAdd(&cnt[cell_in_tile(a, tpx[p], tpy[p], t)], 1);
    __syncthreads();
    int loc = 0;
    for (int c = threadIdx.x; c < C; c += kOrderThreads) loc += 2 * ((cnt[c] + 1) / 2);
    atomicAdd(&s_tot, loc);
    __syncthreads();
    if (threadIdx.x == 0) entries[t] = s_tot;
}

// One workgroup per tile: writes the tile's slots from (tpx, tpy, tperm)
// (points [pstart[t], pstart[t+1]) in arbitrary order) to entries
// [estart[t], estart[t+1]) of (px, py, perm).  rank[] is per-point scratch.
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(SortArgs a, const int32_t *pstart,
                                                              const int32_t *estart, const double *tpx,
                                                              const double *tpy, const int32_t *tperm,
                                                              int32_t *rank, double *px, double *py, int32_t *perm) {
    extern __shared__ int32_t osm[];
    const int C = a.tile_x * a.tile_y;
    int32_t *cnt = osm, *first = osm + C;  // points per cell; class rank of the cell's first slot
    __shared__ int32_t nk[kBankClasses];   // slots per class
    const int t = blockIdx.x;
    const int p0 = pstart[t], p1 = pstart[t + 1];
    if (p0 == p1) return;
    const int e0 = estart[t];
    const int stride = tile_row_stride(a.tile_y, a.W);
    for (int c = threadIdx.x; c < C; c += kOrderThreads) cnt[c] = 0;
    __syncthreads();
    for (int p = p0 + threadIdx.x; p < p1; p += kOrderThreads)
        rank[p] = atomicAdd(&cnt[cell_in_tile(a, tpx[p], tpy[p], t)], 1);
    __syncthreads();
    // one thread per class walks its cells in row-major order
    if (threadIdx.x < kBankClasses) {
        const int k = threadIdx.x;
        int run = 0;
        for (int li = 0; li < a.tile_x; ++li) {
            const int lj0 = ((k - li * stride) % kBankClasses + kBankClasses) % kBankClasses;
            for (int lj = lj0; lj < a.tile_y; lj += kBankClasses) {
                const int c = li * a.tile_y + lj;
                first[c] = run;
                run += (cnt[c] + 1) / 2;
            }
        }
        nk[k] = run;
    }
    __syncthreads();
    for (int p = p0 + threadIdx.x; p < p1; p += kOrderThreads) {
        const int r = rank[p];
        const int cell = cell_in_tile(a, tpx[p], tpy[p], t);
        const int li = cell / a.tile_y, lj = cell - li * a.tile_y;
        const int k = (li * stride + lj) % kBankClasses;
        const int R = first[cell] + r / 2;  // class rank of the point's slot
        // slots before (R, k): every slot of class rank < R, and those of rank R in classes < k
        int slot = 0;
#pragma unroll 8
        for (int k2 = 0; k2 < kBankClasses; ++k2) {
            const int n2 = nk[k2];
            slot += min(n2, R) + ((k2 < k && n2 > R) ? 1 : 0);
        }
        const int dst = e0 + 2 * slot + (r & 1);
        px[dst] = tpx[p];
        py[dst] = tpy[p];
        perm[dst] = tperm[p];
        if (r == cnt[cell] - 1 && !(r & 1)) {  // odd cell: the slot's second entry is a dummy
            px[dst + 1] = tpx[p];
            py[dst + 1] = tpy[p];
            perm[dst + 1] = -1;
        }
    }
}

size_t tile_order_lds_bytes(int tile_x, int tile_y) { return sizeof(int32_t) * 2 * (size_t)tile_x * tile_y; }

TileGeom tile_geom(const psht_plan_s &p) {
    TileGeom a;
    a.sx = p.g.sx;
    a.sy = p.g.sy;
    a.W = p.g.W;
    a.row_lo = p.g.row_lo;
    a.rows_used = p.g.rows_used;
    a.Nphi = p.g.Nphi;
    a.tile_x = p.tile_x;
    a.tile_y = p.tile_y;
    a.ntx = p.ntx;
    a.nty = p.nty;
    return a;
}

hipError_t launch_point_sort_count(psht_plan_s &p, const double *theta, const double *phi, int32_t *d_keys,
                                   int32_t *d_cursor, int32_t *d_pstart, double *tpx, double *tpy, int32_t *tperm,
                                   hipStream_t st) {
    const SortArgs a = tile_geom(p);
    const int64_t n = p.npts;
    hipError_t e = launch_fill_zero(d_cursor, sizeof(int32_t) * (size_t)p.ntiles, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        unsigned nb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_point_keys, dim3(nb), dim3(256), 0, st, a, theta, phi, n, d_keys, d_cursor);
    }
    // d_cursor now holds the counts; scan into pstart and reuse d_cursor as the cursor
    // (the scan reads each count before it overwrites it within the same thread).
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d_cursor, p.ntiles, d_pstart, d_cursor);
    if (n > 0) {
        unsigned nb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_point_scatter, dim3(nb), dim3(256), 0, st, a, theta, phi, n, d_keys, d_cursor, tpx, tpy,
                           tperm);
    }
    // entries per tile (the cursor array is free again), scanned into the plan's tile_start
    hipLaunchKernelGGL(k_tile_entries, dim3((unsigned)p.ntiles), dim3(kOrderThreads),
                       sizeof(int32_t) * (size_t)p.tile_x * p.tile_y, st, a, d_pstart, tpx, tpy, d_cursor);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, d_cursor, p.ntiles, p.d_tile_start, d_cursor);
    return hipGetLastError();
}

hipError_t launch_point_sort_order(psht_plan_s &p, int32_t *d_keys, const int32_t *d_pstart, const double *tpx,
                                   const double *tpy, const int32_t *tperm, unsigned long long *d_bad,
                                   hipStream_t st) {
    if (p.npts == 0) return hipSuccess;
    const SortArgs a = tile_geom(p);
    // keys are no longer needed: they hold the per-point ranks from here on
    hipLaunchKernelGGL(k_tile_order, dim3((unsigned)p.ntiles), dim3(kOrderThreads),
                       tile_order_lds_bytes(p.tile_x, p.tile_y), st, a, d_pstart, p.d_tile_start, tpx, tpy, tperm,
                       d_keys, p.d_px, p.d_py, p.d_perm);
    hipLaunchKernelGGL(k_tile_verify, dim3((unsigned)p.ntiles), dim3(256), 0, st, a, p.d_tile_start, p.ntiles, p.d_px,
                       p.d_py, p.d_perm, d_bad);
    return hipGetLastError();
}

}  // namespace psht
