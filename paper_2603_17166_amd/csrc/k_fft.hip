// Batched FFTs of the Fourier-sphere route and the two uniform stages built
// on them (gfx950).
//
// Theta stage (synthesis), one workgroup per order m:
//   the rings theta_j = Theta_j theta_max / pi, Theta_j = 2 pi j / N2, are
//   completed to the doubled circle with the mirror rule of Sec. I.A (eq. sht):
//   on the doubled sphere F_m(-Theta) = (-1)^(s+m) F_m(Theta); the window w
//   of Sec. II.C is applied, the N2-point DFT gives the Fourier coefficients
//   of the band-limited approximation (the Dirichlet kernel D of eq. Dnz),
//   which are divided by the NUFFT kernel transform, zero-padded to the
//   oversampled grid and transformed back; only the grid rows the points
//   touch are kept.
// Phi stage (synthesis), one workgroup per kept row: divide by the phi kernel
//   transform, zero-pad to the oversampled length, inverse FFT.
// The adjoint stages are the exact transposes.
//
// The FFT is a mixed-radix (4, 2, 3, 5, 7, 11, 13) Stockham transform held in
// LDS: each pass stages its butterfly inputs in registers, synchronises, and
// writes the outputs in place, so one buffer of n complex values suffices.
#include <type_traits>

#include "psht_internal.h"

namespace psht {

template <typename T> struct CT;
template <> struct CT<double> { typedef double2 type; };
template <> struct CT<float> { typedef float2 type; };

template <typename C> __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ inline C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C, typename S> __device__ inline C cscale(C a, S s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }

// A transform's factorization as kernel arguments: the radix of pass p in bits
// 4p .. 4p + 3 of `code` (radices up to 13, at most 16 passes for n <= 8192),
// so it occupies two scalar registers instead of an array.
struct FftDev {
    int n, npass;
    unsigned long long code;
};

static FftDev to_dev(const FftFactors &f) {
    FftDev d;
    d.n = f.n;
    d.npass = f.npass;
    d.code = 0;
    for (int i = 0; i < f.npass && i < 16; ++i) d.code |= (unsigned long long)(f.radix[i] & 15) << (4 * i);
    return d;
}


// e^{sign 2 pi i t / n} from the table tw[k] = e^{-2 pi i k / n}.
template <typename C> __device__ inline C twiddle(const double2 *tw, int k, int sign) {
    double2 w = tw[k];
    C r;
    r.x = w.x;
    r.y = -sign * w.y;
    return r;
}

// cos and sin of 2 pi k / R for the odd radices.
template <int R> struct Rot;
template <> struct Rot<3> {
    static constexpr double c[3] = {1, -0.49999999999999978, -0.50000000000000044};
    static constexpr double s[3] = {0, 0.86602540378443871, -0.86602540378443837};
};
template <> struct Rot<5> {
    static constexpr double c[5] = {1, 0.30901699437494745, -0.80901699437494734, -0.80901699437494756, 0.30901699437494723};
    static constexpr double s[5] = {0, 0.95105651629515353, 0.58778525229247325, -0.58778525229247303, -0.95105651629515364};
};
template <> struct Rot<7> {
    static constexpr double c[7] = {1, 0.62348980185873359, -0.22252093395631434, -0.90096886790241903, -0.90096886790241915, -0.22252093395631459, 0.62348980185873337};
    static constexpr double s[7] = {0, 0.7818314824680298, 0.97492791218182362, 0.43388373911755823, -0.43388373911755801, -0.97492791218182362, -0.78183148246802991};
};
template <> struct Rot<11> {
    static constexpr double c[11] = {1, 0.84125353283118121, 0.41541501300188644, -0.142314838273285, -0.65486073394528499, -0.95949297361449737, -0.95949297361449748, -0.65486073394528521, -0.14231483827328523, 0.41541501300188605, 0.84125353283118121};
    static constexpr double s[11] = {0, 0.54064081745559756, 0.90963199535451833, 0.9898214418809328, 0.75574957435425827, 0.28173255684142967, -0.28173255684142939, -0.75574957435425816, -0.98982144188093268, -0.90963199535451855, -0.54064081745559744};
};
template <> struct Rot<13> {
    static constexpr double c[13] = {1, 0.88545602565320991, 0.56806474673115592, 0.12053668025532301, -0.35460488704253545, -0.74851074817110119, -0.97094181742605201, -0.97094181742605212, -0.7485107481711013, -0.3546048870425359, 0.1205366802553232, 0.56806474673115481, 0.88545602565321002};
    static constexpr double s[13] = {0, 0.46472317204376851, 0.82298386589365635, 0.99270887409805397, 0.93501624268541483, 0.66312265824079519, 0.23931566428755768, -0.23931566428755743, -0.66312265824079497, -0.93501624268541472, -0.99270887409805397, -0.82298386589365702, -0.4647231720437684};
};

// Radix-R DFT in registers: y_q = sum_r v_r e^{sign 2 pi i r q / R}.  Odd R
// uses the symmetric form: with t_r = v_r + v_{R-r} and u_r = v_r - v_{R-r},
// y_q = a_q + sign i b_q and y_{R-q} = a_q - sign i b_q, where
// a_q = v_0 + sum_r t_r cos(2 pi r q / R), b_q = sum_r u_r sin(2 pi r q / R),
// r, q = 1..(R-1)/2, with compile-time constants.
template <typename C, int R> __device__ inline void dft(C *v, int sign) {
    if constexpr (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        C a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d0 = csub(v[1], v[3]);
        C d;  // (sign i) * d0
        d.x = -sign * d0.y;
        d.y = sign * d0.x;
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    } else {
        typedef decltype(v[0].x) S;
        constexpr int H = (R - 1) / 2;
        C t[H + 1], u[H + 1];
        C y0 = v[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            t[r] = cadd(v[r], v[R - r]);
            u[r] = csub(v[r], v[R - r]);
            y0 = cadd(y0, t[r]);
        }
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            C a = v[0], b;
            b.x = b.y = (S)0;
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const S cr = (S)Rot<R>::c[(r * q) % R], sr = (S)Rot<R>::s[(r * q) % R];
                a.x += t[r].x * cr;
                a.y += t[r].y * cr;
                b.x += u[r].x * sr;
                b.y += u[r].y * sr;
            }
            // sign i b = (-sign b.y, sign b.x)
            v[q].x = a.x - sign * b.y;
            v[q].y = a.y + sign * b.x;
            v[R - q].x = a.x + sign * b.y;
            v[R - q].y = a.y - sign * b.x;
        }
        v[0] = y0;
    }
}

// Threads of a workgroup transforming up to MAXN points.  The passes are
// bound by latency (LDS round trips and barriers), so what counts is the
// number of transforms in flight per CU: up to 2560 points (40 KB of FP64
// data) four workgroups of 256 threads fit a CU, where two of 512 did.  The
// longest tier holds up to 128 KB of LDS, one workgroup per CU: 1024 threads
// give each SIMD four waves.
template <typename T> __host__ __device__ constexpr int fft_threads(int maxn) {
    // (the 10240-point tier fills the 160 KB of LDS a gfx950 workgroup may use)
    if constexpr (sizeof(T) == 8) return maxn <= 2560 ? 256 : (maxn <= 4096 ? 512 : (maxn <= 8192 ? 1024 : 512));
    // FP32 data takes half the LDS per transform: the longest tier (64 KB) fits
    // two workgroups of 512 threads per CU (FP32 phi halves at lmax 4096:
    // 0.15 -> 0.13 ms each way); 256 threads up to 4096 points made the Theta
    // stage slower.
    return maxn <= 2560 ? 256 : 512;
}

// One Stockham pass of radix R on buf[0..n) with stride Ns.  Every thread
// holds NB butterflies in registers; NB follows from the largest transform
// length MAXN the kernel is built for, so short transforms do not pay the
// registers of long ones.
template <typename T, int R, int MAXN>
__device__ void fft_pass(typename CT<T>::type *buf, int n, int Ns, int sign, const double2 *tw) {
    typedef typename CT<T>::type C;
    constexpr int NT = fft_threads<T>(MAXN);
    constexpr int NB = (MAXN / R + NT - 1) / NT;
    const int nb = n / R;
    const int tws = n / (Ns * R);
    C v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int b = threadIdx.x + i * NT;
        if (b < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[b + r * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int b = threadIdx.x + i * NT;
        if (b < nb) {
            int k = b % Ns;
            // twiddles w^r (r = 1..R-1) as powers of the one table entry w:
            // one load per butterfly instead of R - 1 scattered ones
            const C w1 = twiddle<C>(tw, k * tws, sign);
            C wr = w1;
            v[i][1] = cmul(v[i][1], w1);
#pragma unroll
            for (int r = 2; r < R; ++r) {
                wr = cmul(wr, w1);
                v[i][r] = cmul(v[i][r], wr);
            }
            dft<C, R>(v[i], sign);
            int d = (b - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[d + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// In-place FFT of buf[0..n) in LDS, n <= MAXN; the caller synchronises before the call.
template <typename T, int MAXN>
__device__ void lds_fft(typename CT<T>::type *buf, const FftDev &f, int sign, const double2 *tw) {
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
        const int R = (int)((f.code >> (4 * p)) & 15);
        switch (R) {
            case 4: fft_pass<T, 4, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 2: fft_pass<T, 2, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 3: fft_pass<T, 3, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 5: fft_pass<T, 5, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 7: fft_pass<T, 7, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 11: fft_pass<T, 11, MAXN>(buf, f.n, Ns, sign, tw); break;
            case 13: fft_pass<T, 13, MAXN>(buf, f.n, Ns, sign, tw); break;
            default: break;
        }
        Ns *= R;
    }
}

// ------------------------------------------------------------ plain rows

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_fft_rows(FftDev f, int sign, const double2 *tw,
                                                          const typename CT<T>::type *in,
                                                          typename CT<T>::type *out) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int64_t row = blockIdx.x;
    for (int k = threadIdx.x; k < f.n; k += fft_threads<T>(MAXN)) buf[k] = in[row * f.n + k];
    __syncthreads();
    lds_fft<T, MAXN>(buf, f, sign, tw);
    for (int k = threadIdx.x; k < f.n; k += fft_threads<T>(MAXN)) out[row * f.n + k] = buf[k];
}

// ------------------------------------------------------------ Theta stage

struct StageArgs {
    FftDev fn2, fnt, fnp;
    const double2 *tw_n2, *tw_nt, *tw_np, *tw_np_full;
    int L, N2, NT, Nphi, nring, mmax, spin, row_lo, rows_used;
    int parts;    // phi FFT as this many transforms of length Nphi / parts (1, 2 or 4)
    bool tsplit;  // Theta grid transform (NT = 2 N2 points) as two N2-point transforms (even / odd rows)
    const double *ring_w;
    const int32_t *ring_mmax;
    const double *psihat_t, *psihat_p;
};

// Column of the Theta stage handled by block b.  Blocks are dealt to the 8
// XCDs round-robin; this map gives each XCD one contiguous range of columns,
// walked in order, so the workgroups resident on an XCD at any time touch
// neighbouring columns of the row-major V array and share its cache lines in
// that XCD's L2 (one column alone would use 16 of every 128 bytes it moves).
// The grid has 8 * ceil(ncol / 8) blocks; blocks past the end return.
__device__ inline int xcd_column(int b, int ncol) {
    const int per = (ncol + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

static inline unsigned xcd_grid(int ncol) { return 8u * (unsigned)((ncol + 7) / 8); }

// The Theta-grid transform of length NT = 2 N2 as two N2-point transforms:
// with the spectrum X_n, |n| <= L < N2 / 2, held at n mod N2, the grid rows
// k = 2 k' + h are sum_n (X_n e^{2 pi i n h / NT}) e^{2 pi i n k' / N2}; the
// adjoint's spectrum is sum_h e^{-2 pi i n h / NT} FFT_N2(rows 2 k' + h)[n].
// Each thread keeps its entries i = tid + q NTHR of the spectrum in
// registers between the two halves.
template <typename T, int MAXN> struct ThetaHalves {
    static constexpr int NTHR = fft_threads<T>(MAXN);
    static constexpr int NQ = (MAXN + NTHR - 1) / NTHR;
};

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_theta_synth(StageArgs a, const double2 *F,
                                                             typename CT<T>::type *V) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int mi = xcd_column(blockIdx.x, 2 * a.mmax + 1);
    if (mi > 2 * a.mmax) return;
    const int am = abs(mi - a.mmax);
    const double sig = ((a.spin + am) & 1) ? -1.0 : 1.0;  // mirror sign (-1)^(s+m)
    const int L = a.L, N2 = a.N2, NT = a.NT;
    const double2 *Fm = F + (int64_t)mi * a.nring;
    for (int k = threadIdx.x; k < N2; k += fft_threads<T>(MAXN)) {
        const int j = k <= L ? k : N2 - k;
        const double wj = (k <= L ? 1.0 : sig) * a.ring_w[j];
        double2 v = make_double2(0.0, 0.0);
        if (a.ring_mmax[j] >= am) v = Fm[j];
        C c;
        c.x = (T)(v.x * wj);
        c.y = (T)(v.y * wj);
        buf[k] = c;
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fn2, -1, a.tw_n2);  // N2 * Fourier coefficient
    const int64_t ldv = 2 * a.mmax + 1;
    // divide by N2 psihat(|n|) and pad to NT: n < 0 moves from N2 - |n| to NT - |n|
    for (int n = 1 + threadIdx.x; n <= L; n += fft_threads<T>(MAXN))
        buf[NT - n] = cscale(buf[N2 - n], (T)(1.0 / (N2 * a.psihat_t[n])));
    __syncthreads();
    for (int k = threadIdx.x; k < NT - L; k += fft_threads<T>(MAXN)) {
        if (k <= L) {
            buf[k] = cscale(buf[k], (T)(1.0 / (N2 * a.psihat_t[k])));
        } else {
            C z;
            z.x = z.y = (T)0;
            buf[k] = z;
        }
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fnt, +1, a.tw_nt);
    for (int r = threadIdx.x; r < a.rows_used; r += fft_threads<T>(MAXN)) {
        int row = (a.row_lo + r) % NT;
        if (row < 0) row += NT;
        V[(int64_t)r * ldv + mi] = buf[row];
    }
}

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_theta_synth_split(StageArgs a, const double2 *F,
                                                             typename CT<T>::type *V) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int mi = xcd_column(blockIdx.x, 2 * a.mmax + 1);
    if (mi > 2 * a.mmax) return;
    const int am = abs(mi - a.mmax);
    const double sig = ((a.spin + am) & 1) ? -1.0 : 1.0;  // mirror sign (-1)^(s+m)
    const int L = a.L, N2 = a.N2, NT = a.NT;
    const double2 *Fm = F + (int64_t)mi * a.nring;
    for (int k = threadIdx.x; k < N2; k += fft_threads<T>(MAXN)) {
        const int j = k <= L ? k : N2 - k;
        const double wj = (k <= L ? 1.0 : sig) * a.ring_w[j];
        double2 v = make_double2(0.0, 0.0);
        if (a.ring_mmax[j] >= am) v = Fm[j];
        C c;
        c.x = (T)(v.x * wj);
        c.y = (T)(v.y * wj);
        buf[k] = c;
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fn2, -1, a.tw_n2);  // N2 * Fourier coefficient
    const int64_t ldv = 2 * a.mmax + 1;
    {
        typedef ThetaHalves<T, MAXN> H;
        C spec[H::NQ];
#pragma unroll
        for (int q = 0; q < H::NQ; ++q) {
            const int i = threadIdx.x + q * H::NTHR;
            if (i < N2) {
                const int n = i <= L ? i : N2 - i;  // |n|
                spec[q] = cscale(buf[i], (T)(1.0 / (N2 * a.psihat_t[n])));
            }
        }
        for (int h = 0; h < 2; ++h) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < H::NQ; ++q) {
                const int i = threadIdx.x + q * H::NTHR;
                if (i < N2) {
                    C v = spec[q];
                    if (h) v = cmul(v, twiddle<C>(a.tw_nt, i <= L ? i : i - N2 + NT, +1));  // e^{2 pi i n / NT}
                    buf[i] = v;
                }
            }
            __syncthreads();
            lds_fft<T, MAXN>(buf, a.fn2, +1, a.tw_n2);
            for (int r = threadIdx.x; r < a.rows_used; r += H::NTHR) {
                int row = (a.row_lo + r) % NT;
                if (row < 0) row += NT;
                if ((row & 1) == h) V[(int64_t)r * ldv + mi] = buf[row >> 1];
            }
        }
    }
}

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_theta_adjoint(StageArgs a, const typename CT<T>::type *V,
                                                               double2 *F) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int mi = xcd_column(blockIdx.x, 2 * a.mmax + 1);
    if (mi > 2 * a.mmax) return;
    const int am = abs(mi - a.mmax);
    const double sig = ((a.spin + am) & 1) ? -1.0 : 1.0;
    const int L = a.L, N2 = a.N2, NT = a.NT;
    const int64_t ldv = 2 * a.mmax + 1;
    C z;
    z.x = z.y = (T)0;
    for (int k = threadIdx.x; k < NT; k += fft_threads<T>(MAXN)) buf[k] = z;
    __syncthreads();
    for (int r = threadIdx.x; r < a.rows_used; r += fft_threads<T>(MAXN)) {
        int row = (a.row_lo + r) % NT;
        if (row < 0) row += NT;
        buf[row] = V[(int64_t)r * ldv + mi];
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fnt, -1, a.tw_nt);
    // keep |n| <= L, divide by N2 psihat, move n < 0 from NT - |n| to N2 - |n|
    for (int k = threadIdx.x; k <= L; k += fft_threads<T>(MAXN)) {
        const T sc = (T)(1.0 / (N2 * a.psihat_t[k]));
        buf[k] = cscale(buf[k], sc);
        if (k >= 1) buf[N2 - k] = cscale(buf[NT - k], sc);
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fn2, +1, a.tw_n2);
    double2 *Fm = F + (int64_t)mi * a.nring;
    for (int j = threadIdx.x; j <= L; j += fft_threads<T>(MAXN)) {
        C v = buf[j];
        double re = v.x, im = v.y;
        if (j > 0) {
            C u = buf[N2 - j];
            re += sig * (double)u.x;
            im += sig * (double)u.y;
        }
        // orders above the ring's polar cut-off: zero, as the synthesis reads them
        const double wj = a.ring_mmax[j] >= am ? a.ring_w[j] : 0.0;
        Fm[j] = make_double2(re * wj, im * wj);
    }
}

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_theta_adjoint_split(StageArgs a, const typename CT<T>::type *V,
                                                               double2 *F) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int mi = xcd_column(blockIdx.x, 2 * a.mmax + 1);
    if (mi > 2 * a.mmax) return;
    const int am = abs(mi - a.mmax);
    const double sig = ((a.spin + am) & 1) ? -1.0 : 1.0;
    const int L = a.L, N2 = a.N2, NT = a.NT;
    const int64_t ldv = 2 * a.mmax + 1;
    C z;
    z.x = z.y = (T)0;
    {
        typedef ThetaHalves<T, MAXN> H;
        C spec[H::NQ];
        for (int h = 0; h < 2; ++h) {
            for (int k = threadIdx.x; k < N2; k += H::NTHR) buf[k] = z;
            __syncthreads();
            for (int r = threadIdx.x; r < a.rows_used; r += H::NTHR) {
                int row = (a.row_lo + r) % NT;
                if (row < 0) row += NT;
                if ((row & 1) == h) buf[row >> 1] = V[(int64_t)r * ldv + mi];
            }
            __syncthreads();
            lds_fft<T, MAXN>(buf, a.fn2, -1, a.tw_n2);
#pragma unroll
            for (int q = 0; q < H::NQ; ++q) {
                const int i = threadIdx.x + q * H::NTHR;
                if (i < N2) {
                    C v = buf[i];
                    if (h) spec[q] = cadd(spec[q], cmul(v, twiddle<C>(a.tw_nt, i <= L ? i : i - N2 + NT, -1)));
                    else spec[q] = v;
                }
            }
            __syncthreads();
        }
        // divide by N2 psihat(|n|); the spectrum already sits at n mod N2
#pragma unroll
        for (int q = 0; q < H::NQ; ++q) {
            const int i = threadIdx.x + q * H::NTHR;
            if (i < N2) buf[i] = cscale(spec[q], (T)(1.0 / (N2 * a.psihat_t[i <= L ? i : N2 - i])));
        }
        __syncthreads();
    }
    lds_fft<T, MAXN>(buf, a.fn2, +1, a.tw_n2);
    double2 *Fm = F + (int64_t)mi * a.nring;
    for (int j = threadIdx.x; j <= L; j += fft_threads<T>(MAXN)) {
        C v = buf[j];
        double re = v.x, im = v.y;
        if (j > 0) {
            C u = buf[N2 - j];
            re += sig * (double)u.x;
            im += sig * (double)u.y;
        }
        // orders above the ring's polar cut-off: zero, as the synthesis reads them
        const double wj = a.ring_mmax[j] >= am ? a.ring_w[j] : 0.0;
        Fm[j] = make_double2(re * wj, im * wj);
    }
}

// -------------------------------------------------------------- phi stage
//
// Long rows are split into S = 2 (or, above twice the LDS limit, 4) parts,
// each a transform of length nh = Np / S in a workgroup of its own, so that
// more transforms are in flight per CU (a 5880-point FP64 row takes 94 KB of
// LDS, a whole CU's worth for one workgroup).  Both directions split their
// output index, so the parts never write the same element:
//   synthesis, outputs k = S k' + h:  U[S k' + h] = sum_m V_m e^{2 pi i m h / Np} e^{2 pi i m k' / nh},
//     a transform of the spectrum with m taken mod nh (for S = 2 every m lands
//     on its own entry, |m| <= mmax < nh / 2; for S = 4 the entries sum the
//     orders that fold onto them);
//   adjoint, frequencies m = S m' + h:  V_m = sum_{k < nh} y_h[k] e^{-2 pi i m' k / nh},
//     y_h[k] = e^{-2 pi i h k / Np} sum_{j < S} U[k + j nh] e^{-2 pi i h j / S}.

// Row and part of block b.  The S parts of a row go to blocks 8 (S q + h) + x,
// which the round-robin dealing of blocks places on the same XCD, so their
// interleaved outputs meet in one L2.
__device__ inline void phi_block(int b, int parts, int &r, int &h) {
    if (parts == 1) {
        r = b;
        h = 0;
        return;
    }
    const int x = b & 7, q = b >> 3;
    h = q % parts;
    r = 8 * (q / parts) + x;
}

static inline unsigned phi_grid(int rows, int parts) {
    return parts == 1 ? (unsigned)rows : 8u * (unsigned)parts * (unsigned)((rows + 7) / 8);
}

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_phi_synth(StageArgs a, const typename CT<T>::type *V,
                                                           typename CT<T>::type *U) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    int r, h;
    phi_block(blockIdx.x, a.parts, r, h);
    if (r >= a.rows_used) return;
    const int Np = a.Nphi, S = a.parts, nh = Np / S, mm = a.mmax;
    const C *Vr = V + (int64_t)r * (2 * mm + 1);
    C *Ur = U + (int64_t)r * Np;
    C z;
    z.x = z.y = (T)0;
    if (S <= 2) {
        for (int k = threadIdx.x; k < nh; k += fft_threads<T>(MAXN)) buf[k] = z;
        __syncthreads();
        // |m| <= mmax < nh / 2: the m taken mod nh land on distinct entries
        for (int mi = threadIdx.x; mi <= 2 * mm; mi += fft_threads<T>(MAXN)) {
            const int m = mi - mm;
            C v = cscale(Vr[mi], (T)(1.0 / a.psihat_p[abs(m)]));
            if (h) v = cmul(v, twiddle<C>(a.tw_np_full, m < 0 ? m + Np : m, +1));
            buf[m < 0 ? m + nh : m] = v;
        }
    } else {
        // entry t sums the orders m = t (mod nh) in [-mmax, mmax]
        for (int t = threadIdx.x; t < nh; t += fft_threads<T>(MAXN)) {
            C acc = z;
            for (int m = t - nh * ((t + mm) / nh); m <= mm; m += nh) {
                C v = cscale(Vr[m + mm], (T)(1.0 / a.psihat_p[abs(m)]));
                if (h) {
                    int e = (int)(((int64_t)m * h) % Np);
                    if (e < 0) e += Np;
                    v = cmul(v, twiddle<C>(a.tw_np_full, e, +1));
                }
                acc = cadd(acc, v);
            }
            buf[t] = acc;
        }
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fnp, +1, a.tw_np);
    for (int k = threadIdx.x; k < nh; k += fft_threads<T>(MAXN)) Ur[S * k + h] = buf[k];
}

template <typename T, int MAXN>
__global__ __launch_bounds__(fft_threads<T>(MAXN)) void k_phi_adjoint(StageArgs a, const typename CT<T>::type *U,
                                                             typename CT<T>::type *V) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    int r, h;
    phi_block(blockIdx.x, a.parts, r, h);
    if (r >= a.rows_used) return;
    const int Np = a.Nphi, S = a.parts, nh = Np / S, mm = a.mmax;
    C *Vr = V + (int64_t)r * (2 * mm + 1);
    const C *Ur = U + (int64_t)r * Np;
    if (S == 1) {
        for (int k = threadIdx.x; k < nh; k += fft_threads<T>(MAXN)) buf[k] = Ur[k];
    } else if (S == 2) {
        for (int k = threadIdx.x; k < nh; k += fft_threads<T>(MAXN)) {
            const C u0 = Ur[k], u1 = Ur[k + nh];
            buf[k] = h ? cmul(csub(u0, u1), twiddle<C>(a.tw_np_full, k, -1)) : cadd(u0, u1);
        }
    } else {
        for (int k = threadIdx.x; k < nh; k += fft_threads<T>(MAXN)) {
            C acc = Ur[k];
            for (int j = 1; j < S; ++j) {
                const C u = Ur[k + j * nh];
                acc = cadd(acc, h ? cmul(u, twiddle<C>(a.tw_np_full, (h * j * nh) % Np, -1)) : u);
            }
            buf[k] = h ? cmul(acc, twiddle<C>(a.tw_np_full, h * k, -1)) : acc;
        }
    }
    __syncthreads();
    lds_fft<T, MAXN>(buf, a.fnp, -1, a.tw_np);
    // frequencies of this part: m = mi - mmax with m = h (mod S)
    const int mi0 = ((h + mm) % S + S) % S;
    for (int mi = mi0 + S * (int)threadIdx.x; mi <= 2 * mm; mi += S * fft_threads<T>(MAXN)) {
        const int m = mi - mm;
        const int f = m < 0 ? m + Np : m;
        const C v = buf[(f - h) / S];
        Vr[mi] = cscale(v, (T)(1.0 / a.psihat_p[abs(m)]));
    }
}

// ---------------------------------------------------------------- launch

static StageArgs stage_args(const psht_plan_s &p) {
    const Geometry &g = p.g;
    StageArgs a;
    a.fn2 = to_dev(p.fft_n2.f);
    a.fnt = to_dev(p.fft_nt.f);
    a.fnp = to_dev(p.g.phi_parts > 1 ? p.fft_np_part.f : p.fft_np.f);
    a.tw_n2 = reinterpret_cast<const double2 *>(p.fft_n2.d_tw);
    a.tw_nt = reinterpret_cast<const double2 *>(p.fft_nt.d_tw);
    a.tw_np = reinterpret_cast<const double2 *>(p.g.phi_parts > 1 ? p.fft_np_part.d_tw : p.fft_np.d_tw);
    a.tw_np_full = reinterpret_cast<const double2 *>(p.fft_np.d_tw);
    a.L = g.Lmax;
    a.N2 = g.N2;
    a.NT = g.Ntheta;
    a.Nphi = g.Nphi;
    a.nring = g.nring;
    a.mmax = g.mmax;
    a.spin = g.spin;
    a.row_lo = g.row_lo;
    a.rows_used = g.rows_used;
    a.parts = p.g.phi_parts;
    a.tsplit = p.theta_split;
    a.ring_w = p.d_ring_w;
    a.ring_mmax = p.d_ring_mmax;
    a.psihat_t = p.d_psihat_t;
    a.psihat_p = p.d_psihat_p;
    return a;
}

template <typename F> static hipError_t set_lds(F kern, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// Calls fn(std::integral_constant<int, MAXN>) for the smallest build size
// MAXN >= n (n <= 10240).
template <typename Fn> static void tier_dispatch(int n, Fn fn) {
    if (n <= 1024) fn(std::integral_constant<int, 1024>());
    else if (n <= 2048) fn(std::integral_constant<int, 2048>());
    else if (n <= 2560) fn(std::integral_constant<int, 2560>());
    else if (n <= 4096) fn(std::integral_constant<int, 4096>());
    else if (n <= 8192) fn(std::integral_constant<int, 8192>());
    else fn(std::integral_constant<int, 10240>());
}

template <typename T>
static hipError_t theta_synth_t(const psht_plan_s &p, const StageArgs &a, const double2 *F, void *V, hipStream_t st) {
    typedef typename CT<T>::type C;
    const int n = p.theta_split ? p.g.N2 : p.g.Ntheta;
    const size_t lds = (size_t)n * sizeof(C);
    hipError_t err = hipSuccess;
    tier_dispatch(n, [&](auto M) {
        constexpr int MX = decltype(M)::value;
        if (p.theta_split) {
            if ((err = set_lds(k_theta_synth_split<T, MX>, lds)) != hipSuccess) return;
            hipLaunchKernelGGL((k_theta_synth_split<T, MX>), dim3(xcd_grid(2 * p.g.mmax + 1)), dim3(fft_threads<T>(MX)),
                               lds, st, a, F, static_cast<C *>(V));
        } else {
            if ((err = set_lds(k_theta_synth<T, MX>, lds)) != hipSuccess) return;
            hipLaunchKernelGGL((k_theta_synth<T, MX>), dim3(xcd_grid(2 * p.g.mmax + 1)), dim3(fft_threads<T>(MX)), lds,
                               st, a, F, static_cast<C *>(V));
        }
    });
    return err;
}

template <typename T>
static hipError_t theta_adjoint_t(const psht_plan_s &p, const StageArgs &a, const void *V, double2 *F, hipStream_t st) {
    typedef typename CT<T>::type C;
    const int n = p.theta_split ? p.g.N2 : p.g.Ntheta;
    const size_t lds = (size_t)n * sizeof(C);
    hipError_t err = hipSuccess;
    tier_dispatch(n, [&](auto M) {
        constexpr int MX = decltype(M)::value;
        if (p.theta_split) {
            if ((err = set_lds(k_theta_adjoint_split<T, MX>, lds)) != hipSuccess) return;
            hipLaunchKernelGGL((k_theta_adjoint_split<T, MX>), dim3(xcd_grid(2 * p.g.mmax + 1)),
                               dim3(fft_threads<T>(MX)), lds, st, a, static_cast<const C *>(V), F);
        } else {
            if ((err = set_lds(k_theta_adjoint<T, MX>, lds)) != hipSuccess) return;
            hipLaunchKernelGGL((k_theta_adjoint<T, MX>), dim3(xcd_grid(2 * p.g.mmax + 1)), dim3(fft_threads<T>(MX)),
                               lds, st, a, static_cast<const C *>(V), F);
        }
    });
    return err;
}

template <typename T>
static hipError_t phi_synth_t(const psht_plan_s &p, const StageArgs &a, const void *V, void *U, hipStream_t st) {
    typedef typename CT<T>::type C;
    const int nh = p.g.Nphi / p.g.phi_parts;
    const size_t lds = (size_t)nh * sizeof(C);
    hipError_t err = hipSuccess;
    tier_dispatch(nh, [&](auto M) {
        constexpr int MX = decltype(M)::value;
        if ((err = set_lds(k_phi_synth<T, MX>, lds)) != hipSuccess) return;
        hipLaunchKernelGGL((k_phi_synth<T, MX>), dim3(phi_grid(p.g.rows_used, p.g.phi_parts)), dim3(fft_threads<T>(MX)), lds,
                           st, a,
                           static_cast<const C *>(V), static_cast<C *>(U));
    });
    return err;
}

template <typename T>
static hipError_t phi_adjoint_t(const psht_plan_s &p, const StageArgs &a, const void *U, void *V, hipStream_t st) {
    typedef typename CT<T>::type C;
    const int nh = p.g.Nphi / p.g.phi_parts;
    const size_t lds = (size_t)nh * sizeof(C);
    hipError_t err = hipSuccess;
    tier_dispatch(nh, [&](auto M) {
        constexpr int MX = decltype(M)::value;
        if ((err = set_lds(k_phi_adjoint<T, MX>, lds)) != hipSuccess) return;
        hipLaunchKernelGGL((k_phi_adjoint<T, MX>), dim3(phi_grid(p.g.rows_used, p.g.phi_parts)), dim3(fft_threads<T>(MX)),
                           lds, st, a,
                           static_cast<const C *>(U), static_cast<C *>(V));
    });
    return err;
}

hipError_t launch_theta_synth(const psht_plan_s &p, const double *F, void *V, hipStream_t st) {
    const StageArgs a = stage_args(p);
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    const hipError_t e = p.g.fp32 ? theta_synth_t<float>(p, a, F2, V, st) : theta_synth_t<double>(p, a, F2, V, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_theta_adjoint(const psht_plan_s &p, const void *V, double *F, hipStream_t st) {
    const StageArgs a = stage_args(p);
    double2 *F2 = reinterpret_cast<double2 *>(F);
    const hipError_t e = p.g.fp32 ? theta_adjoint_t<float>(p, a, V, F2, st) : theta_adjoint_t<double>(p, a, V, F2, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_phi_synth(const psht_plan_s &p, const void *V, void *U, hipStream_t st) {
    const StageArgs a = stage_args(p);
    const hipError_t e = p.g.fp32 ? phi_synth_t<float>(p, a, V, U, st) : phi_synth_t<double>(p, a, V, U, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_phi_adjoint(const psht_plan_s &p, const void *U, void *V, hipStream_t st) {
    const StageArgs a = stage_args(p);
    const hipError_t e = p.g.fp32 ? phi_adjoint_t<float>(p, a, U, V, st) : phi_adjoint_t<double>(p, a, U, V, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename T>
static hipError_t fft_rows_t(const FftTable &t, int batch, int sign, const void *in, void *out, hipStream_t st) {
    typedef typename CT<T>::type C;
    const FftDev f = to_dev(t.f);
    const double2 *tw = reinterpret_cast<const double2 *>(t.d_tw);
    const size_t lds = (size_t)t.n * sizeof(C);
    hipError_t err = hipSuccess;
    tier_dispatch(t.n, [&](auto M) {
        constexpr int MX = decltype(M)::value;
        if ((err = set_lds(k_fft_rows<T, MX>, lds)) != hipSuccess) return;
        hipLaunchKernelGGL((k_fft_rows<T, MX>), dim3(batch), dim3(fft_threads<T>(MX)), lds, st, f, sign, tw,
                           static_cast<const C *>(in), static_cast<C *>(out));
    });
    return err;
}

hipError_t launch_fft_rows(const FftTable &t, int batch, int sign, bool fp32, const void *in, void *out,
                           hipStream_t st) {
    if (batch == 0) return hipSuccess;
    const hipError_t e = fp32 ? fft_rows_t<float>(t, batch, sign, in, out, st) : fft_rows_t<double>(t, batch, sign, in, out, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace psht
