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

struct FftDev {
    int n, npass;
    int radix[24];
};

static FftDev to_dev(const FftFactors &f) {
    FftDev d;
    d.n = f.n;
    d.npass = f.npass;
    for (int i = 0; i < 24; ++i) d.radix[i] = i < f.npass ? f.radix[i] : 1;
    return d;
}

constexpr int kFftThreads = 512;

template <typename T> struct FftLimit;
template <> struct FftLimit<double> { static constexpr int value = kFftMaxLds64; };
template <> struct FftLimit<float> { static constexpr int value = kFftMaxLds32; };

// e^{sign 2 pi i t / n} from the table tw[k] = e^{-2 pi i k / n}.
template <typename C> __device__ inline C twiddle(const double2 *tw, int k, int sign) {
    double2 w = tw[k];
    C r;
    r.x = w.x;
    r.y = -sign * w.y;
    return r;
}

// Radix-R DFT in registers: y_q = sum_r v_r e^{sign 2 pi i r q / R}.
template <typename C, int R> __device__ inline void dft(C *v, const C *wr, int sign) {
    if (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        C a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d0 = csub(v[1], v[3]);
        C d;  // (sign i) * d0
        d.x = -sign * d0.y;
        d.y = sign * d0.x;
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    } else {
        C out[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            C acc = v[0];
#pragma unroll
            for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(v[r], wr[(r * q) % R]));
            out[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = out[q];
    }
}

// One Stockham pass of radix R on buf[0..n) with stride Ns.
template <typename T, int R>
__device__ void fft_pass(typename CT<T>::type *buf, int n, int Ns, int sign, const double2 *tw) {
    typedef typename CT<T>::type C;
    constexpr int NB = (FftLimit<T>::value / R + kFftThreads - 1) / kFftThreads;
    const int nb = n / R;
    const int tws = n / (Ns * R);
    C wr[R];
#pragma unroll
    for (int t = 0; t < R; ++t) wr[t] = twiddle<C>(tw, t * (n / R), sign);
    C v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int b = threadIdx.x + i * kFftThreads;
        if (b < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[b + r * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int b = threadIdx.x + i * kFftThreads;
        if (b < nb) {
            int k = b % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], twiddle<C>(tw, r * k * tws, sign));
            dft<C, R>(v[i], wr, sign);
            int d = (b - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[d + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// In-place FFT of buf[0..n) in LDS; the caller synchronises before the call.
template <typename T>
__device__ void lds_fft(typename CT<T>::type *buf, const FftDev &f, int sign, const double2 *tw) {
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
        const int R = f.radix[p];
        switch (R) {
            case 4: fft_pass<T, 4>(buf, f.n, Ns, sign, tw); break;
            case 2: fft_pass<T, 2>(buf, f.n, Ns, sign, tw); break;
            case 3: fft_pass<T, 3>(buf, f.n, Ns, sign, tw); break;
            case 5: fft_pass<T, 5>(buf, f.n, Ns, sign, tw); break;
            case 7: fft_pass<T, 7>(buf, f.n, Ns, sign, tw); break;
            case 11: fft_pass<T, 11>(buf, f.n, Ns, sign, tw); break;
            case 13: fft_pass<T, 13>(buf, f.n, Ns, sign, tw); break;
            default: break;
        }
        Ns *= R;
    }
}

// ------------------------------------------------------------ plain rows

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(FftDev f, int sign, const double2 *tw,
                                                          const typename CT<T>::type *in,
                                                          typename CT<T>::type *out) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int64_t row = blockIdx.x;
    for (int k = threadIdx.x; k < f.n; k += kFftThreads) buf[k] = in[row * f.n + k];
    __syncthreads();
    lds_fft<T>(buf, f, sign, tw);
    for (int k = threadIdx.x; k < f.n; k += kFftThreads) out[row * f.n + k] = buf[k];
}

// ------------------------------------------------------------ Theta stage

struct StageArgs {
    FftDev fn2, fnt, fnp;
    const double2 *tw_n2, *tw_nt, *tw_np, *tw_np_full;
    int L, N2, NT, Nphi, nring, mmax, spin, row_lo, rows_used;
    bool split;  // phi FFT as two half-length transforms
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

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_theta_synth(StageArgs a, const double2 *F,
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
    for (int k = threadIdx.x; k < N2; k += kFftThreads) {
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
    lds_fft<T>(buf, a.fn2, -1, a.tw_n2);  // N2 * Fourier coefficient
    // divide by N2 psihat(|n|) and pad to NT: n < 0 moves from N2 - |n| to NT - |n|
    for (int n = 1 + threadIdx.x; n <= L; n += kFftThreads)
        buf[NT - n] = cscale(buf[N2 - n], (T)(1.0 / (N2 * a.psihat_t[n])));
    __syncthreads();
    for (int k = threadIdx.x; k < NT - L; k += kFftThreads) {
        if (k <= L) {
            buf[k] = cscale(buf[k], (T)(1.0 / (N2 * a.psihat_t[k])));
        } else {
            C z;
            z.x = z.y = (T)0;
            buf[k] = z;
        }
    }
    __syncthreads();
    lds_fft<T>(buf, a.fnt, +1, a.tw_nt);
    const int64_t ldv = 2 * a.mmax + 1;
    for (int r = threadIdx.x; r < a.rows_used; r += kFftThreads) {
        int row = (a.row_lo + r) % NT;
        if (row < 0) row += NT;
        V[(int64_t)r * ldv + mi] = buf[row];
    }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_theta_adjoint(StageArgs a, const typename CT<T>::type *V,
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
    for (int k = threadIdx.x; k < NT; k += kFftThreads) buf[k] = z;
    __syncthreads();
    for (int r = threadIdx.x; r < a.rows_used; r += kFftThreads) {
        int row = (a.row_lo + r) % NT;
        if (row < 0) row += NT;
        buf[row] = V[(int64_t)r * ldv + mi];
    }
    __syncthreads();
    lds_fft<T>(buf, a.fnt, -1, a.tw_nt);
    // keep |n| <= L, divide by N2 psihat, move n < 0 from NT - |n| to N2 - |n|
    for (int k = threadIdx.x; k <= L; k += kFftThreads) {
        const T sc = (T)(1.0 / (N2 * a.psihat_t[k]));
        buf[k] = cscale(buf[k], sc);
        if (k >= 1) buf[N2 - k] = cscale(buf[NT - k], sc);
    }
    __syncthreads();
    lds_fft<T>(buf, a.fn2, +1, a.tw_n2);
    double2 *Fm = F + (int64_t)mi * a.nring;
    for (int j = threadIdx.x; j <= L; j += kFftThreads) {
        C v = buf[j];
        double re = v.x, im = v.y;
        if (j > 0) {
            C u = buf[N2 - j];
            re += sig * (double)u.x;
            im += sig * (double)u.y;
        }
        const double wj = a.ring_w[j];
        Fm[j] = make_double2(re * wj, im * wj);
    }
}

// -------------------------------------------------------------- phi stage

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_phi_synth(StageArgs a, const typename CT<T>::type *V,
                                                           typename CT<T>::type *U) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int64_t r = blockIdx.x;
    const int Np = a.Nphi, nh = a.split ? Np / 2 : Np, mm = a.mmax;
    const C *Vr = V + r * (2 * mm + 1);
    C *Ur = U + r * Np;
    C z;
    z.x = z.y = (T)0;
    for (int h = 0; h < (a.split ? 2 : 1); ++h) {
        for (int k = threadIdx.x; k < nh; k += kFftThreads) buf[k] = z;
        __syncthreads();
        for (int mi = threadIdx.x; mi <= 2 * mm; mi += kFftThreads) {
            const int m = mi - mm;
            C v = cscale(Vr[mi], (T)(1.0 / a.psihat_p[abs(m)]));
            if (h) v = cmul(v, twiddle<C>(a.tw_np_full, m < 0 ? m + Np : m, +1));
            buf[m < 0 ? m + nh : m] = v;
        }
        __syncthreads();
        lds_fft<T>(buf, a.fnp, +1, a.tw_np);
        if (a.split) {
            for (int k = threadIdx.x; k < nh; k += kFftThreads) Ur[2 * k + h] = buf[k];
        } else {
            for (int k = threadIdx.x; k < nh; k += kFftThreads) Ur[k] = buf[k];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_phi_adjoint(StageArgs a, const typename CT<T>::type *U,
                                                             typename CT<T>::type *V) {
    typedef typename CT<T>::type C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const int64_t r = blockIdx.x;
    const int Np = a.Nphi, nh = a.split ? Np / 2 : Np, mm = a.mmax;
    C *Vr = V + r * (2 * mm + 1);
    const C *Ur = U + r * Np;
    for (int h = 0; h < (a.split ? 2 : 1); ++h) {
        if (a.split) {
            for (int k = threadIdx.x; k < nh; k += kFftThreads) buf[k] = Ur[2 * k + h];
        } else {
            for (int k = threadIdx.x; k < nh; k += kFftThreads) buf[k] = Ur[k];
        }
        __syncthreads();
        lds_fft<T>(buf, a.fnp, -1, a.tw_np);
        for (int mi = threadIdx.x; mi <= 2 * mm; mi += kFftThreads) {
            const int m = mi - mm;
            C v = buf[m < 0 ? m + nh : m];
            if (h) v = cmul(v, twiddle<C>(a.tw_np_full, m < 0 ? m + Np : m, -1));
            v = cscale(v, (T)(1.0 / a.psihat_p[abs(m)]));
            if (h) v = cadd(v, Vr[mi]);
            Vr[mi] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launch

static StageArgs stage_args(const psht_plan_s &p) {
    const Geometry &g = p.g;
    StageArgs a;
    a.fn2 = to_dev(p.fft_n2.f);
    a.fnt = to_dev(p.fft_nt.f);
    a.fnp = to_dev(p.phi_split ? p.fft_np_half.f : p.fft_np.f);
    a.tw_n2 = reinterpret_cast<const double2 *>(p.fft_n2.d_tw);
    a.tw_nt = reinterpret_cast<const double2 *>(p.fft_nt.d_tw);
    a.tw_np = reinterpret_cast<const double2 *>(p.phi_split ? p.fft_np_half.d_tw : p.fft_np.d_tw);
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
    a.split = p.phi_split;
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

hipError_t launch_theta_synth(const psht_plan_s &p, const double *F, void *V, hipStream_t st) {
    StageArgs a = stage_args(p);
    dim3 grid(xcd_grid(2 * p.g.mmax + 1)), block(kFftThreads);
    const double2 *F2 = reinterpret_cast<const double2 *>(F);
    if (p.g.fp32) {
        size_t lds = (size_t)p.g.Ntheta * sizeof(float2);
        set_lds(k_theta_synth<float>, lds);
        hipLaunchKernelGGL(k_theta_synth<float>, grid, block, lds, st, a, F2, static_cast<float2 *>(V));
    } else {
        size_t lds = (size_t)p.g.Ntheta * sizeof(double2);
        set_lds(k_theta_synth<double>, lds);
        hipLaunchKernelGGL(k_theta_synth<double>, grid, block, lds, st, a, F2, static_cast<double2 *>(V));
    }
    return hipGetLastError();
}

hipError_t launch_theta_adjoint(const psht_plan_s &p, const void *V, double *F, hipStream_t st) {
    StageArgs a = stage_args(p);
    dim3 grid(xcd_grid(2 * p.g.mmax + 1)), block(kFftThreads);
    double2 *F2 = reinterpret_cast<double2 *>(F);
    if (p.g.fp32) {
        size_t lds = (size_t)p.g.Ntheta * sizeof(float2);
        set_lds(k_theta_adjoint<float>, lds);
        hipLaunchKernelGGL(k_theta_adjoint<float>, grid, block, lds, st, a, static_cast<const float2 *>(V), F2);
    } else {
        size_t lds = (size_t)p.g.Ntheta * sizeof(double2);
        set_lds(k_theta_adjoint<double>, lds);
        hipLaunchKernelGGL(k_theta_adjoint<double>, grid, block, lds, st, a, static_cast<const double2 *>(V), F2);
    }
    return hipGetLastError();
}

hipError_t launch_phi_synth(const psht_plan_s &p, const void *V, void *U, hipStream_t st) {
    StageArgs a = stage_args(p);
    dim3 grid(p.g.rows_used), block(kFftThreads);
    int nh = p.phi_split ? p.g.Nphi / 2 : p.g.Nphi;
    if (p.g.fp32) {
        size_t lds = (size_t)nh * sizeof(float2);
        set_lds(k_phi_synth<float>, lds);
        hipLaunchKernelGGL(k_phi_synth<float>, grid, block, lds, st, a, static_cast<const float2 *>(V),
                           static_cast<float2 *>(U));
    } else {
        size_t lds = (size_t)nh * sizeof(double2);
        set_lds(k_phi_synth<double>, lds);
        hipLaunchKernelGGL(k_phi_synth<double>, grid, block, lds, st, a, static_cast<const double2 *>(V),
                           static_cast<double2 *>(U));
    }
    return hipGetLastError();
}

hipError_t launch_phi_adjoint(const psht_plan_s &p, const void *U, void *V, hipStream_t st) {
    StageArgs a = stage_args(p);
    dim3 grid(p.g.rows_used), block(kFftThreads);
    int nh = p.phi_split ? p.g.Nphi / 2 : p.g.Nphi;
    if (p.g.fp32) {
        size_t lds = (size_t)nh * sizeof(float2);
        set_lds(k_phi_adjoint<float>, lds);
        hipLaunchKernelGGL(k_phi_adjoint<float>, grid, block, lds, st, a, static_cast<const float2 *>(U),
                           static_cast<float2 *>(V));
    } else {
        size_t lds = (size_t)nh * sizeof(double2);
        set_lds(k_phi_adjoint<double>, lds);
        hipLaunchKernelGGL(k_phi_adjoint<double>, grid, block, lds, st, a, static_cast<const double2 *>(U),
                           static_cast<double2 *>(V));
    }
    return hipGetLastError();
}

hipError_t launch_fft_rows(const FftTable &t, int batch, int sign, bool fp32, const void *in, void *out,
                           hipStream_t st) {
    FftDev f = to_dev(t.f);
    const double2 *tw = reinterpret_cast<const double2 *>(t.d_tw);
    dim3 grid(batch), block(kFftThreads);
    if (batch == 0) return hipSuccess;
    if (fp32) {
        size_t lds = (size_t)t.n * sizeof(float2);
        set_lds(k_fft_rows<float>, lds);
        hipLaunchKernelGGL(k_fft_rows<float>, grid, block, lds, st, f, sign, tw, static_cast<const float2 *>(in),
                           static_cast<float2 *>(out));
    } else {
        size_t lds = (size_t)t.n * sizeof(double2);
        set_lds(k_fft_rows<double>, lds);
        hipLaunchKernelGGL(k_fft_rows<double>, grid, block, lds, st, f, sign, tw, static_cast<const double2 *>(in),
                           static_cast<double2 *>(out));
    }
    return hipGetLastError();
}

}  // namespace psht
