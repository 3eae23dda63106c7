// Field passes of the two-dimensional step (the 2-D runs of Sec. 5.2):
// real-to-complex 2-D FFT of the deposit, the implicit (or, with eps = 0,
// elliptic) mode update, the filtered spectral gradient and the
// complex-to-real inverse FFT of its two components.
//
// Convention: beta_q = L^-2 sum_j phi_j e^{-2 pi i q.j/H},
// grad c(x_j) = sum_q i xi_q Phi_q alpha_q e^{+2 pi i q.j/H}.
//
// Grid sizes H = 8 .. 4096 (a row of 4096 complex values fits in LDS).  Three
// passes per step, each staged through LDS:
//   fwd_rows  R rows of phi per workgroup: each real row along y is read as
//             H/2 complex values, transformed and split into its half
//             spectrum (ky = 0..H/2); the spectrum is written transposed,
//             ky-major, so that the next pass reads whole rows.  Clears the
//             deposit and advances the step counter.
//   xrows     one workgroup per ky: transform along x, update alpha, form
//             i xi_d Phi alpha for d = x, y and inverse-transform each along x.
//   inv_rows  R rows per workgroup and component: gather the transposed
//             spectrum, half-length complex-to-real inverse along y.
#include "internal.h"
#include "lds_fft.h"

namespace sipf {

#ifndef SIPF_XROW_THREADS
#define SIPF_XROW_THREADS 256
#endif
#ifndef SIPF_ROWS2_MUL
#define SIPF_ROWS2_MUL 1
#endif
constexpr int ROW_THREADS = 512;
constexpr int XROW_THREADS = SIPF_XROW_THREADS;

// rows per workgroup of the row passes: R (H/2 + 1) values plus an H-entry
// twiddle table stay within LDS; R rows give R-value runs in the transposed
// spectrum
template <typename T, int H> struct Rows2 {
    static constexpr int R0 = H <= 16 ? H : (H <= 512 ? 16 : (H == 1024 ? 8 : (H == 2048 ? 4 : 2)));
    static constexpr int R1 = R0 * SIPF_ROWS2_MUL;
    static constexpr bool fits = (size_t)(R1 * (H / 2 + 1) + H) * 2 * sizeof(T) <= 150 * 1024;
    static constexpr int R = (H >= 1024 && R1 <= 16 && fits) ? R1 : R0;
};

enum { XR_STEP = 0, XR_GRAD = 1, XR_RHO = 4 };

template <typename T, int H>
__global__ __launch_bounds__(ROW_THREADS) void k2_fwd_rows(const FieldDesc<T>* __restrict__ fds, int consume) {
    using V = cplx_t<T>;
    constexpr int M = H / 2, HH = M + 1, OP = HH, R = Rows2<T, H>::R;
    constexpr int NP = M / 2 + 1;  // pairs (k, M - k) per row
    constexpr int PPT = (R * NP + ROW_THREADS - 1) / ROW_THREADS;
    __shared__ V buf[R * OP];
    __shared__ V tw[H];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int ix0 = blockIdx.x * R;
    const int tid = threadIdx.x, nt = blockDim.x;
    make_twiddles<T, H>(tw);
    T* rows = fd.phi + (size_t)ix0 * H;
    for (int u = tid; u < R * M; u += nt) {
        const int r = u / M, m = u % M;
        buf[r * OP + m] = cmake<V, T>(rows[r * H + 2 * m], rows[r * H + 2 * m + 1]);
    }
    __syncthreads();
    if (consume) {
        for (int u = tid; u < R * H; u += nt) rows[u] = (T)0;
        if (blockIdx.x == 0 && tid == 0 && fd.step != nullptr) *fd.step += 1u;
    }
    lds_fft_g<T, M, -1>(buf, R, OP, 1, tw, 2);
    __syncthreads();
    V za[PPT], zb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < R * NP) {
            const int r = u / NP, k = u % NP;
            za[q] = buf[r * OP + perm_pos_g<M>(k % M)];
            zb[q] = buf[r * OP + perm_pos_g<M>((M - k) % M)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < R * NP) {
            const int r = u / NP, k = u % NP;
            const V zc = cconj(zb[q]);
            const V e = cscale(cadd(za[q], zc), (T)0.5);
            const V dd = csub(za[q], zc);
            const V o = cmake<V, T>(dd.y * (T)0.5, -dd.x * (T)0.5);  // (Z_k - conj Z_{M-k}) / (2i)
            buf[r * OP + k] = cadd(e, cmul(tw[k], o));
            if (k != M - k) buf[r * OP + (M - k)] = cadd(cconj(e), cmul(tw[M - k], cconj(o)));
        }
    }
    __syncthreads();
    for (int u = tid; u < HH * R; u += nt) {
        const int k = u / R, r = u % R;
        fd.B1[(size_t)k * H + ix0 + r] = buf[r * OP + k];
    }
}

template <typename T, int H, int MODE>
__global__ __launch_bounds__(XROW_THREADS) void k2_xrows(const FieldDesc<T>* __restrict__ fds) {
    using V = cplx_t<T>;
    constexpr int NV = (H + XROW_THREADS - 1) / XROW_THREADS;  // spectrum values per thread
    __shared__ V buf[H];
    __shared__ V tw[H];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int ky = blockIdx.x;  // 0 .. H/2
    const int tid = threadIdx.x, nt = blockDim.x;
    make_twiddles<T, H>(tw);
    const T qy = (T)ky;
    const size_t row = (size_t)ky * H;
    if constexpr (MODE == XR_STEP || MODE == XR_RHO) {
        for (int i = tid; i < H; i += nt) buf[i] = fd.B1[row + i];
        __syncthreads();
        lds_fft_g<T, H, -1>(buf, 1, H, 1, tw, 1);
        __syncthreads();
    }
    if constexpr (MODE == XR_RHO) {
        for (int p = tid; p < H; p += nt) {
            const int kx = perm_freq_g<H>(p);
            const T qx = (T)(kx < H / 2 ? kx : kx - H);
            const T q2 = qx * qx + qy * qy;
            const T f = (fd.filt > (T)0 ? exp(-fd.filt * q2) : (T)1) * fd.inv_Ld;
            buf[p] = cscale(buf[p], f);
        }
        __syncthreads();
        lds_fft_g<T, H, +1>(buf, 1, H, 1, tw, 1);
        __syncthreads();
        for (int i = tid; i < H; i += nt) fd.gspec[row + i] = buf[i];
        return;
    } else {
        // alpha (updated in STEP mode) times the filter, kept in registers
        V af[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int p = tid + j * XROW_THREADS;
            if (p < H) {
                const int kx = perm_freq_g<H>(p);
                const T qx = (T)(kx < H / 2 ? kx : kx - H);
                const T q2 = qx * qx + qy * qy;
                V a = fd.alpha[row + p];
                if constexpr (MODE == XR_STEP) {
                    T A, B;
                    mode_ab(fd, q2 * fd.two_pi_over_L * fd.two_pi_over_L + fd.k2, A, B);
                    const V beta = buf[p];
                    const T bs = B * fd.inv_Ld;
                    a = cmake<V, T>(A * a.x + bs * beta.x, A * a.y + bs * beta.y);
                    fd.alpha[row + p] = a;
                }
                af[j] = cscale(a, fd.filt > (T)0 ? exp(-fd.filt * q2) : (T)1);
            }
        }
        for (int d = 0; d < 2; ++d) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int p = tid + j * XROW_THREADS;
                if (p < H) {
                    const int kd = d == 0 ? perm_freq_g<H>(p) : ky;
                    // derivative factor i xi_d, zero at the Nyquist frequency |q_d| = H/2
                    const T q = (T)(kd == H / 2 ? 0 : (kd < H / 2 ? kd : kd - H));
                    const T xi = q * fd.two_pi_over_L;
                    buf[p] = cmake<V, T>(-xi * af[j].y, xi * af[j].x);
                }
            }
            __syncthreads();
            lds_fft_g<T, H, +1>(buf, 1, H, 1, tw, 1);
            __syncthreads();
            V* out = fd.gspec + (size_t)d * (H / 2 + 1) * H + row;
            for (int i = tid; i < H; i += nt) out[i] = buf[i];
        }
    }
}

template <typename T, int H>
__global__ __launch_bounds__(ROW_THREADS) void k2_inv_rows(const FieldDesc<T>* __restrict__ fds, int ncomp) {
    using V = cplx_t<T>;
    constexpr int M = H / 2, HH = M + 1, OP = HH, R = Rows2<T, H>::R;
    constexpr int NP = M / 2 + 1;
    constexpr int PPT = (R * NP + ROW_THREADS - 1) / ROW_THREADS;
    __shared__ V buf[R * OP];
    __shared__ V tw[H];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int d = blockIdx.x % ncomp;
    const int ix0 = (blockIdx.x / ncomp) * R;
    const int tid = threadIdx.x, nt = blockDim.x;
    make_twiddles<T, H>(tw);
    const V* in = fd.gspec + (size_t)d * HH * H;
    for (int u = tid; u < HH * R; u += nt) {
        const int k = u / R, r = u % R;
        buf[r * OP + k] = in[(size_t)k * H + ix0 + r];
    }
    __syncthreads();
    V xa[PPT], xb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < R * NP) {
            const int r = u / NP, k = u % NP;
            xa[q] = buf[r * OP + k];
            xb[q] = buf[r * OP + (M - k)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < R * NP) {
            const int r = u / NP, k = u % NP;
            // Z_k from (X_k, X_{M-k}); Z_{M-k} from (X_{M-k}, X_k) for 0 < k < M - k
            const V s1 = cadd(xa[q], cconj(xb[q])), d1 = csub(xa[q], cconj(xb[q]));
            const V t1 = cmul(cconj(tw[k]), d1);
            buf[r * OP + perm_pos_g<M>(k % M)] = cmake<V, T>(s1.x - t1.y, s1.y + t1.x);
            if (k != 0 && k != M - k) {
                const V s2 = cadd(xb[q], cconj(xa[q])), d2 = csub(xb[q], cconj(xa[q]));
                const V t2 = cmul(cconj(tw[M - k]), d2);
                buf[r * OP + perm_pos_g<M>(M - k)] = cmake<V, T>(s2.x - t2.y, s2.y + t2.x);
            }
        }
    }
    __syncthreads();
    lds_fft_g<T, M, +1>(buf, R, OP, 1, tw, 2);
    __syncthreads();
    T* outp = fd.G + (size_t)d * H * H + (size_t)ix0 * H;
    for (int u = tid; u < R * M; u += nt) {
        const int r = u / M, m = u % M;
        const V v = buf[r * OP + m];
        outp[r * H + 2 * m] = v.x;
        outp[r * H + 2 * m + 1] = v.y;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int H>
static hipError_t fwd_rows_h(const FieldDesc<T>* fd, int count, bool consume, hipStream_t s) {
    launch_kernel((k2_fwd_rows<T, H>), dim3(H / Rows2<T, H>::R, count), dim3(ROW_THREADS), 0, s, fd, consume ? 1 : 0);
    return hipGetLastError();
}
template <typename T, int H>
static hipError_t xrows_h(const FieldDesc<T>* fd, int count, int mode, hipStream_t s) {
    const dim3 g(H / 2 + 1, count), b(XROW_THREADS);
    switch (mode) {
        case XP_STEP: launch_kernel((k2_xrows<T, H, XR_STEP>), g, b, 0, s, fd); break;
        case XP_GRAD: launch_kernel((k2_xrows<T, H, XR_GRAD>), g, b, 0, s, fd); break;
        case XP_RHO: launch_kernel((k2_xrows<T, H, XR_RHO>), g, b, 0, s, fd); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename T, int H>
static hipError_t inv_rows_h(const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s) {
    launch_kernel((k2_inv_rows<T, H>), dim3((H / Rows2<T, H>::R) * ncomp, count), dim3(ROW_THREADS), 0, s, fd, ncomp);
    return hipGetLastError();
}

#define SIPF_H2_SWITCH(H, FN, ...)                \
    switch (H) {                                  \
        case 8: return FN<T, 8>(__VA_ARGS__);     \
        case 16: return FN<T, 16>(__VA_ARGS__);   \
        case 32: return FN<T, 32>(__VA_ARGS__);   \
        case 64: return FN<T, 64>(__VA_ARGS__);   \
        case 128: return FN<T, 128>(__VA_ARGS__); \
        case 256: return FN<T, 256>(__VA_ARGS__); \
        case 512: return FN<T, 512>(__VA_ARGS__); \
        case 1024: return FN<T, 1024>(__VA_ARGS__); \
        case 2048: return FN<T, 2048>(__VA_ARGS__); \
        case 4096: return FN<T, 4096>(__VA_ARGS__); \
        default: return hipErrorInvalidValue;     \
    }

template <typename T> hipError_t launch_fwd_rows2(int H, const FieldDesc<T>* fd, int count, bool consume, hipStream_t s) {
    SIPF_H2_SWITCH(H, fwd_rows_h, fd, count, consume, s)
}
template <typename T> hipError_t launch_xrows2(int H, const FieldDesc<T>* fd, int count, int mode, hipStream_t s) {
    SIPF_H2_SWITCH(H, xrows_h, fd, count, mode, s)
}
template <typename T> hipError_t launch_inv_rows2(int H, const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s) {
    SIPF_H2_SWITCH(H, inv_rows_h, fd, count, ncomp, s)
}

bool fft2d_size_supported(int H) {
    return H == 8 || H == 16 || H == 32 || H == 64 || H == 128 || H == 256 || H == 512 || H == 1024 || H == 2048 ||
           H == 4096;
}

template hipError_t launch_fwd_rows2<float>(int, const FieldDesc<float>*, int, bool, hipStream_t);
template hipError_t launch_fwd_rows2<double>(int, const FieldDesc<double>*, int, bool, hipStream_t);
template hipError_t launch_xrows2<float>(int, const FieldDesc<float>*, int, int, hipStream_t);
template hipError_t launch_xrows2<double>(int, const FieldDesc<double>*, int, int, hipStream_t);
template hipError_t launch_inv_rows2<float>(int, const FieldDesc<float>*, int, int, hipStream_t);
template hipError_t launch_inv_rows2<double>(int, const FieldDesc<double>*, int, int, hipStream_t);

}  // namespace sipf
