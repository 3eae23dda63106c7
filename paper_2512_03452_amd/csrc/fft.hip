// Field passes of the SIPF-PIC step: real-to-complex 3-D FFT of the deposit,
// implicit mode update, filtered spectral gradient and complex-to-real 3-D
// inverse FFT of its three components (Algorithm 2's last line, the mode
// update and the gradient lines of Algorithm 4).
//
// Transform convention (Sec. 3.1): beta_q = L^-3 sum_j phi_j e^{-2 pi i q.j/H},
// grad c(x_j) = sum_q i xi_q Phi_q alpha_q e^{+2 pi i q.j/H}.
//
// Three passes over HBM per step, each staged through LDS (five at H = 256,
// where a plane pass splits into a row pass and a column pass, see below):
//   fwd_planes  one workgroup per x-plane: each real row along z is read as
//               H/2 complex values, transformed, and split into its half
//               spectrum (kz = 0..H/2); then the plane is transformed along y.
//               Also zeroes the deposit grid for the next step and advances
//               the step counter.
//   xpencils    one workgroup per 16 consecutive (ky, kz) x-pencils: transform
//               along x, alpha <- A alpha + B beta, form i xi_d Phi alpha for
//               d = 0,1,2 and inverse-transform each along x.
//   inv_planes  one workgroup per (component, x-plane): inverse along y, then
//               the half-length complex-to-real inverse along z.
//
// The LDS FFT (lds_fft.h) leaves the forward transform in a digit-permuted
// order and takes that order back in the inverse; the x and y frequency axes
// of the stored spectra use it.
#include "internal.h"
#include "lds_fft.h"

namespace sipf {

int fft_perm(int N, int k) {
    int N1 = 0, N2 = 1;
    switch (N) {
#define SIPF_SPLIT_CASE(n) case n: N1 = Split<n>::N1; N2 = Split<n>::N2; break;
        SIPF_SPLIT_CASE(3) SIPF_SPLIT_CASE(4) SIPF_SPLIT_CASE(5) SIPF_SPLIT_CASE(6) SIPF_SPLIT_CASE(8)
        SIPF_SPLIT_CASE(11) SIPF_SPLIT_CASE(12) SIPF_SPLIT_CASE(16) SIPF_SPLIT_CASE(22) SIPF_SPLIT_CASE(23)
        SIPF_SPLIT_CASE(32) SIPF_SPLIT_CASE(45) SIPF_SPLIT_CASE(46) SIPF_SPLIT_CASE(64) SIPF_SPLIT_CASE(90)
        SIPF_SPLIT_CASE(128) SIPF_SPLIT_CASE(256)
#undef SIPF_SPLIT_CASE
        case 512: case 1024: case 2048: case 4096: {
            const int M = N / 16;
            return (k % 16) * M + fft_perm(M, k / 16);
        }
        default: return -1;
    }
    return (k % N1) * N2 + k / N1;
}

// 3-D grids: powers of two 8 .. 256 and the mixed-radix sizes 12, 22, 46, 90;
// FP64 up to 64 (the plane passes' LDS)
bool fft_size_supported(int H, bool fp64) {
    switch (H) {
        case 8: case 12: case 16: case 22: case 32: case 46: case 64: return true;
        case 90: case 128: case 256: return !fp64;
        default: return false;
    }
}

// threads of the plane passes: the forward pass has only H workgroups and the
// inverse 3H, so a plane gets 1024 threads (measured at H = 128: 16.9 -> 13.3
// us forward, 19.6 -> 17.6 us inverse, against 512)
#ifndef SIPF_FWD_THREADS
#define SIPF_FWD_THREADS 1024
#endif
#ifndef SIPF_INV_THREADS
#define SIPF_INV_THREADS 1024
#endif
constexpr int FWD_THREADS = SIPF_FWD_THREADS;
constexpr int PLANE_THREADS = SIPF_INV_THREADS;
// x-pencil and y-column passes: 512 threads (measured x-pencil pass: H = 128
// 25.1 / 22.1 / 31.4 us and H = 64 11.0 / 8.7 / 7.9 us at 256 / 512 / 1024)
constexpr int PENCIL_THREADS = 512;
#ifndef SIPF_KB
#define SIPF_KB 16
#endif
constexpr int KB = SIPF_KB;  // kz columns per x-pencil workgroup

// v, or zero when ok is false (per component: a select of whole vector
// values goes through scratch memory).
template <typename V> __device__ __forceinline__ V keep_if(bool ok, const V& v) {
    V r;
    r.x = ok ? v.x : 0;
    r.y = ok ? v.y : 0;
    return r;
}

// Copy of N elements by the NT threads of a workgroup, element u read by
// ld(u) and written by st(u, v): every read of a thread is issued before its
// first write, so a copy between HBM and LDS costs one memory round trip (a
// loop of read-then-write pairs waits for each read in turn).  Threads past
// the end re-read element N - 1 and write nothing.
template <int NT, int N, typename V, typename Ld, typename St>
__device__ __forceinline__ void stage(const Ld& ld, const St& st) {
    constexpr int R = (N + NT - 1) / NT;
    V v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int u = (int)threadIdx.x + q * NT;
        v[q] = ld(N % NT == 0 ? u : min(u, N - 1));
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int u = (int)threadIdx.x + q * NT;
        if (N % NT == 0 || u < N) st(u, v[q]);
    }
}

// ---------------------------------------------------------------------------
// Pass 1: x-plane -> half spectrum along z, transformed along y.
//
// Real rows along z by the half-length method: row x (length H = 2M) is read
// as z[m] = x[2m] + i x[2m+1], transformed with an M-point FFT, and
//   E_k = (Z_k + conj Z_{M-k}) / 2,  O_k = (Z_k - conj Z_{M-k}) / (2i),
//   X_k = E_k + exp(-2 pi i k / H) O_k,   k = 0 .. M,
// so one plane buffer of H x (M+1) values holds both stages.  The pairs
// (k, M-k) are read into registers before they are written back, since the
// FFT leaves Z in permuted order.
// ---------------------------------------------------------------------------
template <typename T, int H>
__global__ __launch_bounds__(FWD_THREADS) void k_fwd_planes(const FieldDesc<T>* __restrict__ fds, int consume) {
    using V = cplx_t<T>;
    constexpr int M = H / 2;
    constexpr int HH = M + 1;
    constexpr int OP = HH;  // row pitch (complex)
    constexpr int NP = M / 2 + 1;  // pairs (k, M - k) per row, k = 0 .. M/2
    constexpr int PPT = (H * NP + FWD_THREADS - 1) / FWD_THREADS;
    __shared__ V buf[H * OP];
    __shared__ V tw[H];
    __shared__ V twm[M];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int ix = blockIdx.x % H;
    const int comp = blockIdx.x / H;  // component of a multi-grid input (phi + comp H^3)
    const int tid = threadIdx.x, nt = blockDim.x;
    make_twiddles<T, H>(tw);
    make_twiddles<T, M>(twm);
    T* plane = fd.phi + ((size_t)comp * H + ix) * H * H;
    V* pv = reinterpret_cast<V*>(plane);  // (x[2m], x[2m+1]) of row r at r M + m
    stage<FWD_THREADS, H * M, V>([&](int u) { return pv[u]; },
                                 [&](int u, const V& v) { buf[(u / M) * OP + u % M] = v; });
    __syncthreads();
    if (consume) {
        // the deposit grid is consumed: clear it for the next step's particle pass
        for (int u = tid; u < H * M; u += nt) pv[u] = cmake<V, T>(0, 0);
        if (ix == 0 && comp == 0 && tid == 0 && fd.step != nullptr) *fd.step += 1u;
    }
    lds_fft<T, M, -1>(buf, H, OP, 1, twm);
    __syncthreads();
    V za[PPT], zb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * FWD_THREADS;
        if (u < H * NP) {
            const int row = u / NP, k = u % NP;
            za[q] = buf[row * OP + perm_pos<M>(k % M)];
            zb[q] = buf[row * OP + perm_pos<M>((M - k) % M)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * FWD_THREADS;
        if (u < H * NP) {
            const int row = u / NP, k = u % NP;
            const V zc = cconj(zb[q]);
            const V e = cscale(cadd(za[q], zc), (T)0.5);
            const V dd = csub(za[q], zc);
            const V o = cmake<V, T>(dd.y * (T)0.5, -dd.x * (T)0.5);  // (Z_k - conj Z_{M-k}) / (2i)
            buf[row * OP + k] = cadd(e, cmul(tw[k], o));
            if (k != M - k) buf[row * OP + (M - k)] = cadd(cconj(e), cmul(tw[M - k], cconj(o)));
        }
    }
    __syncthreads();
    lds_fft<T, H, -1>(buf, HH, 1, OP, tw);
    __syncthreads();
    V* out = fd.B1 + ((size_t)comp * H + ix) * H * HH;
    stage<FWD_THREADS, H * HH, V>([&](int u) { return buf[u]; }, [&](int u, const V& v) { out[u] = v; });
}

// ---------------------------------------------------------------------------
// Pass 2: x-pencils, mode update, filtered gradient spectra, inverse along x.
// ---------------------------------------------------------------------------
template <typename T, int H, int MODE>
__device__ __forceinline__ void adjoint_pencils(const FieldDesc<T>& fd, int c0, int ncol, T qy, int ky, int kz,
                                                cplx_t<T>* lds, const cplx_t<T>* tw);

// MODE_STEP: forward x of B1, mode update of alpha, three gradient spectra
//            i xi_d Phi alpha, inverse x into gspec.
// MODE_GRAD: the three gradient spectra of alpha (no update).
// MODE_ADJ_SRC: adjoint of the source term: L^-3 B abar (abar in alpha), inverse x
//            into gspec component 0.
// MODE_ADJ_ACC: adjoint of the gradient and of the propagation: forward x of the
//            three transformed grids in B1, abar <- A abar + sum_d (-i xi_d Phi) B1_d.
// MODE_RHO:  forward x of B1 (a deposit), Gaussian factor Phi and L^-3, inverse x
//            into gspec component 0: the regularised density rho_hat * G0 after
//            the inverse plane pass.
// MODE_ADJ_ACC_SRC: MODE_ADJ_ACC, then MODE_ADJ_SRC of the updated abar in the
//            same pass (the reverse sweep needs the source term of abar^(n-1)
//            right after accumulating it).
enum { MODE_STEP = 0, MODE_GRAD = 1, MODE_ADJ_SRC = 2, MODE_ADJ_ACC = 3, MODE_RHO = 4, MODE_ADJ_ACC_SRC = 5 };

// A block is KB consecutive columns of the half spectrum flattened over
// (ky, kz) (column c = ky_position (H/2 + 1) + kz), all H x rows of each: a
// row of the block is KB contiguous values starting at a multiple of KB, one
// aligned 128-byte line in FP32 (blocks of KB kz values of one ky straddled
// two lines, since H/2 + 1 is odd).  Every entry a thread touches lies in the
// same column (the thread count is a multiple of KB), so ky and kz are the
// thread's own.
//
// At H = 128 (FP32) the registers are budgeted for three workgroups per CU
// (six waves per SIMD), so that all 520 blocks are resident at once; smaller
// grids have fewer blocks than CUs and leave the count to the compiler.
template <typename T, int H, int MODE>
__global__ __launch_bounds__(PENCIL_THREADS) __attribute__((amdgpu_waves_per_eu(H >= 128 ? 6 : 1))) void k_xpencils(
    const FieldDesc<T>* __restrict__ fds) {
    constexpr bool UPDATE = MODE == MODE_STEP;
    using V = cplx_t<T>;
    constexpr int HH = H / 2 + 1;
    constexpr int NC = H * HH;       // columns (ky, kz): the pitch of an x row in HBM
    constexpr int BP = KB + 1;       // pitch (complex) of one x row in LDS, one grid
    constexpr int BP3 = 3 * KB + 1;  // the same for the three gradient components side by side
    constexpr int NB = H * KB;       // entries of the block
    constexpr int NT = PENCIL_THREADS;
    constexpr int R = (NB + NT - 1) / NT;
    static_assert(NT % KB == 0, "a thread's entries share one column");
    __shared__ V lds[H * BP3];
    __shared__ V tw[H];
    V* buf = lds;
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int c0 = blockIdx.x * KB;
    const int ncol = min(KB, NC - c0);
    const int tid = threadIdx.x;
    make_twiddles<T, H>(tw);
    // the thread's column (a column past ncol takes the last valid one)
    const int cc = c0 + min(tid % KB, ncol - 1);
    const int kyp = cc / HH;
    const int kz = cc - kyp * HH;
    const int ky = perm_freq<H>(kyp);
    const T qy = (T)(ky < H / 2 ? ky : ky - H);
    // entry u of the block: x row (or permuted kx position) u / KB, column u % KB
    // (columns past ncol read the last valid one and are written as zero)
    auto gidx = [&](int u) { return (size_t)(u / KB) * NC + c0 + min(u % KB, ncol - 1); };
    if constexpr (MODE == MODE_ADJ_SRC || MODE == MODE_ADJ_ACC || MODE == MODE_ADJ_ACC_SRC) {
        adjoint_pencils<T, H, MODE>(fd, c0, ncol, qy, ky, kz, lds, tw);
        return;
    }
    const V zero = cmake<V, T>(0, 0);
    if constexpr (MODE == MODE_RHO) {
        stage<NT, NB, V>([&](int u) { return fd.B1[gidx(u)]; },
                         [&](int u, const V& v) { buf[(u / KB) * BP + u % KB] = keep_if(u % KB < ncol, v); });
        __syncthreads();
        lds_fft<T, H, -1>(buf, KB, 1, BP, tw);
        __syncthreads();
        for (int u = tid; u < NB; u += NT) {
            const int p = u / KB, j = u % KB;
            const int kx = perm_freq<H>(p);
            const T qx = (T)(kx < H / 2 ? kx : kx - H);
            const T qz = (T)kz;
            const T q2 = qx * qx + qy * qy + qz * qz;
            const T f = (fd.filt > (T)0 ? exp(-fd.filt * q2) : (T)1) * fd.inv_Ld;
            const V b = buf[p * BP + j];
            buf[p * BP + j] = j < ncol ? cmake<V, T>(b.x * f, b.y * f) : zero;
        }
        __syncthreads();
        lds_fft<T, H, +1>(buf, KB, 1, BP, tw);
        __syncthreads();
        stage<NT, NB, V>([&](int u) { return buf[(u / KB) * BP + u % KB]; },
                         [&](int u, const V& v) { if (u % KB < ncol) fd.gspec[gidx(u)] = v; });
        return;
    }
    // alpha of the block, read together with B1 (before the transform)
    V av[R];
#pragma unroll
    for (int q = 0; q < R; ++q) av[q] = fd.alpha[gidx(min(tid + q * NT, NB - 1))];
    if (UPDATE) {
        stage<NT, NB, V>([&](int u) { return fd.B1[gidx(u)]; },
                         [&](int u, const V& v) { buf[(u / KB) * BP + u % KB] = keep_if(u % KB < ncol, v); });
        __syncthreads();
        lds_fft<T, H, -1>(buf, KB, 1, BP, tw);
        __syncthreads();
    }
    // spectral update in permuted kx order (position p holds kx = perm_freq(p)),
    // then Phi alpha, kept in registers
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int u = tid + q * NT;
        const int p = u / KB, j = u % KB;
        V a = zero;
        if (u < NB && j < ncol) {
            const int kx = perm_freq<H>(p);
            const T qx = (T)(kx < H / 2 ? kx : kx - H);
            const T qz = (T)kz;
            const T q2 = qx * qx + qy * qy + qz * qz;
            a = av[q];
            if (UPDATE) {
                const T xi2 = q2 * fd.two_pi_over_L * fd.two_pi_over_L;
                T A, B;
                mode_ab(fd, xi2 + fd.k2, A, B);
                const V beta = buf[p * BP + j];
                const T bs = B * fd.inv_Ld;
                a = cmake<V, T>(A * a.x + bs * beta.x, A * a.y + bs * beta.y);
                fd.alpha[gidx(u)] = a;
            }
            const T phi = fd.filt > (T)0 ? exp(-fd.filt * q2) : (T)1;
            a = cmake<V, T>(a.x * phi, a.y * phi);
        }
        av[q] = a;
    }
    if (UPDATE) __syncthreads();  // beta is read: the three components overwrite it
    // i xi_d Phi alpha for d = 0, 1, 2 in columns d KB + j (zero at the Nyquist
    // frequency |q_d| = H/2), transformed along x together
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int u = tid + q * NT;
        if (u < NB) {
            const int p = u / KB, j = u % KB;
            const int kd[3] = {perm_freq<H>(p), ky, kz};
            const V a = av[q];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T qd = (T)(kd[d] == H / 2 ? 0 : (kd[d] < H / 2 ? kd[d] : kd[d] - H));
                const T xi = qd * fd.two_pi_over_L;
                lds[p * BP3 + d * KB + j] = cmake<V, T>(-xi * a.y, xi * a.x);
            }
        }
    }
    __syncthreads();
    lds_fft<T, H, +1>(lds, 3 * KB, 1, BP3, tw);
    __syncthreads();
    // component d of entry u at column d KB + u % KB
#pragma unroll
    for (int d = 0; d < 3; ++d)
        stage<NT, NB, V>([&](int u) { return lds[(u / KB) * BP3 + d * KB + u % KB]; },
                         [&](int u, const V& v) { if (u % KB < ncol) fd.gspec[(size_t)d * H * H * HH + gidx(u)] = v; });
}

// lds holds H (3 KB + 1) values: one grid block at pitch KB + 1, or the three
// components side by side at pitch 3 KB + 1.
template <typename T, int H, int MODE>
__device__ __forceinline__ void adjoint_pencils(const FieldDesc<T>& fd, int c0, int ncol, T qy, int ky, int kz,
                                                cplx_t<T>* lds, const cplx_t<T>* tw) {
    using V = cplx_t<T>;
    constexpr int HH = H / 2 + 1;
    constexpr int BP = KB + 1;
    constexpr int BP3 = 3 * KB + 1;
    constexpr int NB = H * KB;
    constexpr int NT = PENCIL_THREADS;
    constexpr int R = (NB + NT - 1) / NT;
    const int tid = threadIdx.x;
    const V zero = cmake<V, T>(0, 0);
    constexpr int NC = H * HH;
    auto gidx = [&](int u) { return (size_t)(u / KB) * NC + c0 + min(u % KB, ncol - 1); };
    auto factors = [&](int p, T& A, T& B, T& phi, T (&xi)[3]) {
        const int kx = perm_freq<H>(p);
        const T qx = (T)(kx < H / 2 ? kx : kx - H);
        const T qz = (T)kz;
        const T q2 = qx * qx + qy * qy + qz * qz;
        const T xi2 = q2 * fd.two_pi_over_L * fd.two_pi_over_L;
        mode_ab(fd, xi2 + fd.k2, A, B);
        phi = fd.filt > (T)0 ? exp(-fd.filt * q2) : (T)1;
        const int kd[3] = {kx, ky, kz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T q = (T)(kd[d] == H / 2 ? 0 : (kd[d] < H / 2 ? kd[d] : kd[d] - H));
            xi[d] = q * fd.two_pi_over_L;
        }
    };
    // L^-3 B a of the block into lds (pitch BP), inverse along x, into gspec component 0
    auto source_out = [&]() {
        __syncthreads();
        lds_fft<T, H, +1>(lds, KB, 1, BP, tw);
        __syncthreads();
        stage<NT, NB, V>([&](int u) { return lds[(u / KB) * BP + u % KB]; },
                         [&](int u, const V& v) { if (u % KB < ncol) fd.gspec[gidx(u)] = v; });
    };
    if constexpr (MODE == MODE_ADJ_SRC) {
        stage<NT, NB, V>([&](int u) { return fd.alpha[gidx(u)]; },
                         [&](int u, const V& a) {
                             const int p = u / KB, j = u % KB;
                             V v = zero;
                             if (j < ncol) {
                                 T A, B, phi, xi[3];
                                 factors(p, A, B, phi, xi);
                                 const T sc = B * fd.inv_Ld;
                                 v = cmake<V, T>(a.x * sc, a.y * sc);
                             }
                             lds[p * BP + j] = v;
                         });
        source_out();
    } else {
        // abar of the block, read together with the three transformed grids
        V av[R];
#pragma unroll
        for (int q = 0; q < R; ++q) av[q] = fd.alpha[gidx(min(tid + q * NT, NB - 1))];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            stage<NT, NB, V>([&](int u) { return fd.B1[(size_t)d * H * H * HH + gidx(u)]; },
                             [&](int u, const V& v) { lds[(u / KB) * BP3 + d * KB + u % KB] = keep_if(u % KB < ncol, v); });
        __syncthreads();
        lds_fft<T, H, -1>(lds, 3 * KB, 1, BP3, tw);
        __syncthreads();
        // abar <- A abar + sum_d (-i xi_d Phi) F(Gbar_d)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int u = tid + q * NT;
            const int p = u / KB, j = u % KB;
            V out = zero;
            if (u < NB && j < ncol) {
                T A, B, phi, xi[3];
                factors(p, A, B, phi, xi);
                V acc = zero;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const V g = lds[p * BP3 + d * KB + j];
                    const T c = xi[d] * phi;
                    // (-i c) g = (c g.y, -c g.x)
                    acc.x += c * g.y;
                    acc.y -= c * g.x;
                }
                const V a = av[q];
                const V na = cmake<V, T>(A * a.x + acc.x, A * a.y + acc.y);
                fd.alpha[gidx(u)] = na;
                const T sc = B * fd.inv_Ld;
                out = cmake<V, T>(na.x * sc, na.y * sc);
            }
            av[q] = out;
        }
        if constexpr (MODE == MODE_ADJ_ACC_SRC) {
            __syncthreads();  // the transformed grids are read
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int u = tid + q * NT;
                if (u < NB) lds[(u / KB) * BP + u % KB] = av[q];
            }
            source_out();
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse along y, complex-to-real inverse along z, per component.
//
// Along z the half spectrum X_0 .. X_M of each row gives the M-point input
//   Z_k = (X_k + conj X_{M-k}) + i exp(+2 pi i k / H) (X_k - conj X_{M-k}),
// whose inverse transform is z[m] = x[2m] + i x[2m+1] (unnormalised, as the
// gradient synthesis needs).
// ---------------------------------------------------------------------------
template <typename T, int H>
__global__ __launch_bounds__(PLANE_THREADS) void k_inv_planes(const FieldDesc<T>* __restrict__ fds, int ncomp) {
    using V = cplx_t<T>;
    constexpr int M = H / 2;
    constexpr int HH = M + 1;
    constexpr int OP = HH;
    constexpr int NP = M / 2 + 1;
    constexpr int PPT = (H * NP + PLANE_THREADS - 1) / PLANE_THREADS;
    __shared__ V buf[H * OP];
    __shared__ V tw[H];
    __shared__ V twm[M];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    // blocks 8c + r (c = (ix / 8) ncomp + d) keep the components of a plane on
    // one XCD; grids that are not a multiple of 8 take block ix ncomp + d
    const int b = blockIdx.x;
    int d, ix;
    if constexpr (H % 8 == 0) {
        const int grp = b / 8, r = b % 8;
        d = grp % ncomp;
        ix = (grp / ncomp) * 8 + r;
    } else {
        d = b % ncomp;
        ix = b / ncomp;
    }
    const int tid = threadIdx.x;
    make_twiddles<T, H>(tw);
    make_twiddles<T, M>(twm);
    const V* in = fd.gspec + ((size_t)d * H + ix) * H * HH;
    stage<PLANE_THREADS, H * HH, V>([&](int u) { return in[u]; }, [&](int u, const V& v) { buf[u] = v; });
    __syncthreads();
    lds_fft<T, H, +1>(buf, HH, 1, OP, tw);
    __syncthreads();
    V xa[PPT], xb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * PLANE_THREADS;
        if (u < H * NP) {
            const int row = u / NP, k = u % NP;
            xa[q] = buf[row * OP + k];
            xb[q] = buf[row * OP + (M - k)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * PLANE_THREADS;
        if (u < H * NP) {
            const int row = u / NP, k = u % NP;
            // Z_k from (X_k, X_{M-k}); Z_{M-k} from (X_{M-k}, X_k) for 0 < k < M - k
            const V s1 = cadd(xa[q], cconj(xb[q])), d1 = csub(xa[q], cconj(xb[q]));
            const V t1 = cmul(cconj(tw[k]), d1);
            buf[row * OP + perm_pos<M>(k % M)] = cmake<V, T>(s1.x - t1.y, s1.y + t1.x);
            if (k != 0 && k != M - k) {
                const V s2 = cadd(xb[q], cconj(xa[q])), d2 = csub(xb[q], cconj(xa[q]));
                const V t2 = cmul(cconj(tw[M - k]), d2);
                buf[row * OP + perm_pos<M>(M - k)] = cmake<V, T>(s2.x - t2.y, s2.y + t2.x);
            }
        }
    }
    __syncthreads();
    lds_fft<T, M, +1>(buf, H, OP, 1, twm);
    __syncthreads();
    V* outp = reinterpret_cast<V*>(fd.G + ((size_t)d * H + ix) * H * H);  // (x[2m], x[2m+1]) pairs
    stage<PLANE_THREADS, H * M, V>([&](int u) { return buf[(u / M) * OP + u % M]; },
                                   [&](int u, const V& v) { outp[u] = v; });
}

// ---------------------------------------------------------------------------
// Grids whose yz-plane of half spectrum does not fit in LDS (H = 256: 264 KB
// in FP32).  Each plane pass splits in two, with one more trip through HBM:
//   fwd_zrows  ZROWS rows along z per workgroup: the half-length real
//              transform of fwd_planes, written to B1 with y in natural
//              order; consumes the deposit and advances the step counter.
//   ycols      KB kz columns of one x-plane per workgroup, transformed along
//              y in place (forward: natural -> digit-permuted y, as
//              fwd_planes leaves it; inverse: permuted -> natural).
//   inv_zrows  ZROWS rows per workgroup: the half-length complex-to-real
//              inverse of inv_planes.
// ---------------------------------------------------------------------------
constexpr int ZROWS = 16;
constexpr int ROW_THREADS = 256;

template <typename T, int H>
__global__ __launch_bounds__(ROW_THREADS) void k_fwd_zrows(const FieldDesc<T>* __restrict__ fds, int consume) {
    using V = cplx_t<T>;
    constexpr int M = H / 2;
    constexpr int HH = M + 1;
    constexpr int OP = HH;
    constexpr int NP = M / 2 + 1;
    constexpr int PPT = (ZROWS * NP + ROW_THREADS - 1) / ROW_THREADS;
    constexpr int NRB = H * H / ZROWS;  // row blocks per component
    __shared__ V buf[ZROWS * OP];
    __shared__ V tw[H];
    __shared__ V twm[M];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int comp = blockIdx.x / NRB;
    const size_t row0 = (size_t)(blockIdx.x % NRB) * ZROWS;  // row r = x H + y
    const int tid = threadIdx.x, nt = blockDim.x;
    make_twiddles<T, H>(tw);
    make_twiddles<T, M>(twm);
    T* rows = fd.phi + ((size_t)comp * H * H + row0) * H;
    V* rv = reinterpret_cast<V*>(rows);
    stage<ROW_THREADS, ZROWS * M, V>([&](int u) { return rv[u]; },
                                     [&](int u, const V& v) { buf[(u / M) * OP + u % M] = v; });
    __syncthreads();
    if (consume) {
        for (int u = tid; u < ZROWS * M; u += nt) rv[u] = cmake<V, T>(0, 0);
        if (blockIdx.x == 0 && tid == 0 && fd.step != nullptr) *fd.step += 1u;
    }
    lds_fft<T, M, -1>(buf, ZROWS, OP, 1, twm);
    __syncthreads();
    V za[PPT], zb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < ZROWS * NP) {
            const int row = u / NP, k = u % NP;
            za[q] = buf[row * OP + perm_pos<M>(k % M)];
            zb[q] = buf[row * OP + perm_pos<M>((M - k) % M)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < ZROWS * NP) {
            const int row = u / NP, k = u % NP;
            const V zc = cconj(zb[q]);
            const V e = cscale(cadd(za[q], zc), (T)0.5);
            const V dd = csub(za[q], zc);
            const V o = cmake<V, T>(dd.y * (T)0.5, -dd.x * (T)0.5);
            buf[row * OP + k] = cadd(e, cmul(tw[k], o));
            if (k != M - k) buf[row * OP + (M - k)] = cadd(cconj(e), cmul(tw[M - k], cconj(o)));
        }
    }
    __syncthreads();
    V* out = fd.B1 + ((size_t)comp * H * H + row0) * HH;
    stage<ROW_THREADS, ZROWS * HH, V>([&](int u) { return buf[u]; }, [&](int u, const V& v) { out[u] = v; });
}

template <typename T, int H, int DIR>
__global__ __launch_bounds__(PENCIL_THREADS) void k_ycols(const FieldDesc<T>* __restrict__ fds) {
    using V = cplx_t<T>;
    constexpr int HH = H / 2 + 1;
    constexpr int NKB = (HH + KB - 1) / KB;
    constexpr int BP = KB + 1;
    __shared__ V buf[H * BP];
    __shared__ V tw[H];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int kb = blockIdx.x % NKB, rest = blockIdx.x / NKB;
    const int x = rest % H, comp = rest / H;
    const int kz0 = kb * KB;
    const int ncol = min(KB, HH - kz0);
    V* base = (DIR < 0 ? fd.B1 : fd.gspec) + ((size_t)comp * H + x) * H * HH;
    make_twiddles<T, H>(tw);
    auto gi = [&](int u) { return (size_t)(u / KB) * HH + kz0 + min(u % KB, ncol - 1); };
    stage<PENCIL_THREADS, H * KB, V>(
        [&](int u) { return base[gi(u)]; },
        [&](int u, const V& v) { buf[(u / KB) * BP + u % KB] = keep_if(u % KB < ncol, v); });
    __syncthreads();
    lds_fft<T, H, DIR>(buf, KB, 1, BP, tw);
    __syncthreads();
    stage<PENCIL_THREADS, H * KB, V>([&](int u) { return buf[(u / KB) * BP + u % KB]; },
                                     [&](int u, const V& v) { if (u % KB < ncol) base[gi(u)] = v; });
}

template <typename T, int H>
__global__ __launch_bounds__(ROW_THREADS) void k_inv_zrows(const FieldDesc<T>* __restrict__ fds) {
    using V = cplx_t<T>;
    constexpr int M = H / 2;
    constexpr int HH = M + 1;
    constexpr int OP = HH;
    constexpr int NP = M / 2 + 1;
    constexpr int PPT = (ZROWS * NP + ROW_THREADS - 1) / ROW_THREADS;
    constexpr int NRB = H * H / ZROWS;
    __shared__ V buf[ZROWS * OP];
    __shared__ V tw[H];
    __shared__ V twm[M];
    const FieldDesc<T>& fd = fds[blockIdx.y];
    const int d = blockIdx.x / NRB;
    const size_t row0 = (size_t)(blockIdx.x % NRB) * ZROWS;
    const int tid = threadIdx.x;
    make_twiddles<T, H>(tw);
    make_twiddles<T, M>(twm);
    const V* in = fd.gspec + ((size_t)d * H * H + row0) * HH;
    stage<ROW_THREADS, ZROWS * HH, V>([&](int u) { return in[u]; }, [&](int u, const V& v) { buf[u] = v; });
    __syncthreads();
    V xa[PPT], xb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < ZROWS * NP) {
            const int row = u / NP, k = u % NP;
            xa[q] = buf[row * OP + k];
            xb[q] = buf[row * OP + (M - k)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int u = tid + q * ROW_THREADS;
        if (u < ZROWS * NP) {
            const int row = u / NP, k = u % NP;
            const V s1 = cadd(xa[q], cconj(xb[q])), d1 = csub(xa[q], cconj(xb[q]));
            const V t1 = cmul(cconj(tw[k]), d1);
            buf[row * OP + perm_pos<M>(k % M)] = cmake<V, T>(s1.x - t1.y, s1.y + t1.x);
            if (k != 0 && k != M - k) {
                const V s2 = cadd(xb[q], cconj(xa[q])), d2 = csub(xb[q], cconj(xa[q]));
                const V t2 = cmul(cconj(tw[M - k]), d2);
                buf[row * OP + perm_pos<M>(M - k)] = cmake<V, T>(s2.x - t2.y, s2.y + t2.x);
            }
        }
    }
    __syncthreads();
    lds_fft<T, M, +1>(buf, ZROWS, OP, 1, twm);
    __syncthreads();
    V* outp = reinterpret_cast<V*>(fd.G + ((size_t)d * H * H + row0) * H);
    stage<ROW_THREADS, ZROWS * M, V>([&](int u) { return buf[(u / M) * OP + u % M]; },
                                     [&](int u, const V& v) { outp[u] = v; });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// grids above 128 take the split passes (a plane of half spectrum does not fit in LDS)
#ifndef SIPF_MAX_PLANE_H
#define SIPF_MAX_PLANE_H 128
#endif
constexpr int MAX_PLANE_H = SIPF_MAX_PLANE_H;

template <typename T, int H>
static hipError_t fwd_planes_h(const FieldDesc<T>* fd, int count, int ncomp, bool consume, hipStream_t s) {
    if constexpr (H > MAX_PLANE_H) {
        static_assert((H * H) % ZROWS == 0, "row blocks");
        constexpr int NKB = (H / 2 + 1 + KB - 1) / KB;
        launch_kernel((k_fwd_zrows<T, H>), dim3(ncomp * H * H / ZROWS, count), dim3(ROW_THREADS), 0, s, fd,
                      consume ? 1 : 0);
        launch_kernel((k_ycols<T, H, -1>), dim3(ncomp * H * NKB, count), dim3(PENCIL_THREADS), 0, s, fd);
    } else {
        launch_kernel((k_fwd_planes<T, H>), dim3(H * ncomp, count), dim3(FWD_THREADS), 0, s, fd, consume ? 1 : 0);
    }
    return hipGetLastError();
}
template <typename T, int H>
static hipError_t xpencils_h(const FieldDesc<T>* fd, int count, int mode, hipStream_t s) {
    const dim3 g((H * (H / 2 + 1) + KB - 1) / KB, count), b(PENCIL_THREADS);
    switch (mode) {
        case MODE_STEP: launch_kernel((k_xpencils<T, H, MODE_STEP>), g, b, 0, s, fd); break;
        case MODE_GRAD: launch_kernel((k_xpencils<T, H, MODE_GRAD>), g, b, 0, s, fd); break;
        case MODE_ADJ_SRC: launch_kernel((k_xpencils<T, H, MODE_ADJ_SRC>), g, b, 0, s, fd); break;
        case MODE_ADJ_ACC: launch_kernel((k_xpencils<T, H, MODE_ADJ_ACC>), g, b, 0, s, fd); break;
        case MODE_ADJ_ACC_SRC: launch_kernel((k_xpencils<T, H, MODE_ADJ_ACC_SRC>), g, b, 0, s, fd); break;
        case MODE_RHO: launch_kernel((k_xpencils<T, H, MODE_RHO>), g, b, 0, s, fd); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename T, int H>
static hipError_t inv_planes_h(const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s) {
    if constexpr (H > MAX_PLANE_H) {
        constexpr int NKB = (H / 2 + 1 + KB - 1) / KB;
        launch_kernel((k_ycols<T, H, +1>), dim3(ncomp * H * NKB, count), dim3(PENCIL_THREADS), 0, s, fd);
        launch_kernel((k_inv_zrows<T, H>), dim3(ncomp * H * H / ZROWS, count), dim3(ROW_THREADS), 0, s, fd);
    } else {
        launch_kernel((k_inv_planes<T, H>), dim3(ncomp * H, count), dim3(PLANE_THREADS), 0, s, fd, ncomp);
    }
    return hipGetLastError();
}

#define SIPF_H_SWITCH(H, FN, ...)                         \
    switch (H) {                                          \
        case 8: return FN<T, 8>(__VA_ARGS__);             \
        case 12: return FN<T, 12>(__VA_ARGS__);           \
        case 16: return FN<T, 16>(__VA_ARGS__);           \
        case 22: return FN<T, 22>(__VA_ARGS__);           \
        case 32: return FN<T, 32>(__VA_ARGS__);           \
        case 46: return FN<T, 46>(__VA_ARGS__);           \
        case 64: return FN<T, 64>(__VA_ARGS__);           \
        case 90: if constexpr (sizeof(T) == 4) return FN<T, 90>(__VA_ARGS__); else return hipErrorInvalidValue; \
        case 128: if constexpr (sizeof(T) == 4) return FN<T, 128>(__VA_ARGS__); else return hipErrorInvalidValue; \
        case 256: if constexpr (sizeof(T) == 4) return FN<T, 256>(__VA_ARGS__); else return hipErrorInvalidValue; \
        default: return hipErrorInvalidValue;             \
    }

template <typename T>
hipError_t launch_fwd_planes(int H, const FieldDesc<T>* fd, int count, int ncomp, bool consume, hipStream_t s) {
    SIPF_H_SWITCH(H, fwd_planes_h, fd, count, ncomp, consume, s)
}
template <typename T> hipError_t launch_xpencils(int H, const FieldDesc<T>* fd, int count, int mode, hipStream_t s) {
    SIPF_H_SWITCH(H, xpencils_h, fd, count, mode, s)
}
template <typename T> hipError_t launch_inv_planes(int H, const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s) {
    SIPF_H_SWITCH(H, inv_planes_h, fd, count, ncomp, s)
}

template hipError_t launch_fwd_planes<float>(int, const FieldDesc<float>*, int, int, bool, hipStream_t);
template hipError_t launch_fwd_planes<double>(int, const FieldDesc<double>*, int, int, bool, hipStream_t);
template hipError_t launch_xpencils<float>(int, const FieldDesc<float>*, int, int, hipStream_t);
template hipError_t launch_xpencils<double>(int, const FieldDesc<double>*, int, int, hipStream_t);
template hipError_t launch_inv_planes<float>(int, const FieldDesc<float>*, int, int, hipStream_t);
template hipError_t launch_inv_planes<double>(int, const FieldDesc<double>*, int, int, hipStream_t);

}  // namespace sipf
