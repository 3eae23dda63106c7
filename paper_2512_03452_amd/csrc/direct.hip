// The direct SIPF method (Algorithm 1): every particle meets every Fourier
// mode, O(P H^3) work per step, no grid.  It is the in-house baseline the
// particle-in-cell step is measured against.
//
//   beta_q  = M0 / (P L^3) sum_p exp(-i xi_q . X_p)          (eq. beta_hat_comp)
//   alpha_q <- A_q alpha_q + B_q beta_q                       (eq. alpha_hat_update)
//   grad c(X_p) = Re sum_q i xi_q Phi_q alpha_q exp(i xi_q . X_p)   (eq. gradc)
// over the full index set U = {-H/2 .. H/2-1}^3, spectra in natural order
// (array index k stands for q = k for k < H/2 and q = k - H otherwise).
//
// The exponentials are separable: for a fixed (qx, qy) the phases along qz
// form a geometric sequence, so a thread evaluates one sincos and then
// advances by a complex multiplication per qz (exp(-/+ i 2 pi z / L) per
// particle, computed once).  In FP32 the sequence is re-anchored with a fresh
// sincos every DIR_ANCHOR terms, so that the rounding of the repeated
// multiplication stays that of a few steps.  Three kernels per step:
//   dir_beta    thread = (kx, ky, run of QZ consecutive q_z); the particles of
//               one slice of the particle range pass through LDS; per-slice
//               partial sums.  Also advances the step counter.
//   dir_modes   thread = mode: sums the slice partials in a fixed order, forms
//               the gradient coefficients i xi Phi alpha^(n-1), then updates
//               alpha.
//   dir_grad    thread = particle, workgroup row = slice of the (kx, ky)
//               pairs: the gradient sum at the particle over the slice (the
//               coefficients of DIR_PAIRS pairs at a time pass through LDS).
//   dir_push    sums the slices in a fixed order and pushes: Algorithm 1
//               (Euler-Maruyama) or the split step of Algorithm 4.
#include "internal.h"
#include "pass_common.h"
#include "sipf.h"

namespace sipf {

constexpr int DIR_THREADS = 256;
constexpr int DIR_PCHUNK = 256;  // particles staged per LDS pass of dir_beta
constexpr int DIR_PAIRS = 8;     // (kx, ky) pairs staged per LDS pass of dir_push
constexpr int DIR_ANCHOR = 8;    // FP32: phase terms between fresh sincos evaluations

__device__ __forceinline__ int signed_q(int k, int H) { return k < H / 2 ? k : k - H; }

// exp(-2 pi i t) with t reduced to [-1/2, 1/2] first
template <typename T> __device__ __forceinline__ cplx_t<T> cis_neg(T t) {
    t -= rint(t);
    T s, c;
    if constexpr (sizeof(T) == 4) sincospif(-2.0f * t, &s, &c);
    else sincospi(-2.0 * t, &s, &c);
    return cmake<cplx_t<T>, T>(c, s);
}

template <typename T, int H, int QZ>
__global__ __launch_bounds__(DIR_THREADS) void k_dir_beta(DirDesc<T> d, cplx_t<T>* __restrict__ part) {
    using V = cplx_t<T>;
    constexpr int NZC = H / QZ;
    __shared__ T sx[DIR_PCHUNK], sy[DIR_PCHUNK], sz[DIR_PCHUNK];
    __shared__ V sstep[DIR_PCHUNK];
    const int tid = threadIdx.x;
    const int c = blockIdx.x * DIR_THREADS + tid;  // column: (kx, ky, run of q_z)
    const bool active = c < H * H * NZC;
    const int zc = c % NZC, rest = c / NZC;
    const int qx = signed_q(rest / H, H), qy = signed_q(rest % H, H);
    const int qz0 = signed_q(zc * QZ, H);  // runs of QZ indices hold consecutive q_z (QZ divides H/2)
    const int64_t per = (d.P + gridDim.y - 1) / gridDim.y;
    const int64_t p0 = (int64_t)blockIdx.y * per;
    const int64_t p1 = min(d.P, p0 + per);
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && d.step != nullptr) *d.step += 1u;
    V acc[QZ];
#pragma unroll
    for (int j = 0; j < QZ; ++j) acc[j] = cmake<V, T>(0, 0);
    for (int64_t b = p0; b < p1; b += DIR_PCHUNK) {
        const int n = (int)min((int64_t)DIR_PCHUNK, p1 - b);
        __syncthreads();
        if (tid < n) {
            const T x = d.x[b + tid] * d.invL, y = d.y[b + tid] * d.invL, z = d.z[b + tid] * d.invL;
            sx[tid] = x;
            sy[tid] = y;
            sz[tid] = z;
            sstep[tid] = cis_neg<T>(z);
        }
        __syncthreads();
        if (active) {
            for (int i = 0; i < n; ++i) {
                const T base = (T)qx * sx[i] + (T)qy * sy[i];
                V e = cis_neg<T>(base + (T)qz0 * sz[i]);
                const V st = sstep[i];
#pragma unroll
                for (int j = 0; j < QZ; ++j) {
                    if (sizeof(T) == 4 && j > 0 && j % DIR_ANCHOR == 0) e = cis_neg<T>(base + (T)(qz0 + j) * sz[i]);
                    acc[j] = cadd(acc[j], e);
                    e = cmul(e, st);
                }
            }
        }
    }
    if (active) {
        V* out = part + (size_t)blockIdx.y * H * H * H + (size_t)c * QZ;
#pragma unroll
        for (int j = 0; j < QZ; ++j) out[j] = acc[j];
    }
}

template <typename T, int H>
__global__ __launch_bounds__(DIR_THREADS) void k_dir_modes(DirDesc<T> d, const cplx_t<T>* __restrict__ part,
                                                           int nslices) {
    using V = cplx_t<T>;
    const int m = blockIdx.x * DIR_THREADS + threadIdx.x;
    if (m >= H * H * H) return;
    const int kz = m % H, ky = (m / H) % H, kx = m / (H * H);
    const T qx = (T)signed_q(kx, H), qy = (T)signed_q(ky, H), qz = (T)signed_q(kz, H);
    V beta = cmake<V, T>(0, 0);
    for (int s = 0; s < nslices; ++s) beta = cadd(beta, part[(size_t)s * H * H * H + m]);
    beta = cscale(beta, d.bscale);
    const V a = d.alpha[m];
    const T q2 = qx * qx + qy * qy + qz * qz;
    const T phi = d.fd.filt > (T)0 ? exp(-d.fd.filt * q2) : (T)1;
    const T w = d.fd.two_pi_over_L;
    const T xs[3] = {qx * w, qy * w, qz * w};
#pragma unroll
    for (int c = 0; c < 3; ++c)  // i xi_c Phi alpha
        d.gc[(size_t)c * H * H * H + m] = cmake<V, T>(-xs[c] * phi * a.y, xs[c] * phi * a.x);
    T A, B;
    mode_ab(d.fd, q2 * w * w + d.fd.k2, A, B);
    d.alpha[m] = cmake<V, T>(A * a.x + B * beta.x, A * a.y + B * beta.y);
}

// the particle's position at which the drift is taken (Y = X + W^- for the
// split step, X for Euler-Maruyama) and its remaining noise
template <typename T, int SCHEME>
__device__ __forceinline__ void dir_noise(const DirDesc<T>& d, int64_t p, T& x, T& y, T& z, T& w0, T& w1, T& w2) {
    x = d.x[p];
    y = d.y[p];
    z = d.z[p];
    T zn[6];
    const uint32_t n = *d.step;  // advanced by this step's dir_beta
    if (SCHEME == SIPF_STRANG) {
        noise6<3, T>((uint32_t)p, n, d.inst, d.k0, d.k1, zn);
        x += d.s * zn[0];
        y += d.s * zn[1];
        z += d.s * zn[2];
        w0 = zn[3];
        w1 = zn[4];
        w2 = zn[5];
    } else {
        noise6<2, T>((uint32_t)p, n, d.inst, d.k0, d.k1, zn);
        w0 = zn[0];
        w1 = zn[1];
        w2 = zn[2];
    }
}

// partial gradient sums over the (kx, ky) pairs of slice blockIdx.y
template <typename T, int H, int SCHEME>
__global__ __launch_bounds__(DIR_THREADS) void k_dir_grad(DirDesc<T> d, T* __restrict__ gpart) {
    using V = cplx_t<T>;
    __shared__ V sg[3][DIR_PAIRS][H];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * DIR_THREADS + tid;
    const bool active = p < d.P;
    T x = 0, y = 0, z = 0, w0, w1, w2;
    if (active) dir_noise<T, SCHEME>(d, p, x, y, z, w0, w1, w2);
    const T xl = x * d.invL, yl = y * d.invL, zl = z * d.invL;
    // exp(+i xi . X): conjugate of cis_neg
    V st = cis_neg<T>(zl);
    st.y = -st.y;
    T g0 = 0, g1 = 0, g2 = 0;
    // pairs [first, last) of this slice; the last group of DIR_PAIRS may be ragged
    const int first = (int)((int64_t)blockIdx.y * H * H / gridDim.y);
    const int last = (int)((int64_t)(blockIdx.y + 1) * H * H / gridDim.y);
    for (int pr0 = first; pr0 < last; pr0 += DIR_PAIRS) {
        const int npr = min(DIR_PAIRS, last - pr0);
        __syncthreads();
        for (int u = tid; u < 3 * DIR_PAIRS * H; u += DIR_THREADS) {
            const int c = u / (DIR_PAIRS * H), r = u % (DIR_PAIRS * H);
            const int pr = r / H, j = r % H;
            // q_z ascends from -H/2: storage index (j + H/2) mod H
            if (pr < npr) sg[c][pr][j] = d.gc[(size_t)c * H * H * H + (size_t)(pr0 + pr) * H + (j + H / 2) % H];
        }
        __syncthreads();
        if (active) {
            for (int pr = 0; pr < npr; ++pr) {
                const int kx = (pr0 + pr) / H, ky = (pr0 + pr) % H;
                const T base = (T)signed_q(kx, H) * xl + (T)signed_q(ky, H) * yl;
                V e = cis_neg<T>(-(base - (T)(H / 2) * zl));
#pragma unroll 8
                for (int j = 0; j < H; ++j) {
                    if (sizeof(T) == 4 && j > 0 && j % DIR_ANCHOR == 0) e = cis_neg<T>(-(base + (T)(j - H / 2) * zl));
                    const V a = sg[0][pr][j], b = sg[1][pr][j], c = sg[2][pr][j];
                    g0 += a.x * e.x - a.y * e.y;
                    g1 += b.x * e.x - b.y * e.y;
                    g2 += c.x * e.x - c.y * e.y;
                    e = cmul(e, st);
                }
            }
        }
    }
    if (active) {
        T* out = gpart + (size_t)blockIdx.y * 3 * d.P;
        out[p] = g0;
        out[d.P + p] = g1;
        out[2 * d.P + p] = g2;
    }
}

// sum of the slices in a fixed order, then the push
template <typename T, int SCHEME>
__global__ __launch_bounds__(DIR_THREADS) void k_dir_push(DirDesc<T> d, const T* __restrict__ gpart, int ms) {
    const int64_t p = (int64_t)blockIdx.x * DIR_THREADS + threadIdx.x;
    if (p >= d.P) return;
    T x, y, z, w0, w1, w2;
    dir_noise<T, SCHEME>(d, p, x, y, z, w0, w1, w2);
    T g0 = 0, g1 = 0, g2 = 0;
    for (int k = 0; k < ms; ++k) {
        const T* g = gpart + (size_t)k * 3 * d.P;
        g0 += g[p];
        g1 += g[d.P + p];
        g2 += g[2 * d.P + p];
    }
    const T nx = wrap_box(x + d.chitau * g0 + d.s * w0, d.L, d.halfL, d.invL);
    const T ny = wrap_box(y + d.chitau * g1 + d.s * w1, d.L, d.halfL, d.invL);
    const T nz = wrap_box(z + d.chitau * g2 + d.s * w2, d.L, d.halfL, d.invL);
    d.x[p] = nx;
    d.y[p] = ny;
    d.z[p] = nz;
    if (!(isfinite(nx) && isfinite(ny) && isfinite(nz))) atomicOr(d.err, 1);
}

// q_z run length of dir_beta: the largest divisor of H/2 up to 32 (runs must
// not straddle q_z = H/2 -> -H/2)
constexpr int dir_qz_of(int H) {
    int q = H / 2 < 32 ? H / 2 : 32;
    while ((H / 2) % q != 0) --q;
    return q;
}
int dir_qz(int H) { return dir_qz_of(H); }

// slices of the (kx, ky) pairs in the gradient sum: enough workgroups to fill
// the device when the particles alone do not
int dir_mode_slices(int H, int64_t P) {
    const int64_t pb = (P + DIR_THREADS - 1) / DIR_THREADS;
    int ms = 1;
    while (ms * pb < 2048 && ms * 2 * DIR_PAIRS <= H * H && ms < 64) ms *= 2;  // >= DIR_PAIRS pairs per slice
    return ms;
}

int dir_slices(int H, int64_t P) {
    const int64_t cols = (int64_t)H * H * (H / dir_qz(H));
    const int64_t bx = (cols + DIR_THREADS - 1) / DIR_THREADS;
    int64_t s = (2048 + bx - 1) / bx;
    s = std::min<int64_t>(s, (P + 63) / 64);
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, 1024));
}

template <typename T, int H>
static hipError_t dir_step_h(const DirDesc<T>& d, cplx_t<T>* part, int nslices, T* gpart, int ms, hipStream_t s) {
    constexpr int QZ = dir_qz_of(H);
    const int cols = H * H * (H / QZ);
    launch_kernel((k_dir_beta<T, H, QZ>), dim3((cols + DIR_THREADS - 1) / DIR_THREADS, nslices), dim3(DIR_THREADS), 0,
                  s, d, part);
    launch_kernel((k_dir_modes<T, H>), dim3((H * H * H + DIR_THREADS - 1) / DIR_THREADS), dim3(DIR_THREADS), 0, s, d,
                  (const cplx_t<T>*)part, nslices);
    const unsigned pb = (unsigned)((d.P + DIR_THREADS - 1) / DIR_THREADS);
    if (d.scheme == SIPF_STRANG) {
        launch_kernel((k_dir_grad<T, H, SIPF_STRANG>), dim3(pb, ms), dim3(DIR_THREADS), 0, s, d, gpart);
        launch_kernel((k_dir_push<T, SIPF_STRANG>), dim3(pb), dim3(DIR_THREADS), 0, s, d, (const T*)gpart, ms);
    } else {
        launch_kernel((k_dir_grad<T, H, SIPF_EM>), dim3(pb, ms), dim3(DIR_THREADS), 0, s, d, gpart);
        launch_kernel((k_dir_push<T, SIPF_EM>), dim3(pb), dim3(DIR_THREADS), 0, s, d, (const T*)gpart, ms);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_direct_step(const DirDesc<T>& d, cplx_t<T>* part, int nslices, T* gpart, int ms, hipStream_t s) {
    if (ms < 1 || ms > d.H * d.H) return hipErrorInvalidValue;
    switch (d.H) {
        case 8: return dir_step_h<T, 8>(d, part, nslices, gpart, ms, s);
        case 12: return dir_step_h<T, 12>(d, part, nslices, gpart, ms, s);
        case 16: return dir_step_h<T, 16>(d, part, nslices, gpart, ms, s);
        case 22: return dir_step_h<T, 22>(d, part, nslices, gpart, ms, s);
        case 32: return dir_step_h<T, 32>(d, part, nslices, gpart, ms, s);
        case 46: return dir_step_h<T, 46>(d, part, nslices, gpart, ms, s);
        case 64: return dir_step_h<T, 64>(d, part, nslices, gpart, ms, s);
        case 90:
            if constexpr (sizeof(T) == 4) return dir_step_h<T, 90>(d, part, nslices, gpart, ms, s);
            else return hipErrorInvalidValue;
        case 128:
            if constexpr (sizeof(T) == 4) return dir_step_h<T, 128>(d, part, nslices, gpart, ms, s);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_direct_step<float>(const DirDesc<float>&, cplx_t<float>*, int, float*, int, hipStream_t);
template hipError_t launch_direct_step<double>(const DirDesc<double>&, cplx_t<double>*, int, double*, int,
                                               hipStream_t);

}  // namespace sipf
