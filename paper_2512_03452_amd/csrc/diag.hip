// Run-time diagnostics of the numerical experiments (Sec. 5.2, 5.5): maximum
// and mass of the regularised density rho_hat * G0 on the grid, the share of
// the energy of c_hat in the modes |q| >= 4, the integral of c_hat, and the
// particle moments R_num = mean sqrt(x1^2 + x2^2) and m2 = mean |X|^2.
//
// Two deterministic passes: nb workgroups per instance (enough to stream the
// particles at full bandwidth) reduce strided slices of the grid, the half
// spectrum and the particles into per-block partials (FP64); one workgroup
// per instance then combines the partials with a fixed assignment of blocks
// to threads and a fixed tree.  The half spectrum stands for the full one: the
// planes kz = 0 and kz = H/2 hold every one of their modes once, the other
// planes hold one of each conjugate pair, which counts twice.

#include "internal.h"

namespace sipf {

constexpr int DIAG_THREADS = 256;

int diag_blocks(int64_t P, int64_t ng) {
    const int64_t work = std::max<int64_t>(P, ng);
    const int64_t nb = (work + DIAG_THREADS * 16 - 1) / (DIAG_THREADS * 16);
    return (int)std::min<int64_t>(std::max<int64_t>(nb, 1), DIAG_MAX_BLOCKS);
}

template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double (*red)[DIAG_THREADS], int tid) {
    for (int k = 0; k < NV; ++k) red[k][tid] = v[k];
    __syncthreads();
    for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) {
            for (int k = 0; k < NV; ++k) {
                if (k == 1) red[k][tid] = fmax(red[k][tid], red[k][tid + s]);
                else red[k][tid] += red[k][tid + s];
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(DIAG_THREADS) void k_diag_partials(const DiagDesc<T>* __restrict__ dd,
                                                                double* __restrict__ part) {
    const DiagDesc<T> d = dd[blockIdx.y];
    if ((int)blockIdx.x >= d.nb) return;
    const int tid = threadIdx.x;
    const int64_t stride = (int64_t)d.nb * DIAG_THREADS;
    const int64_t first = (int64_t)blockIdx.x * DIAG_THREADS + tid;
    const int H = d.H, HH = H / 2 + 1;
    double v[DIAG_NVAL];
    for (int k = 0; k < DIAG_NVAL; ++k) v[k] = 0.0;
    v[1] = -INFINITY;
    const bool two = d.dim == 2;
    const int64_t ng = two ? (int64_t)H * H : (int64_t)H * H * H;
    for (int64_t i = first; i < ng; i += stride) {
        const double r = (double)d.rho[i];
        v[0] += r;
        v[1] = fmax(v[1], r);
    }
    // frequency of a storage position along a permuted axis
    auto freq = [&](int pos) {
        const int r = pos % d.pm;
        return pos / d.pm + d.pt * (r / d.n2 + d.n1 * (r % d.n2));
    };
    const int64_t ns = two ? (int64_t)HH * H : (int64_t)H * H * HH;
    for (int64_t i = first; i < ns; i += stride) {
        int qx, qy, qz, kh;
        if (two) {
            kh = (int)(i / H);  // ky, the halved axis
            const int kx = freq((int)(i % H));
            qx = kx < H / 2 ? kx : kx - H;
            qy = kh;
            qz = 0;
        } else {
            kh = (int)(i % HH);  // kz, the halved axis
            const int64_t row = i / HH;
            const int kx = freq((int)(row / H)), ky = freq((int)(row % H));
            qx = kx < H / 2 ? kx : kx - H;
            qy = ky < H / 2 ? ky : ky - H;
            qz = kh;
        }
        const int q2 = qx * qx + qy * qy + qz * qz;
        const cplx_t<T> a = d.alpha[i];
        const double w = (kh == 0 || kh == H / 2) ? 1.0 : 2.0;
        const double e = w * ((double)a.x * (double)a.x + (double)a.y * (double)a.y);
        v[2] += e;
        if (q2 >= 16) v[3] += e;
        if (i == 0) v[4] = (double)a.x;
    }
    for (int64_t i = first; i < d.P; i += stride) {
        const double x = (double)d.x[i], y = (double)d.y[i], z = two ? 0.0 : (double)d.z[i];
        const double rxy2 = x * x + y * y;
        v[5] += sqrt(rxy2);
        v[6] += rxy2 + z * z;
    }
    __shared__ double red[DIAG_NVAL][DIAG_THREADS];
    block_reduce<DIAG_NVAL>(v, red, tid);
    if (tid < DIAG_NVAL) part[((size_t)blockIdx.y * DIAG_MAX_BLOCKS + blockIdx.x) * DIAG_NVAL + tid] = red[tid][0];
}

// one workgroup per instance: thread t combines blocks t, t + 256, ... in
// order, then a fixed tree over the threads
template <typename T>
__global__ __launch_bounds__(DIAG_THREADS) void k_diag_finish(const DiagDesc<T>* __restrict__ dd,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ out) {
    const int nb = dd[blockIdx.x].nb;
    const int tid = threadIdx.x;
    const double* p = part + (size_t)blockIdx.x * DIAG_MAX_BLOCKS * DIAG_NVAL;
    double v[DIAG_NVAL];
    for (int k = 0; k < DIAG_NVAL; ++k) v[k] = 0.0;
    v[1] = -INFINITY;
    for (int b = tid; b < nb; b += DIAG_THREADS) {
        for (int k = 0; k < DIAG_NVAL; ++k) {
            const double x = p[(size_t)b * DIAG_NVAL + k];
            v[k] = k == 1 ? fmax(v[k], x) : v[k] + x;
        }
    }
    __shared__ double red[DIAG_NVAL][DIAG_THREADS];
    block_reduce<DIAG_NVAL>(v, red, tid);
    if (tid < DIAG_NVAL) out[(size_t)blockIdx.x * DIAG_NVAL + tid] = red[tid][0];
}

template <typename T>
hipError_t launch_diag(const DiagDesc<T>* d, int n, int nbmax, double* part, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nbmax < 1 || nbmax > DIAG_MAX_BLOCKS) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_diag_partials<T>), dim3(nbmax, n), dim3(DIAG_THREADS), 0, s, d, part);
    hipLaunchKernelGGL((k_diag_finish<T>), dim3(n), dim3(DIAG_THREADS), 0, s, d, part, out);
    return hipGetLastError();
}

template hipError_t launch_diag<float>(const DiagDesc<float>*, int, int, double*, double*, hipStream_t);
template hipError_t launch_diag<double>(const DiagDesc<double>*, int, int, double*, double*, hipStream_t);

}  // namespace sipf
