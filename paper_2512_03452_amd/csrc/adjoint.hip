// Reverse-mode kernels of the SIPF-PIC step along a fixed noise path.
//
// Forward step n (Algorithm 4, split form):
//   Y = X + s Z-,  v = I*G(Y),  X' = wrap(Y + chi tau v + s Z+),
// with G the filtered gradient grids of alpha^(n-1) and phi = I(X) the deposit.
// Reverse, with Xbar' the cotangent of X' (floor() locally constant, wrap = id):
//   chibar += tau Xbar'.v,   vbar = chi tau Xbar',   Ybar = Xbar' + J^T vbar,
//   sbar   += Xbar'.Z+ + Ybar.Z-,   Gbar += I(vbar at Y)   (transpose of I*,
//   the adjoint relation <I rho, f> = <rho, I* f> of Sec. 3.1),
//   Xbar   = Ybar + (M0/P)(H/L) sum_gamma phibar[g + gamma] dF_gamma/dlambda.
// Euler-Maruyama (eq. rho_hat_update): Y = X, sbar += Xbar'.Z.
// Cotangents of positions are stored by original particle id.
#include "internal.h"
#include "sipf.h"

namespace sipf {

#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ void adj_atomic_add(float* p, float v) {
    __builtin_amdgcn_global_atomic_fadd_f32((GLOBAL float*)p, v);
}
__device__ __forceinline__ void adj_atomic_add(double* p, double v) {
    __builtin_amdgcn_global_atomic_fadd_f64((GLOBAL double*)p, v);
}

// sum over the 32 nodes of Gamma_4 of phibar[node] * dF/dlambda (eq. 4ord)
template <typename T>
__device__ __forceinline__ void deposit_grad(const T* __restrict__ phibar, T x, T y, T z, T hl, int H, T& gx_, T& gy_,
                                             T& gz_) {
    const int Hm = H - 1;
    const T s[3] = {x * hl, y * hl, z * hl};
    int g[3];
    T F[3][4], D[3][4], dS[3], S = (T)1;
    for (int a = 0; a < 3; ++a) {
        const T f = floor(s[a]);
        g[a] = (int)f;
        const T l = s[a] - f;
        const T om = (T)1 - l;
        const T lo = l * om;
        F[a][0] = -((T)2 - l) * lo * (T)(1.0 / 6.0);
        F[a][1] = om;
        F[a][2] = l;
        F[a][3] = -((T)1 + l) * lo * (T)(1.0 / 6.0);
        D[a][0] = -((T)2 - (T)6 * l + (T)3 * l * l) * (T)(1.0 / 6.0);
        D[a][1] = (T)-1;
        D[a][2] = (T)1;
        D[a][3] = -((T)1 - (T)3 * l * l) * (T)(1.0 / 6.0);
        S += lo * (T)0.5;
        dS[a] = ((T)1 - (T)2 * l) * (T)0.5;
    }
    auto node = [&](int i, int j, int k) -> T {
        const int ix = (g[0] - 1 + i) & Hm, iy = (g[1] - 1 + j) & Hm, iz = (g[2] - 1 + k) & Hm;
        return phibar[((size_t)ix * H + iy) * H + iz];
    };
    T ax = 0, ay = 0, az = 0;
    // inner nodes: F = X Y Z S
    for (int i = 1; i <= 2; ++i)
        for (int j = 1; j <= 2; ++j)
            for (int k = 1; k <= 2; ++k) {
                const T p = node(i, j, k);
                const T xyz = F[0][i] * F[1][j] * F[2][k];
                ax += p * (D[0][i] * F[1][j] * F[2][k] * S + xyz * dS[0]);
                ay += p * (F[0][i] * D[1][j] * F[2][k] * S + xyz * dS[1]);
                az += p * (F[0][i] * F[1][j] * D[2][k] * S + xyz * dS[2]);
            }
    // outer nodes: F = X Y Z with one index in {0, 3}
    for (int o = 0; o < 2; ++o) {
        const int e = o ? 3 : 0;
        for (int u = 1; u <= 2; ++u)
            for (int v = 1; v <= 2; ++v) {
                {  // outer on x: (e, u, v)
                    const T p = node(e, u, v);
                    ax += p * D[0][e] * F[1][u] * F[2][v];
                    ay += p * F[0][e] * D[1][u] * F[2][v];
                    az += p * F[0][e] * F[1][u] * D[2][v];
                }
                {  // outer on y: (u, e, v)
                    const T p = node(u, e, v);
                    ax += p * D[0][u] * F[1][e] * F[2][v];
                    ay += p * F[0][u] * D[1][e] * F[2][v];
                    az += p * F[0][u] * F[1][e] * D[2][v];
                }
                {  // outer on z: (u, v, e)
                    const T p = node(u, v, e);
                    ax += p * D[0][u] * F[1][v] * F[2][e];
                    ay += p * F[0][u] * D[1][v] * F[2][e];
                    az += p * F[0][u] * F[1][v] * D[2][e];
                }
            }
    }
    gx_ = ax;
    gy_ = ay;
    gz_ = az;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_seed(AdjDesc<T> a) {
    const T c = a.wmass * a.hl;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.P; i += (int64_t)gridDim.x * blockDim.x) {
        T gx, gy, gz;
        deposit_grad(a.phibar, a.x[i], a.y[i], a.z[i], a.hl, a.H, gx, gy, gz);
        const size_t p = a.id[i];
        a.xbar[3 * p] = c * gx;
        a.xbar[3 * p + 1] = c * gy;
        a.xbar[3 * p + 2] = c * gz;
    }
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

template <typename T, int SCHEME>
__global__ __launch_bounds__(256) void k_adj_step(AdjDesc<T> a) {
    __shared__ double sh[8];
    const int H = a.H, Hm = H - 1;
    const size_t H3 = (size_t)H * H * H;
    const T hl = a.hl;
    double chib = 0, sb = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.P; i += (int64_t)gridDim.x * blockDim.x) {
        const T X[3] = {a.x[i], a.y[i], a.z[i]};
        const uint32_t pid = a.id[i];
        T zm[3], zp[3], Y[3];
        if (SCHEME == SIPF_STRANG) {
            noise3<T>(pid, a.n, 0u, a.inst, a.k0, a.k1, zm[0], zm[1], zm[2]);
            noise3<T>(pid, a.n, 1u, a.inst, a.k0, a.k1, zp[0], zp[1], zp[2]);
            for (int d = 0; d < 3; ++d) Y[d] = X[d] + a.s * zm[d];
        } else {
            noise3<T>(pid, a.n, 0u, a.inst, a.k0, a.k1, zp[0], zp[1], zp[2]);
            for (int d = 0; d < 3; ++d) {
                zm[d] = 0;
                Y[d] = X[d];
            }
        }
        // trilinear value and Jacobian at Y
        int gi[3][2];
        T w[3][2], dw[3][2];
        for (int d = 0; d < 3; ++d) {
            const T sv = Y[d] * hl;
            const T f = floor(sv);
            const int g = (int)f;
            const T l = sv - f;
            gi[d][0] = g & Hm;
            gi[d][1] = (g + 1) & Hm;
            w[d][0] = (T)1 - l;
            w[d][1] = l;
            dw[d][0] = -hl;
            dw[d][1] = hl;
        }
        T v[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        size_t idx[8];
        T wt[8];
        int q = 0;
        for (int ia = 0; ia < 2; ++ia)
            for (int ib = 0; ib < 2; ++ib)
                for (int ic = 0; ic < 2; ++ic, ++q) {
                    idx[q] = ((size_t)gi[0][ia] * H + gi[1][ib]) * H + gi[2][ic];
                    wt[q] = w[0][ia] * w[1][ib] * w[2][ic];
                    const T dx = dw[0][ia] * w[1][ib] * w[2][ic];
                    const T dy = w[0][ia] * dw[1][ib] * w[2][ic];
                    const T dz = w[0][ia] * w[1][ib] * dw[2][ic];
                    for (int d = 0; d < 3; ++d) {
                        const T gv = a.G[d * H3 + idx[q]];
                        v[d] += wt[q] * gv;
                        J[d][0] += dx * gv;
                        J[d][1] += dy * gv;
                        J[d][2] += dz * gv;
                    }
                }
        T xb[3];
        for (int d = 0; d < 3; ++d) xb[d] = a.xbar[3 * (size_t)pid + d];
        chib += (double)(a.tau * (xb[0] * v[0] + xb[1] * v[1] + xb[2] * v[2]));
        T vb[3], yb[3];
        for (int d = 0; d < 3; ++d) vb[d] = a.chitau * xb[d];
        for (int e = 0; e < 3; ++e) yb[e] = xb[e] + vb[0] * J[0][e] + vb[1] * J[1][e] + vb[2] * J[2][e];
        if (SCHEME == SIPF_STRANG)
            sb += (double)(xb[0] * zp[0] + xb[1] * zp[1] + xb[2] * zp[2] + yb[0] * zm[0] + yb[1] * zm[1] +
                           yb[2] * zm[2]);
        else
            sb += (double)(xb[0] * zp[0] + xb[1] * zp[1] + xb[2] * zp[2]);
        // transpose of the gather: scatter vbar with the trilinear weights at Y
        for (int k = 0; k < 8; ++k)
            for (int d = 0; d < 3; ++d) adj_atomic_add(a.Gbar + d * H3 + idx[k], wt[k] * vb[d]);
        // transpose of the deposit at X
        if (a.phibar != nullptr) {
            T gx, gy, gz;
            deposit_grad(a.phibar, X[0], X[1], X[2], hl, H, gx, gy, gz);
            const T c = a.wmass * hl;
            yb[0] += c * gx;
            yb[1] += c * gy;
            yb[2] += c * gz;
        }
        for (int d = 0; d < 3; ++d) a.xbar[3 * (size_t)pid + d] = yb[d];
    }
    const double tc = block_sum(chib, sh);
    const double ts = block_sum(sb, sh);
    if (threadIdx.x == 0) {
        atomicAdd(a.acc, tc);
        atomicAdd(a.acc + 1, ts);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* __restrict__ u, const T* __restrict__ v, int64_t n, double* out) {
    __shared__ double sh[8];
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += (double)u[i] * (double)v[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(out, t);
}

template <typename T> __global__ void k_axpby(T* y, const T* x, T a, T b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }
__global__ void k_zero_f64(double* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

static int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <typename T> hipError_t launch_adj_seed(const AdjDesc<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_seed<T>), dim3(grid_for(a.P)), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_adj_step(const AdjDesc<T>& a, hipStream_t s) {
    if (a.scheme == SIPF_STRANG)
        hipLaunchKernelGGL((k_adj_step<T, SIPF_STRANG>), dim3(grid_for(a.P)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_adj_step<T, SIPF_EM>), dim3(grid_for(a.P)), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_dot(const T* u, const T* v, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(grid_for(n)), dim3(256), 0, s, u, v, n, out);
    return hipGetLastError();
}
template <typename T> hipError_t launch_axpby(T* y, const T* x, T a, T b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n)), dim3(256), 0, s, y, x, a, b, n);
    return hipGetLastError();
}
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}
hipError_t launch_zero_f64(double* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

#define SIPF_ADJ_INST(T)                                                                \
    template hipError_t launch_adj_seed<T>(const AdjDesc<T>&, hipStream_t);            \
    template hipError_t launch_adj_step<T>(const AdjDesc<T>&, hipStream_t);            \
    template hipError_t launch_dot<T>(const T*, const T*, int64_t, double*, hipStream_t); \
    template hipError_t launch_axpby<T>(T*, const T*, T, T, int64_t, hipStream_t);
SIPF_ADJ_INST(float)
SIPF_ADJ_INST(double)

}  // namespace sipf
