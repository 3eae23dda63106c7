// Positivity-preserving deposit: the smoothing near the edge of the particle
// cloud that Remark `smoothness` (Sec. 3.1) calls for so that the operator-
// splitting update of Sec. 3.4 keeps the concentration non-negative.  The paper
// cites the procedure without giving it; the one built here:
//
//   After the order-4 deposit (the particle pass), rounds of
//     flag    node j is flagged when phi_j < -thresh;
//     switch  every particle still on order 4 whose 32 stencil nodes include
//             a flagged node moves to the order-2 weights of eq. 2ord: it adds
//             (F2 - F4) w to its nodes (-w W (S - 1) on the 8 inner nodes,
//             -w F_outer on the 24 outer ones) and records the round's tag;
//   until a round switches nobody; then clamp phi_j <- max(phi_j, 0).
//
// Both weight sets sum to one, so every switch conserves the mass.  In exact
// arithmetic the rounds alone leave no negative node (a negative node keeps an
// order-4 contributor with a negative weight until it switches); the clamp
// removes what the fixed-point windows' rounding leaves behind.  thresh sits
// at the rounding of one contribution: a node further below zero is either
// truly negative or rounding of switched particles alone, which switches
// nobody.  The flag grid is rebuilt before each switch pass, so the decisions
// of one round do not depend on the order of its atomics.
//
// A particle in cell c touches nodes in c + {-1..2}^3 only, so before each
// switch pass the flags are dilated over that box (three separable passes of
// four reads) into a per-cell byte; a particle whose cell byte is clear stops
// after that one read, the others check their 32 nodes exactly.
#include "internal.h"
#include "pass_common.h"

namespace sipf {

constexpr int POS_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(POS_THREADS) void k_pos_flag(const T* __restrict__ phi, int64_t n, T thresh,
                                                          uint8_t* __restrict__ flag) {
    for (int64_t j = (int64_t)blockIdx.x * POS_THREADS + threadIdx.x; j < n; j += (int64_t)gridDim.x * POS_THREADS)
        flag[j] = phi[j] < -thresh ? 1 : 0;
}

// out[c] = OR over t = -1..2 of in[c + t e_axis] (periodic)
template <bool P2>
__global__ __launch_bounds__(POS_THREADS) void k_pos_dilate(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                            int H, int axis) {
    const Wrap<P2> wr{H, H - 1};
    const int n = H * H * H;  // H <= 256: fits int
    const int stride = axis == 0 ? H * H : (axis == 1 ? H : 1);
    for (int j = blockIdx.x * POS_THREADS + threadIdx.x; j < n; j += gridDim.x * POS_THREADS) {
        const int c = (j / stride) % H;  // coordinate along the axis
        const int base = j - c * stride;
        uint8_t v = 0;
#pragma unroll
        for (int t = -1; t <= 2; ++t) v |= in[base + wr(c + t) * stride];
        out[j] = v;
    }
}

template <typename T, bool P2>
__global__ __launch_bounds__(POS_THREADS) void k_pos_switch(const PartDesc<T>* __restrict__ pd,
                                                            const uint8_t* __restrict__ flag,
                                                            const uint8_t* __restrict__ touch, uint32_t* __restrict__ sw,
                                                            uint32_t tag, int* __restrict__ count) {
    const PartDesc<T>& a = *pd;
    const int64_t i = (int64_t)blockIdx.x * POS_THREADS + threadIdx.x;
    if (i >= a.P) return;
    const int H = a.H;
    const Wrap<P2> wr{H, H - 1};
    const T sx = a.x[i] * a.hl, sy = a.y[i] * a.hl, sz = a.z[i] * a.hl;
    const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
    const int gx = (int)fx, gy = (int)fy, gz = (int)fz;
    if (!touch[((size_t)wr(gx) * H + wr(gy)) * H + wr(gz)] || sw[i] == tag) return;
    int ix[4], iy[4], iz[4];  // nodes g - 1 .. g + 2 along each axis
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        ix[j] = wr(gx - 1 + j);
        iy[j] = wr(gy - 1 + j);
        iz[j] = wr(gz - 1 + j);
    }
    auto node = [&](int a1, int b1, int c1) { return ((size_t)ix[a1] * H + iy[b1]) * H + iz[c1]; };
    bool hit = false;
#pragma unroll
    for (int p = 1; p <= 2; ++p)
#pragma unroll
        for (int q = 1; q <= 2; ++q) {
            hit |= flag[node(p, q, 1)] | flag[node(p, q, 2)];                  // inner
            hit |= flag[node(0, p, q)] | flag[node(3, p, q)];                  // outer on x
            hit |= flag[node(p, 0, q)] | flag[node(p, 3, q)];                  // outer on y
            hit |= flag[node(p, q, 0)] | flag[node(p, q, 3)];                  // outer on z
        }
    if (!hit) return;
    sw[i] = tag;
    atomicAdd(count, 1);
    const Axis4<T> ax = axis4(sx - fx), ay = axis4(sy - fy), az = axis4(sz - fz);
    const T S1 = (ax.w0 * ax.w1 + ay.w0 * ay.w1 + az.w0 * az.w1) * (T)0.5;  // S - 1
    const T m = -a.wmass;
    const T wx[2] = {ax.w0, ax.w1}, wy[2] = {ay.w0, ay.w1}, wz[2] = {az.w0, az.w1};
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const T pyz = wy[p] * wz[q], pxz = wx[p] * wz[q], pxy = wx[p] * wy[q];
            gatomic_add(a.phi + node(1, 1 + p, 1 + q), m * wx[0] * pyz * S1);
            gatomic_add(a.phi + node(2, 1 + p, 1 + q), m * wx[1] * pyz * S1);
            gatomic_add(a.phi + node(0, 1 + p, 1 + q), m * ax.wm * pyz);
            gatomic_add(a.phi + node(3, 1 + p, 1 + q), m * ax.wp * pyz);
            gatomic_add(a.phi + node(1 + p, 0, 1 + q), m * ay.wm * pxz);
            gatomic_add(a.phi + node(1 + p, 3, 1 + q), m * ay.wp * pxz);
            gatomic_add(a.phi + node(1 + p, 1 + q, 0), m * az.wm * pxy);
            gatomic_add(a.phi + node(1 + p, 1 + q, 3), m * az.wp * pxy);
        }
}

template <typename T>
__global__ __launch_bounds__(POS_THREADS) void k_pos_clamp(T* __restrict__ phi, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * POS_THREADS + threadIdx.x; j < n; j += (int64_t)gridDim.x * POS_THREADS)
        if (phi[j] < (T)0) phi[j] = (T)0;
}

static int grid_blocks(int64_t n) {
    const int64_t b = (n + POS_THREADS - 1) / POS_THREADS;
    return (int)(b < 4096 ? b : 4096);
}

template <typename T> hipError_t launch_pos_flag(const T* phi, int64_t n, T thresh, uint8_t* flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pos_flag<T>), dim3(grid_blocks(n)), dim3(POS_THREADS), 0, s, phi, n, thresh, flag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pos_switch(const PartDesc<T>* pd, int64_t P, int H, const uint8_t* flag, uint8_t* tmp,
                             uint8_t* touch, uint32_t* sw, uint32_t tag, int* count, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    const bool p2 = (H & (H - 1)) == 0;
    const int nb = grid_blocks((int64_t)H * H * H);
    const unsigned pb = (unsigned)((P + POS_THREADS - 1) / POS_THREADS);
    if (p2) {
        hipLaunchKernelGGL((k_pos_dilate<true>), dim3(nb), dim3(POS_THREADS), 0, s, flag, touch, H, 0);
        hipLaunchKernelGGL((k_pos_dilate<true>), dim3(nb), dim3(POS_THREADS), 0, s, touch, tmp, H, 1);
        hipLaunchKernelGGL((k_pos_dilate<true>), dim3(nb), dim3(POS_THREADS), 0, s, tmp, touch, H, 2);
        hipLaunchKernelGGL((k_pos_switch<T, true>), dim3(pb), dim3(POS_THREADS), 0, s, pd, flag, touch, sw, tag, count);
    } else {
        hipLaunchKernelGGL((k_pos_dilate<false>), dim3(nb), dim3(POS_THREADS), 0, s, flag, touch, H, 0);
        hipLaunchKernelGGL((k_pos_dilate<false>), dim3(nb), dim3(POS_THREADS), 0, s, touch, tmp, H, 1);
        hipLaunchKernelGGL((k_pos_dilate<false>), dim3(nb), dim3(POS_THREADS), 0, s, tmp, touch, H, 2);
        hipLaunchKernelGGL((k_pos_switch<T, false>), dim3(pb), dim3(POS_THREADS), 0, s, pd, flag, touch, sw, tag,
                           count);
    }
    return hipGetLastError();
}

template <typename T> hipError_t launch_pos_clamp(T* phi, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pos_clamp<T>), dim3(grid_blocks(n)), dim3(POS_THREADS), 0, s, phi, n);
    return hipGetLastError();
}

#define SIPF_POS_INST(T)                                                                                     \
    template hipError_t launch_pos_flag<T>(const T*, int64_t, T, uint8_t*, hipStream_t);                     \
    template hipError_t launch_pos_switch<T>(const PartDesc<T>*, int64_t, int, const uint8_t*, uint8_t*,    \
                                             uint8_t*, uint32_t*, uint32_t, int*, hipStream_t);              \
    template hipError_t launch_pos_clamp<T>(T*, int64_t, hipStream_t);

SIPF_POS_INST(float)
SIPF_POS_INST(double)

}  // namespace sipf
