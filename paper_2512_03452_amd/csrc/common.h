// Device-side building blocks of the SIPF-PIC step on gfx950: complex helpers,
// the Philox4x32-10 normal stream and the particle/grid stencil weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sipf {

// ---------------------------------------------------------------------------
// complex values: float2 / double2 (re, im)
// ---------------------------------------------------------------------------
template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename cplx<T>::type;

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
template <typename V, typename T> __device__ __forceinline__ V cscale(V a, T s) { a.x *= s; a.y *= s; return a; }
template <typename V, typename T> __device__ __forceinline__ V cmake(T re, T im) { V r; r.x = re; r.y = im; return r; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  A round maps the counter
// (c0,c1,c2,c3) under key (k0,k1) to
//   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// and the key is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u32x4 { uint32_t v0, v1, v2, v3; };

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.v0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.v2;
        u32x4 n;
        n.v0 = (uint32_t)(p1 >> 32) ^ c.v1 ^ k0;
        n.v1 = (uint32_t)p1;
        n.v2 = (uint32_t)(p0 >> 32) ^ c.v3 ^ k1;
        n.v3 = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform in [2^-24, 1 - 2^-24]: ((r >> 9) + 1/2) 2^-23, exact in float and double.
template <typename T> __device__ __forceinline__ T u01(uint32_t r) {
    return ((T)(r >> 9) + (T)0.5) * (T)1.1920928955078125e-07;  // 2^-23
}

// Box-Muller: (z0, z1) = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1),
//             z2       = sqrt(-2 ln u2) cos 2 pi u3.
// float: the hardware transcendentals (v_log_f32 is log2; v_sin/v_cos take
// revolutions, so cos 2 pi u is one instruction); u in [2^-24, 1) keeps every
// argument in range.
__device__ __forceinline__ void normals3(u32x4 r, float& z0, float& z1, float& z2) {
    const float u0 = u01<float>(r.v0), u1 = u01<float>(r.v1);
    const float u2 = u01<float>(r.v2), u3 = u01<float>(r.v3);
    constexpr float m2ln2 = -1.3862943611198906f;  // -2 ln 2
    const float a = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float b = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    z0 = a * __builtin_amdgcn_cosf(u1);
    z1 = a * __builtin_amdgcn_sinf(u1);
    z2 = b * __builtin_amdgcn_cosf(u3);
}
__device__ __forceinline__ void normals3(u32x4 r, double& z0, double& z1, double& z2) {
    const double u0 = u01<double>(r.v0), u1 = u01<double>(r.v1);
    const double u2 = u01<double>(r.v2), u3 = u01<double>(r.v3);
    const double a = sqrt(-2.0 * log(u0));
    const double b = sqrt(-2.0 * log(u2));
    double s1, c1;
    sincospi(2.0 * u1, &s1, &c1);
    z0 = a * c1;
    z1 = a * s1;
    z2 = b * cospi(2.0 * u3);
}

// Normal 3-vector of particle id at step n, slot, instance (key = seed).
template <typename T>
__device__ __forceinline__ void noise3(uint32_t id, uint32_t n, uint32_t slot, uint32_t inst,
                                       uint32_t k0, uint32_t k1, T& z0, T& z1, T& z2) {
    u32x4 c{id, n, slot, inst};
    normals3(philox4x32_10(c, k0, k1), z0, z1, z2);
}

// ---------------------------------------------------------------------------
// Stencil weights (Sec. 3.1).  Per axis, with l = lambda_s:
//   hat factors        w0 = 1 - l, w1 = l                      (eq. 2ord)
//   outer factors      wm = -(2 - l) l (1 - l) / 6  (node -1)
//                      wp = -(1 + l)(1 - l) l / 6   (node +2)  (eq. 4ord)
//   inner correction   S  = 1 + sum_s l_s (1 - l_s) / 2        (eq. 4ord)
// Inner node j in {0,1}^3:  prod_s w_{j_s} * S.
// Outer node on axis a:     w{m,p}(l_a) * prod_{s != a} w_{j_s}(l_s).
// ---------------------------------------------------------------------------
template <typename T> struct Axis4 {
    T w0, w1, wm, wp;
};
template <typename T> __device__ __forceinline__ Axis4<T> axis4(T l) {
    Axis4<T> a;
    const T om = (T)1 - l;
    const T lo = l * om;
    a.w0 = om;
    a.w1 = l;
    a.wm = -((T)2 - l) * lo * (T)(1.0 / 6.0);
    a.wp = -((T)1 + l) * lo * (T)(1.0 / 6.0);
    return a;
}

}  // namespace sipf
