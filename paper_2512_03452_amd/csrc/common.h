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
        // three-input XOR in one gfx950 v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        n.v0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.v1, k0, 0x96);
        n.v1 = (uint32_t)p1;
        n.v2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.v3, k1, 0x96);
        n.v3 = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// One Philox call gives six 21-bit fields (126 of its 128 bits):
//   f_i = r_i >> 11 (i < 4), f_4 = (r0 & 0x7FF) << 10 | (r1 & 0x3FF),
//   f_5 = (r2 & 0x7FF) << 10 | (r3 & 0x3FF),
// uniforms u = (f + 1/2) 2^-21 in [2^-22, 1 - 2^-22] (exact in float), and
// three Box-Muller pairs (z_2j, z_2j+1) = sqrt(-2 ln u_2j) (cos, sin)(2 pi u_2j+1).
// NPAIR = 3 gives all six normals, NPAIR = 2 the first four.
template <typename T> __device__ __forceinline__ T u01_21(uint32_t f) {
    return ((T)f + (T)0.5) * (T)4.76837158203125e-07;  // 2^-21
}
__device__ __forceinline__ void fields21(u32x4 r, uint32_t f[6]) {
    f[0] = r.v0 >> 11;
    f[1] = r.v1 >> 11;
    f[2] = r.v2 >> 11;
    f[3] = r.v3 >> 11;
    f[4] = ((r.v0 & 0x7FFu) << 10) | (r.v1 & 0x3FFu);
    f[5] = ((r.v2 & 0x7FFu) << 10) | (r.v3 & 0x3FFu);
}
// float: u = (f + 1/2) 2^-21 is formed from bits as the float 1 + (f + 1/2)
// 2^-21 (mantissa 4 f + 2) minus 1, both steps exact, so it equals
// u01_21<float>(f) without an integer-to-float conversion.  The hardware
// transcendentals follow (v_log_f32 is log2; v_sin/v_cos take revolutions,
// so cos 2 pi u is one instruction); u in [2^-22, 1) keeps every argument in
// range.
__device__ __forceinline__ float u01_21_bits(uint32_t mant) { return __uint_as_float(0x3F800000u | mant) - 1.0f; }
template <int NPAIR> __device__ __forceinline__ void normals6(u32x4 r, float z[6]) {
    // mantissas 4 f_i + 2 of the six fields (see fields21)
    uint32_t m[6];
    m[0] = ((r.v0 >> 9) & 0x7FFFFCu) | 2u;
    m[1] = ((r.v1 >> 9) & 0x7FFFFCu) | 2u;
    m[2] = ((r.v2 >> 9) & 0x7FFFFCu) | 2u;
    m[3] = ((r.v3 >> 9) & 0x7FFFFCu) | 2u;
    m[4] = ((r.v0 << 12) & 0x7FF000u) | ((r.v1 << 2) & 0xFFCu) | 2u;
    m[5] = ((r.v2 << 12) & 0x7FF000u) | ((r.v3 << 2) & 0xFFCu) | 2u;
    constexpr float m2ln2 = -1.3862943611198906f;  // -2 ln 2
#pragma unroll
    for (int j = 0; j < NPAIR; ++j) {
        const float a = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u01_21_bits(m[2 * j])));
        const float b = u01_21_bits(m[2 * j + 1]);
        z[2 * j] = a * __builtin_amdgcn_cosf(b);
        z[2 * j + 1] = a * __builtin_amdgcn_sinf(b);
    }
}
template <int NPAIR> __device__ __forceinline__ void normals6(u32x4 r, double z[6]) {
    uint32_t f[6];
    fields21(r, f);
#pragma unroll
    for (int j = 0; j < NPAIR; ++j) {
        const double a = sqrt(-2.0 * log(u01_21<double>(f[2 * j])));
        double s, c;
        sincospi(2.0 * u01_21<double>(f[2 * j + 1]), &s, &c);
        z[2 * j] = a * c;
        z[2 * j + 1] = a * s;
    }
}

// The normals of particle id at step n (counter (id, n, 0, instance), key =
// seed): split step W^- from z[0..2] and W^+ from z[3..5]; Euler-Maruyama W
// from z[0..2] (NPAIR = 2).
template <int NPAIR, typename T>
__device__ __forceinline__ void noise6(uint32_t id, uint32_t n, uint32_t inst, uint32_t k0, uint32_t k1, T z[6]) {
    u32x4 c{id, n, 0u, inst};
    normals6<NPAIR>(philox4x32_10(c, k0, k1), z);
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
