// Device helpers shared by the particle passes of the forward step and of its
// adjoint: global-pointer casts, fixed-point window accumulators, small
// integer division, wave reductions and window geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sipf {

#define GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLOBAL T* gp(T* p) { return (GLOBAL T*)p; }
template <typename T> __device__ __forceinline__ const GLOBAL T* gp(const T* p) { return (const GLOBAL T*)p; }

__device__ __forceinline__ void gatomic_add(float* p, float v) { __builtin_amdgcn_global_atomic_fadd_f32(gp(p), v); }
__device__ __forceinline__ void gatomic_add(double* p, double v) { __builtin_amdgcn_global_atomic_fadd_f64(gp(p), v); }

template <typename T> __device__ __forceinline__ int ifloor(T v) { return (int)floor(v); }

// Fixed-point accumulator of the LDS deposit window.  Float atomic adds on
// LDS run ~25x slower than integer ones on gfx950, so weights are rounded to
// integers at a power-of-two scale 2^S chosen per work item so that no node
// sum can overflow, summed exactly with integer LDS atomics, and converted
// back once when the window is added to the grid.
template <typename T> struct Fixed;
template <> struct Fixed<float> {
    using I = int32_t;
    using U = uint32_t;
    static constexpr int BITS = 30;
    __device__ static I quant(float v) { return (I)rintf(v); }
};
template <> struct Fixed<double> {
    using I = long long;
    using U = unsigned long long;
    static constexpr int BITS = 62;
    __device__ static I quant(double v) { return (I)rint(v); }
};

// Exact round-to-nearest integer of |v| < 2^22 (float) or 2^51 (double): in
// v + 1.5 2^23 (resp. 1.5 2^52) the unit in the last place is 1, so the low
// mantissa bits of the sum hold round(v) offset by the magic constant.
template <typename T> struct Magic;
template <> struct Magic<float> {
    static constexpr float M = 12582912.0f;
    static constexpr int MAXS = 21;
    __device__ static int32_t take(float v) { return __float_as_int(v) - 0x4B400000; }
};
template <> struct Magic<double> {
    static constexpr double M = 6755399441055744.0;
    static constexpr int MAXS = 50;
    __device__ static long long take(double v) { return __double_as_longlong(v) - 0x4338000000000000LL; }
};

// floor(v + 1/2) as an integer in one instruction (|v| < 2^31).
__device__ __forceinline__ int round_half_up(float v) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// a * b + c for 0 <= a, b < 2^24 (24-bit multiply, full rate)
__device__ __forceinline__ int mad24(int a, int b, int c) { return (int)__umul24((unsigned)a, (unsigned)b) + c; }

// q = e / d, r = e % d for 0 <= e < 2^20, 0 < d < 2^10: float reciprocal
// estimate, corrected by one step.
__device__ __forceinline__ void divmod_small(int e, int d, float inv_d, int& q, int& r) {
    q = (int)((float)e * inv_d);
    r = e - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
}
// (i, j, k) of flat index e in a box of sizes (., ey, ez), row-major
__device__ __forceinline__ void unflatten3(int e, int ey, int ez, float inv_ez, float inv_ey, int& i, int& j, int& k) {
    int r;
    divmod_small(e, ez, inv_ez, r, k);
    divmod_small(r, ey, inv_ey, i, j);
}

template <typename T> __device__ __forceinline__ T wrap_box(T v, T L, T halfL, T invL) {
    return v - L * floor((v + halfL) * invL);
}

__device__ __forceinline__ int wave_min(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Window along one axis covering relative cells [lo, hi] of a chunk whose
// reference cell is r: origin and width, or the whole axis when it would wrap.
__device__ __forceinline__ void axis_window(int r, int lo, int hi, int H, int& o, int& W) {
    const int w = hi - lo + 1;
    if (w >= H) {
        o = 0;
        W = H;
    } else {
        o = (r + lo) & (H - 1);
        W = w;
    }
}

// Periodic grid index onto [0, H): a mask when H is a power of two, else the
// remainder, which holds for any int argument.
template <bool P2> struct Wrap {
    int H, m;  // m = H - 1
    __device__ __forceinline__ int operator()(int v) const {
        if constexpr (P2) {
            return v & m;
        } else {
            const int r = v % H;
            return r < 0 ? r + H : r;
        }
    }
};

// axis_window for any grid size
template <bool P2>
__device__ __forceinline__ void axis_window(int r, int lo, int hi, const Wrap<P2>& wr, int& o, int& W) {
    const int w = hi - lo + 1;
    if (w >= wr.H) {
        o = 0;
        W = wr.H;
    } else {
        o = wr(r + lo);
        W = w;
    }
}

// Work queue of the persistent item passes.  The item list's header holds the
// item count n (hdr[0], written by the sort) and a ticket counter (hdr[1],
// zero between launches).  Workgroup b takes item b first; with more items
// than workgroups it then draws tickets t for item grid + t, in list order,
// until a draw is past the end, so items of uneven cost spread over the
// workgroups that free up first.  Each workgroup's last draw is that failing
// one, hence a launch draws exactly n tickets and the draw that returns n - 1
// is its last: it puts the counter back to zero.  Launches that share a
// header must not overlap (they run on one stream).  Call with the whole
// workgroup after an item; returns the next item (>= n: none).
__device__ __forceinline__ int next_item(int* hdr, int n, int* slot) {
    const int grid = (int)gridDim.x;
    if (n <= grid) return n;
    __syncthreads();  // the item's use of LDS has ended
    if (threadIdx.x == 0) {
        const int t = atomicAdd(hdr + 1, 1);
        if (t == n - 1) atomicExch(hdr + 1, 0);
        *slot = grid + t;
    }
    __syncthreads();
    return *slot;
}

}  // namespace sipf
