// Particle pass of the SIPF-PIC step: binning, the fourth-order deposit
// (Definition particle2grid, Algorithm 2), the trilinear gather of the
// gradient (Definition grid2particle, Algorithm 3) and the stochastic push
// (Algorithm 4 split step / eq. rho_hat_update), in one launch per step.
//
// Particles are kept approximately sorted by tile (T^3 cells, tiles in Morton
// order) by a periodic counting sort.  A workgroup takes a contiguous chunk of
// the sorted array (a work item), measures the bounding box of the chunk's
// cells, and, when the box plus the stencil reach (-1..+2) fits, accumulates
// the deposit in an LDS window in fixed point with integer LDS atomics, then
// adds the window into the global grid once.  A chunk whose box does not fit
// (sparse regions, long drift since the last sort) deposits straight into the
// global grid with atomics; the result is the same sum in a different order.
// Two forms of the FP32 pass: the two-phase one (deposit all of an item's
// particles, then stage the gradient window and push them) and the sorted one
// (each item kept sorted by cell between steps, runs of equal cells summed in
// registers before the LDS adds, deposit and push in one loop).  The sort also
// serves the two-dimensional pass (particles2d.hip): tiles of T^2 cells.
#include <climits>

#include "internal.h"
#include "pass_common.h"
#include "sipf.h"

namespace sipf {

constexpr int PT = 512;            // threads per particle-pass workgroup
constexpr int PPT = 8;             // particles held in registers per thread
constexpr int CH = PT * PPT;       // particles per work item at most
#ifndef SIPF_SORT_THREADS
#define SIPF_SORT_THREADS 512
#endif
#ifndef SIPF_SORT_PER_THREAD
#define SIPF_SORT_PER_THREAD 8
#endif
constexpr int SORT_THREADS = SIPF_SORT_THREADS;  // threads per sort workgroup
constexpr int SORT_PER_THREAD = SIPF_SORT_PER_THREAD;
constexpr int SORT_CHUNK = SORT_THREADS * SORT_PER_THREAD;
constexpr int MAX_KEYS = 4096;     // (H / tile)^3 <= 16^3, (H / tile)^2 <= 64^2
constexpr int MIN_WINDOW_ITEM = 64;  // smaller items deposit and gather straight from global memory

// Push phase: re-read each particle (1) or keep the item's particles in
// registers from the load phase (0); unroll factor of the push loop.
#ifndef SIPF_RELOAD
#define SIPF_RELOAD 1
#endif
#ifndef SIPF_PUSH_UNROLL
#define SIPF_PUSH_UNROLL 8
#endif
// Minimum waves per SIMD the register allocation of the two-phase passes
// (FP64 steps, and the deposit-only and push-only passes of both precisions)
// must leave room for; 0 leaves it to the compiler.  A budget of six waves
// spilled 50-105 VGPRs in FP64: on the adjoint workload (P = 2e6, H = 64, 100
// steps) the compiler's choice took the FP64 forward from 27.1 to 22.8 ms and
// forward + adjoint from 87.5 to 73.5 ms (a budget of four: 24.8 and 76.2 ms);
// FP32 forward + adjoint 36.9 -> 36.5 ms.
#ifndef SIPF_PART_WAVES
#define SIPF_PART_WAVES 0
#endif
#if SIPF_PART_WAVES > 0
#define SIPF_PART_ATTR __attribute__((amdgpu_waves_per_eu(SIPF_PART_WAVES)))
#else
#define SIPF_PART_ATTR
#endif

int particle_threads() { return PT; }
int particle_chunk() { return CH; }
int sort_max_keys() { return MAX_KEYS; }

// Bit b of v (< 32) moved to bit 3b: three shift-or-mask steps that move
// groups of bits apart by 8, 4 and 2 places.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 31u;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    return (v | (v << 2)) & 0x09249249u;
}

// Bit b of v (< 64) moved to bit 2b.
__device__ __forceinline__ uint32_t spread2(uint32_t v) {
    v &= 63u;
    v = (v | (v << 4)) & 0x0F0Fu;
    v = (v | (v << 2)) & 0x3333u;
    return (v | (v << 1)) & 0x5555u;
}

// Tile coordinate of position v along one axis: a shift when H and the tile
// side are powers of two (tshift >= 0), else a division by the tile side (the
// last tile of the axis may then be partial).
template <typename T>
__device__ __forceinline__ uint32_t tile_coord(const PartDesc<T>& a, T v) {
    const int g = ifloor(v * a.hl);
    if (a.tshift >= 0) return (uint32_t)(g & (a.H - 1)) >> a.tshift;
    int c = g % a.H;
    if (c < 0) c += a.H;
    return (uint32_t)(c / a.tile);
}
// Morton key of a tile (up to 32 tiles per axis in 3-D, 64 in 2-D)
template <int DIM> __device__ __forceinline__ uint32_t key_of_tile(uint32_t tx, uint32_t ty, uint32_t tz) {
    if constexpr (DIM == 3) return (spread3(tx) << 2) | (spread3(ty) << 1) | spread3(tz);
    else return (spread2(tx) << 1) | spread2(ty);
}
// Morton key of the tile of the cell containing (x, y, z)
template <typename T, int DIM>
__device__ __forceinline__ uint32_t key_of(const PartDesc<T>& a, T x, T y, T z) {
    return key_of_tile<DIM>(tile_coord(a, x), tile_coord(a, y), DIM == 3 ? tile_coord(a, z) : 0u);
}
// Tiles per axis of an instance's sort grid
template <typename T> __device__ __forceinline__ int tiles_per_axis(const PartDesc<T>& a) {
    return a.tshift >= 0 ? (a.H >> a.tshift) : (a.H + a.tile - 1) / a.tile;
}

// Runs of equal keys in consecutive lanes of a wave (call with the whole
// wave).  Returns the run's length at its first lane and 0 at the others;
// head receives the first lane of the caller's run.  The particles are in
// tile order from the previous sort and mostly still in their tiles, so a
// wave's 64 keys form one or a few runs: one LDS atomic per run instead of
// per particle (atomics of a wave on one LDS word serialise).
__device__ __forceinline__ uint32_t lane_runs(uint32_t key, int& head) {
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool first = lane == 0 || prev != key;
    const uint64_t heads = __ballot(first);
    head = 63 - __clzll((long long)(heads & ((2ull << lane) - 1ull)));  // bit 0 is always set
    if (!first) return 0u;
    const uint64_t after = lane == 63 ? 0ull : heads >> (lane + 1);
    return after ? (uint32_t)__builtin_ctzll(after) + 1u : (uint32_t)(64 - lane);
}

// Tile counts of the next sort, taken by the 3-D particle pass of the step
// before it, so that the sort needs no histogram pass of its own.  A work
// item's particles shared one tile at the last sort and move less than a
// tile per step, so the item sums its pushed particles' tiles in LDS slots
// for the 5^3 tiles within two of a reference tile (that of the item's first
// particle before the push), one LDS add per run of equal tiles in
// consecutive lanes, and adds the nonzero slots to the counts once per item;
// a particle whose tile lies farther away (or every particle, on grids of
// fewer than 5 tiles per axis) adds to the counts directly.
// The slot and reference accesses go through LDS-address-space pointers: the
// generic pointers of the struct let the compiler merge the LDS and the
// global adds into one flat atomic, which the barrier that follows did not
// wait for (counts were lost).
constexpr int TC_SLOTS = 125;
#define LDS_AS __attribute__((address_space(3)))
struct TileCount {
    uint32_t* counts;  // the item's instance's counts (MAX_KEYS words), null when not counting
    uint32_t* slot;    // LDS, TC_SLOTS words, zero between items
    int* ref;          // LDS, the item's reference tile (3 words)
    __device__ __forceinline__ LDS_AS uint32_t* lslot() const { return (LDS_AS uint32_t*)slot; }
    __device__ __forceinline__ LDS_AS int* lref() const { return (LDS_AS int*)ref; }
};

// Thread 0: the reference tile of the item, from its first particle (read by
// the item's threads after the next barrier).
template <typename T>
__device__ __forceinline__ void tc_reference(const TileCount& tc, const PartDesc<T>& a, T x, T y, T z) {
    if (tc.counts != nullptr && threadIdx.x == 0) {
        LDS_AS int* r = tc.lref();
        r[0] = (int)tile_coord(a, x);
        r[1] = (int)tile_coord(a, y);
        r[2] = (int)tile_coord(a, z);
    }
}

// Slot of tile t relative to the reference (or -1 when it lies farther than
// two tiles on an axis, or the grid has fewer than 5 tiles per axis).
__device__ __forceinline__ int tc_slot(const LDS_AS int* r, const uint32_t t[3], int nt) {
    bool near = nt >= 5;
    int slot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int o = (int)t[d] - r[d];  // periodic offset in (-nt/2, nt/2]
        if (o > nt / 2) o -= nt;
        else if (o <= -((nt + 1) / 2)) o += nt;
        near = near && o >= -2 && o <= 2;
        slot = slot * 5 + (o + 2);
    }
    return near ? slot : -1;
}

// Count the tile of (x, y, z) for lanes with ok set (call with the whole wave).
// Usually every particle of a wave is in lane 0's tile: then lane 0 adds the
// wave's count once; otherwise each run of equal tiles in consecutive lanes
// adds once.
template <typename T>
__device__ __forceinline__ void tc_add(const TileCount& tc, const PartDesc<T>& a, bool ok, T x, T y, T z) {
    if (tc.counts == nullptr) return;
    const int nt = tiles_per_axis(a);
    const uint32_t t[3] = {ok ? tile_coord(a, x) : 0u, ok ? tile_coord(a, y) : 0u, ok ? tile_coord(a, z) : 0u};
    const uint32_t code = t[0] | (t[1] << 5) | (t[2] << 10);  // at most 32 tiles per axis
    const LDS_AS int* r = tc.lref();
    const uint64_t valid = __ballot(ok);
    if (valid == 0ull) return;
    const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)code);
    if ((valid & 1ull) && __ballot(ok && code == c0) == valid) {
        if ((threadIdx.x & 63) == 0) {
            const uint32_t n = (uint32_t)__popcll(valid);
            const int sl = tc_slot(r, t, nt);
            if (sl >= 0)
                __hip_atomic_fetch_add(tc.lslot() + sl, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_add(gp(tc.counts) + key_of_tile<3>(t[0], t[1], t[2]), n, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    const int sl = tc_slot(r, t, nt);
    const uint32_t id = !ok ? 0xFFFFFFFFu : sl >= 0 ? (uint32_t)sl : (uint32_t)TC_SLOTS + key_of_tile<3>(t[0], t[1], t[2]);
    int head;
    const uint32_t len = lane_runs(id, head);
    if (ok && len) {
        if (id < (uint32_t)TC_SLOTS)
            __hip_atomic_fetch_add(tc.lslot() + id, len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(gp(tc.counts) + (id - TC_SLOTS), len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Add the item's slots to the counts and clear them (whole workgroup, after
// the item's last tc_add).
template <typename T> __device__ __forceinline__ void tc_flush(const TileCount& tc, const PartDesc<T>& a) {
    if (tc.counts == nullptr) return;
    __syncthreads();
    const int s = threadIdx.x;
    if (s < TC_SLOTS) {
        LDS_AS uint32_t* sl = tc.lslot();
        const LDS_AS int* r = tc.lref();
        const uint32_t c = sl[s];
        if (c != 0u) {
            const int nt = tiles_per_axis(a);
            const int off[3] = {s / 25 - 2, (s / 5) % 5 - 2, s % 5 - 2};
            uint32_t t[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int v = (r[d] + off[d]) % nt;
                t[d] = (uint32_t)(v < 0 ? v + nt : v);
            }
            __hip_atomic_fetch_add(gp(tc.counts) + key_of_tile<3>(t[0], t[1], t[2]), c, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            sl[s] = 0u;
        }
    }
}

// ---------------------------------------------------------------------------
// deposit of one particle: 32 nodes of Gamma_4 with the weights of eq. 4ord.
// sink(index, F) receives the window index and the weight F (without mass).
// ---------------------------------------------------------------------------
template <typename T, typename Sink, bool P2>
__device__ __forceinline__ void deposit_one(Sink& sink, T x, T y, T z, T hl, const Wrap<P2>& wr, int ox, int oy, int oz,
                                            int Wy, int Wz) {
    const T sx = x * hl, sy = y * hl, sz = z * hl;
    const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
    const int gx = (int)fx, gy = (int)fy, gz = (int)fz;
    const Axis4<T> ax = axis4(sx - fx), ay = axis4(sy - fy), az = axis4(sz - fz);
    const T S = (T)1 + (ax.w0 * ax.w1 + ay.w0 * ay.w1 + az.w0 * az.w1) * (T)0.5;
    const int WyWz = Wy * Wz;
    int cx[4], cy[4], cz[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cx[j] = wr(gx - 1 + j - ox) * WyWz;
        cy[j] = wr(gy - 1 + j - oy) * Wz;
        cz[j] = wr(gz - 1 + j - oz);
    }
    const T wx[2] = {ax.w0, ax.w1}, wy[2] = {ay.w0, ay.w1}, wz[2] = {az.w0, az.w1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T pyz = wy[a] * wz[b];
            const T pxz = wx[a] * wz[b];
            const T pxy = wx[a] * wy[b];
            const T Spyz = S * pyz;
            // inner nodes (0/1, a, b)
            sink(cx[1] + cy[1 + a] + cz[1 + b], wx[0] * Spyz);
            sink(cx[2] + cy[1 + a] + cz[1 + b], wx[1] * Spyz);
            // outer nodes on x: (-1, a, b) and (2, a, b)
            sink(cx[0] + cy[1 + a] + cz[1 + b], ax.wm * pyz);
            sink(cx[3] + cy[1 + a] + cz[1 + b], ax.wp * pyz);
            // outer nodes on y: (a, -1, b) and (a, 2, b)
            sink(cx[1 + a] + cy[0] + cz[1 + b], ay.wm * pxz);
            sink(cx[1 + a] + cy[3] + cz[1 + b], ay.wp * pxz);
            // outer nodes on z: (a, b, -1) and (a, b, 2)
            sink(cx[1 + a] + cy[1 + b] + cz[0], az.wm * pxy);
            sink(cx[1 + a] + cy[1 + b] + cz[3], az.wp * pxy);
        }
    }
}

template <typename T> struct LdsSink {
    typename Fixed<T>::I* win;
    T scale;  // 2^S
    __device__ __forceinline__ void operator()(int idx, T F) const {
        atomicAdd(reinterpret_cast<typename Fixed<T>::U*>(win + idx), (typename Fixed<T>::U)Fixed<T>::quant(F * scale));
    }
};
template <typename T> struct GlobalSink {
    T* phi;
    T m;
    __device__ __forceinline__ void operator()(int idx, T F) const { gatomic_add(phi + idx, F * m); }
};

// trilinear interpolation (eq. 2ord) of three planar grids of node pitch n3,
// nodes (ix[a], iy[b], iz[c]) with row strides (Wy, Wz)
template <typename T, typename P>
__device__ __forceinline__ void trilinear3(P G, size_t n3, int Wy, int Wz, const int* ix, const int* iy, const int* iz,
                                           T lx, T ly, T lz, T& vx, T& vy, T& vz) {
    const T wx[2] = {(T)1 - lx, lx}, wy[2] = {(T)1 - ly, ly}, wz[2] = {(T)1 - lz, lz};
    T ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const size_t idx = ((size_t)ix[a] * Wy + iy[b]) * Wz + iz[c];
                const T w = wx[a] * wy[b] * wz[c];
                ax += w * G[idx];
                ay += w * G[n3 + idx];
                az += w * G[2 * n3 + idx];
            }
    vx = ax;
    vy = ay;
    vz = az;
}

// Fixed widths of the fast windows (cells per axis): the deposit window holds
// the item's cells plus the stencil reach, the gradient window the cells plus
// the trilinear reach and the W^- margin.  With compile-time strides every
// stencil node is an immediate offset from one LDS address.
template <typename T> struct Win;
// Odd widths keep all three axes in the LDS bank index (a power-of-two
// stride would drop the slowest axis from it).
#ifndef SIPF_WIN_D
#define SIPF_WIN_D 19
#endif
#ifndef SIPF_WIN_G
#define SIPF_WIN_G 15
#endif
template <> struct Win<float> { static constexpr int D = SIPF_WIN_D, G = SIPF_WIN_G; };
template <> struct Win<double> { static constexpr int D = 15, G = 11; };
// a window plane must fit one workgroup (plane_map)
static_assert(Win<float>::D * Win<float>::D <= PT && Win<double>::D * Win<double>::D <= PT, "window plane");
static_assert(Win<float>::G * Win<float>::G <= PT && Win<double>::G * Win<double>::G <= PT, "window plane");

// Fused FP32 pass: both fast windows are live at once, the deposit window first.
template <typename T> constexpr int fused_dep_bytes() {
    return (Win<T>::D * Win<T>::D * Win<T>::D * (int)sizeof(typename Fixed<T>::I) + 255) / 256 * 256;
}
template <typename T> constexpr int fused_win_bytes() {
    return fused_dep_bytes<T>() + (3 * Win<T>::G * Win<T>::G * Win<T>::G * (int)sizeof(T) + 255) / 256 * 256;
}
// FP32 items are also counting-sorted by cell when they are written back:
// 16-bit counts packed in pairs for the (D - 3)^3 cells of the largest box
// plus one overflow key, and eight wave totals.
constexpr int SORT_KEYS_MAX = (Win<float>::D - 3) * (Win<float>::D - 3) * (Win<float>::D - 3) + 1;
constexpr int SORT_WORDS_MAX = (SORT_KEYS_MAX + 1) / 2;
template <typename T> constexpr int fused_bytes() {
    return fused_win_bytes<T>() + ((SORT_WORDS_MAX + PT / 64) * 4 + 255) / 256 * 256;
}
// the write-out staging (one float4 per particle) fits in the two windows
static_assert(CH * 16 <= fused_win_bytes<float>(), "staging");

// LDS bytes the particle pass needs per workgroup (the larger fast window)
int particle_window_bytes(bool fp64) {
    const int d32 = Win<float>::D * Win<float>::D * Win<float>::D * 4;
    const int g32 = 3 * Win<float>::G * Win<float>::G * Win<float>::G * 4;
    const int d64 = Win<double>::D * Win<double>::D * Win<double>::D * 8;
    const int g64 = 3 * Win<double>::G * Win<double>::G * Win<double>::G * 8;
    const int b = fp64 ? (d64 > g64 ? d64 : g64) : (d32 > g32 ? d32 : g32);
    return (b + 255) / 256 * 256;
}

// Thread -> (i0, j, k) for walking a window of ey x ez columns along i with
// stride nrep = PT / (ey ez) (ey ez <= PT); threads beyond nrep ey ez get
// i0 = INT_MAX and do nothing.
__device__ __forceinline__ void plane_map(int ey, int ez, int& i0, int& j, int& k, int& nrep) {
    const int pl = ey * ez;
    nrep = PT / pl;
    const int t = threadIdx.x;
    j = 0;
    k = 0;
    if (t < nrep * pl) {
        int r;
        divmod_small(t, pl, 1.0f / (float)pl, i0, r);
        divmod_small(r, ez, 1.0f / (float)ez, j, k);
    } else {
        i0 = INT_MAX;
    }
}

// Deposit of one particle into a fixed-stride fixed-point window whose node
// (i, j, k) is at (i D + j) D + k, origin (ox, oy, oz).  The scale 2^S is
// folded into the x factors (every Gamma_4 weight has exactly one).
template <typename T, bool P2>
__device__ __forceinline__ void deposit_fast(typename Fixed<T>::I* win, T x, T y, T z, T hl, const Wrap<P2>& wr, int ox,
                                             int oy, int oz, T scale) {
    constexpr int D = Win<T>::D;
    using U = typename Fixed<T>::U;
    const T sx = x * hl, sy = y * hl, sz = z * hl;
    const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
    const int gx = (int)fx, gy = (int)fy, gz = (int)fz;
    const Axis4<T> ax = axis4(sx - fx), ay = axis4(sy - fy), az = axis4(sz - fz);
    const T S = (T)1 + (ax.w0 * ax.w1 + ay.w0 * ay.w1 + az.w0 * az.w1) * (T)0.5;
    const int base = (wr(gx - 1 - ox) * D + wr(gy - 1 - oy)) * D + wr(gz - 1 - oz);
    U* w = reinterpret_cast<U*>(win) + base;
    const T X[4] = {ax.wm * scale, ax.w0 * scale, ax.w1 * scale, ax.wp * scale};
    const T Y[4] = {ay.wm, ay.w0, ay.w1, ay.wp};
    const T Z[4] = {az.wm, az.w0, az.w1, az.wp};
#define SIPF_ADD(i, j, k, a, b) atomicAdd(w + ((i) * D + (j)) * D + (k), (U)Magic<T>::take(fma(a, b, Magic<T>::M)))
#pragma unroll
    for (int j = 1; j <= 2; ++j)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            const T yz = Y[j] * Z[k];
            const T Syz = S * yz;
            SIPF_ADD(1, j, k, X[1], Syz);  // inner nodes
            SIPF_ADD(2, j, k, X[2], Syz);
            SIPF_ADD(0, j, k, X[0], yz);   // outer nodes on x
            SIPF_ADD(3, j, k, X[3], yz);
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            const T xz = X[i] * Z[k];
            SIPF_ADD(i, 0, k, Y[0], xz);   // outer nodes on y
            SIPF_ADD(i, 3, k, Y[3], xz);
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int j = 1; j <= 2; ++j) {
            const T xy = X[i] * Y[j];
            SIPF_ADD(i, j, 0, Z[0], xy);   // outer nodes on z
            SIPF_ADD(i, j, 3, Z[3], xy);
        }
#undef SIPF_ADD
}

// Trilinear gather from a fixed-stride window (node (i, j, k) at (i G + j) G + k,
// three planes of G^3); false if the cell is not covered by the loaded part
// (ex, ey, ez) of the window.
template <typename T, bool P2>
__device__ __forceinline__ bool gather_fast(const T* Gw, int gx, int gy, int gz, T lx, T ly, T lz, const Wrap<P2>& wr,
                                            int ox, int oy, int oz, int ex, int ey, int ez, T& vx, T& vy, T& vz) {
    constexpr int G = Win<T>::G;
    constexpr int G3 = G * G * G;
    const int ix = wr(gx - ox), iy = wr(gy - oy), iz = wr(gz - oz);
    if (ix > ex - 2 || iy > ey - 2 || iz > ez - 2) return false;
    const T* p = Gw + mad24(mad24(ix, G, iy), G, iz);
    const T wx[2] = {(T)1 - lx, lx}, wy[2] = {(T)1 - ly, ly}, wz[2] = {(T)1 - lz, lz};
    T ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const T wab = wx[a] * wy[b];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T w = wab * wz[c];
                const int o = (a * G + b) * G + c;
                ax += w * p[o];
                ay += w * p[G3 + o];
                az += w * p[2 * G3 + o];
            }
        }
    vx = ax;
    vy = ay;
    vz = az;
    return true;
}

// One work item: particles [beg, beg + cnt) of one instance, held in registers.
template <typename T, bool DEP, bool PUSH, int SCHEME, bool P2>
__device__ __forceinline__ void item_pass(const PartDesc<T>& a, int64_t beg, int cnt, unsigned char* lds,
                                          int win_bytes, int* sh, const TileCount& tc) {
    using I = typename Fixed<T>::I;
    const int tid = threadIdx.x;
    const int H = a.H, Hh = H / 2;
    const Wrap<P2> wr{H, H - 1};
    const T hl = a.hl;
    T px[PPT], py[PPT], pz[PPT];
#if !SIPF_RELOAD
    uint32_t pid[PPT];
#endif
    // uniform per-item bases and 32-bit offsets; lanes past the end load the
    // item's last particle (cnt >= 1), so all loads issue without branches
    const T* ix = a.x + beg;
    const T* iy = a.y + beg;
    const T* iz = a.z + beg;
    const uint32_t* iid = a.id + beg;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int j = tid + k * PT;
        const uint32_t jj = (uint32_t)(j < cnt ? j : cnt - 1);
        px[k] = gp(ix)[jj];
        py[k] = gp(iy)[jj];
        pz[k] = gp(iz)[jj];
#if !SIPF_RELOAD
        if (PUSH) pid[k] = gp(iid)[jj];
#endif
    }
    if (tc.counts != nullptr) {
        tc_reference(tc, a, px[0], py[0], pz[0]);
        __syncthreads();
    }
    const bool windows = cnt >= MIN_WINDOW_ITEM;
    int rx = 0, ry = 0, rz = 0;
    if (windows) {
        // bounding box of the item's cells, relative to the first particle's cell
        if (tid < 3) sh[tid] = INT_MAX;
        else if (tid < 6) sh[tid] = INT_MIN;
        __syncthreads();
        rx = wr(ifloor(gp(a.x)[beg] * hl));
        ry = wr(ifloor(gp(a.y)[beg] * hl));
        rz = wr(ifloor(gp(a.z)[beg] * hl));
        int mnx = INT_MAX, mny = INT_MAX, mnz = INT_MAX, mxx = INT_MIN, mxy = INT_MIN, mxz = INT_MIN;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (tid + k * PT < cnt) {
                const int cx = wr(wr(ifloor(px[k] * hl)) - rx + Hh) - Hh;
                const int cy = wr(wr(ifloor(py[k] * hl)) - ry + Hh) - Hh;
                const int cz = wr(wr(ifloor(pz[k] * hl)) - rz + Hh) - Hh;
                mnx = min(mnx, cx); mxx = max(mxx, cx);
                mny = min(mny, cy); mxy = max(mxy, cy);
                mnz = min(mnz, cz); mxz = max(mxz, cz);
            }
        }
        mnx = wave_min(mnx); mny = wave_min(mny); mnz = wave_min(mnz);
        mxx = wave_max(mxx); mxy = wave_max(mxy); mxz = wave_max(mxz);
        if ((tid & 63) == 0) {
            atomicMin(&sh[0], mnx); atomicMin(&sh[1], mny); atomicMin(&sh[2], mnz);
            atomicMax(&sh[3], mxx); atomicMax(&sh[4], mxy); atomicMax(&sh[5], mxz);
        }
        __syncthreads();
    }

    if (DEP && windows && H > Win<T>::D && sh[3] - sh[0] + 4 <= Win<T>::D && sh[4] - sh[1] + 4 <= Win<T>::D &&
        sh[5] - sh[2] + 4 <= Win<T>::D) {
        // fast path: fixed-stride window, nodes -1..+2 around the box
        constexpr int D = Win<T>::D;
        I* win = reinterpret_cast<I*>(lds);
        const int ox = wr(rx + sh[0] - 1), oy = wr(ry + sh[1] - 1), oz = wr(rz + sh[2] - 1);
        const int ex = sh[3] - sh[0] + 4, ey = sh[4] - sh[1] + 4, ez = sh[5] - sh[2] + 4;
        // each thread owns one (j, k) column of the window and walks i
        int i0, wj, wk, nrep;
        plane_map(ey, ez, i0, wj, wk, nrep);
        for (int i = i0; i < ex; i += nrep) win[(i * D + wj) * D + wk] = 0;
        const int need = (11 * cnt + 7) / 8;
        const int S = min(Magic<T>::MAXS, Fixed<T>::BITS - (32 - __clz(need)));
        const T scale = (T)ldexp(1.0, S);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (tid + k * PT < cnt) deposit_fast<T>(win, px[k], py[k], pz[k], hl, wr, ox, oy, oz, scale);
        __syncthreads();
        const T back = a.wmass * (T)ldexp(1.0, -S);
        {
            const int nyz = wr(oy + wj) * H + wr(oz + wk);
            for (int i = i0; i < ex; i += nrep) {
                const I v = win[(i * D + wj) * D + wk];
                if (v != 0) gatomic_add(a.phi + wr(ox + i) * H * H + nyz, (T)v * back);
            }
        }
        __syncthreads();  // the window memory is reused below
    } else if (DEP) {
        int ox = 0, oy = 0, oz = 0, Wx = H, Wy = H, Wz = H;
        bool use_win = false;
        if (windows) {
            // nodes -1..+2 around every cell of the box
            axis_window(rx, sh[0] - 1, sh[3] + 2, wr, ox, Wx);
            axis_window(ry, sh[1] - 1, sh[4] + 2, wr, oy, Wy);
            axis_window(rz, sh[2] - 1, sh[5] + 2, wr, oz, Wz);
            use_win = (int64_t)Wx * Wy * Wz * (int64_t)sizeof(I) <= win_bytes;
        }
        if (use_win) {
            I* win = reinterpret_cast<I*>(lds);
            const int nw = Wx * Wy * Wz;
            for (int e = tid; e < nw; e += PT) win[e] = 0;
            // 2^S with S = BITS - bitlength(ceil(11 cnt / 8)): |sum of F| <= 1.375 cnt per node
            const int need = (11 * cnt + 7) / 8;
            const int S = Fixed<T>::BITS - (32 - __clz(need));
            const T scale = (T)ldexp(1.0, S);
            __syncthreads();
            LdsSink<T> sink{win, scale};
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (tid + k * PT < cnt) deposit_one(sink, px[k], py[k], pz[k], hl, wr, ox, oy, oz, Wy, Wz);
            __syncthreads();
            const T back = a.wmass * (T)ldexp(1.0, -S);
            const int WyWz = Wy * Wz;
            for (int e = tid; e < nw; e += PT) {
                const I v = win[e];
                if (v != 0) {
                    const int ex = e / WyWz, r = e - ex * WyWz;
                    const int ey = r / Wz, ez = r - ey * Wz;
                    const size_t node = ((size_t)wr(ox + ex) * H + wr(oy + ey)) * H + wr(oz + ez);
                    gatomic_add(a.phi + node, (T)v * back);
                }
            }
            __syncthreads();  // the window memory is reused below
        } else {
            GlobalSink<T> sink{a.phi, a.wmass};
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (tid + k * PT < cnt) deposit_one(sink, px[k], py[k], pz[k], hl, wr, 0, 0, 0, H, H);
        }
    }

    if (PUSH) {
        // gradient window: cells of the box (+ margin for the W^- displacement) and +1 for the trilinear reach
        int ox = 0, oy = 0, oz = 0, Wx = H, Wy = H, Wz = H;
        bool use_win = false, fast = false;
        const T* Gl = reinterpret_cast<const T*>(lds);
        size_t n3 = 0;
        if (windows && H > Win<T>::G) {
            constexpr int G = Win<T>::G;
            constexpr int G3 = G * G * G;
            for (int m = a.gmargin; m >= 0 && !fast; --m)
                fast = sh[3] - sh[0] + 2 + 2 * m <= G && sh[4] - sh[1] + 2 + 2 * m <= G &&
                       sh[5] - sh[2] + 2 + 2 * m <= G;
            if (fast) {
                int m = a.gmargin;
                while (sh[3] - sh[0] + 2 + 2 * m > G || sh[4] - sh[1] + 2 + 2 * m > G || sh[5] - sh[2] + 2 + 2 * m > G) --m;
                ox = wr(rx + sh[0] - m);
                oy = wr(ry + sh[1] - m);
                oz = wr(rz + sh[2] - m);
                Wx = sh[3] - sh[0] + 2 + 2 * m;
                Wy = sh[4] - sh[1] + 2 + 2 * m;
                Wz = sh[5] - sh[2] + 2 + 2 * m;
                T* Gw = reinterpret_cast<T*>(lds);
                const int H3 = H * H * H;
                int i0, wj, wk, nrep;
                plane_map(Wy, Wz, i0, wj, wk, nrep);
                const int nyz = wr(oy + wj) * H + wr(oz + wk);
                for (int i = i0; i < Wx; i += nrep) {
                    const int node = wr(ox + i) * H * H + nyz;
                    const int o = (i * G + wj) * G + wk;
                    Gw[o] = gp(a.G)[node];
                    Gw[G3 + o] = gp(a.G)[H3 + node];
                    Gw[2 * G3 + o] = gp(a.G)[2 * H3 + node];
                }
                __syncthreads();
            }
        }
        if (windows && !fast) {
            for (int m = a.gmargin; m >= 0 && !use_win; --m) {
                axis_window(rx, sh[0] - m, sh[3] + 1 + m, wr, ox, Wx);
                axis_window(ry, sh[1] - m, sh[4] + 1 + m, wr, oy, Wy);
                axis_window(rz, sh[2] - m, sh[5] + 1 + m, wr, oz, Wz);
                use_win = 3 * (int64_t)Wx * Wy * Wz * (int64_t)sizeof(T) <= win_bytes;
            }
            if (use_win) {
                T* Gw = reinterpret_cast<T*>(lds);
                const int nw = Wx * Wy * Wz;
                n3 = (size_t)nw;
                const size_t H3 = (size_t)H * H * H;
                const int WyWz = Wy * Wz;
                for (int e = tid; e < nw; e += PT) {
                    const int ex = e / WyWz, r = e - ex * WyWz;
                    const int ey = r / Wz, ez = r - ey * Wz;
                    const size_t node = ((size_t)wr(ox + ex) * H + wr(oy + ey)) * H + wr(oz + ez);
                    Gw[e] = gp(a.G)[node];
                    Gw[nw + e] = gp(a.G)[H3 + node];
                    Gw[2 * nw + e] = gp(a.G)[2 * H3 + node];
                }
                __syncthreads();
            }
        }
        const uint32_t n = *a.step + 1u;
        const size_t H3 = (size_t)H * H * H;
#pragma unroll SIPF_PUSH_UNROLL
        for (int k = 0; k < PPT; ++k) {
            const int j = tid + k * PT;
            const bool valid = j < cnt;
            T nx = (T)0, ny = (T)0, nz = (T)0;
            if (valid) {
#if SIPF_RELOAD
            // re-read from L2 rather than holding eight particles in registers
            const T x = gp(ix)[j], y = gp(iy)[j], z = gp(iz)[j];
            const uint32_t idk = gp(iid)[j];
#else
            const T x = px[k], y = py[k], z = pz[k];
            const uint32_t idk = pid[k];
#endif
            T yx, yy, yz, w0, w1, w2;
            T zn[6];
            if (SCHEME == SIPF_STRANG) {
                noise6<3, T>(idk, n, a.inst, a.k0, a.k1, zn);
                yx = x + a.s * zn[0];
                yy = y + a.s * zn[1];
                yz = z + a.s * zn[2];
                w0 = zn[3];
                w1 = zn[4];
                w2 = zn[5];
            } else {
                noise6<2, T>(idk, n, a.inst, a.k0, a.k1, zn);
                w0 = zn[0];
                w1 = zn[1];
                w2 = zn[2];
                yx = x;
                yy = y;
                yz = z;
            }
            const T sx = yx * hl, sy = yy * hl, sz = yz * hl;
            const T fx = floor(sx), fy = floor(sy), fz = floor(sz);
            const int gx = (int)fx, gy = (int)fy, gz = (int)fz;
            int ix[2] = {wr(gx - ox), wr(gx + 1 - ox)};
            int iy[2] = {wr(gy - oy), wr(gy + 1 - oy)};
            int iz[2] = {wr(gz - oz), wr(gz + 1 - oz)};
            T vx, vy, vz;
            const bool inside = !fast && use_win && (Wx == H || ix[0] <= Wx - 2) && (Wy == H || iy[0] <= Wy - 2) &&
                                (Wz == H || iz[0] <= Wz - 2);
            if (fast && gather_fast<T>(Gl, gx, gy, gz, sx - fx, sy - fy, sz - fz, wr, ox, oy, oz, Wx, Wy, Wz, vx, vy,
                                       vz)) {
                // gathered from the fixed-stride window
            } else if (inside) {
                trilinear3<T>(Gl, n3, Wy, Wz, ix, iy, iz, sx - fx, sy - fy, sz - fz, vx, vy, vz);
            } else {
                ix[0] = wr(gx); ix[1] = wr(gx + 1);
                iy[0] = wr(gy); iy[1] = wr(gy + 1);
                iz[0] = wr(gz); iz[1] = wr(gz + 1);
                trilinear3<T>(gp(a.G), H3, H, H, ix, iy, iz, sx - fx, sy - fy, sz - fz, vx, vy, vz);
            }
            nx = wrap_box(yx + a.chitau * vx + a.s * w0, a.L, a.halfL, a.invL);
            ny = wrap_box(yy + a.chitau * vy + a.s * w1, a.L, a.halfL, a.invL);
            nz = wrap_box(yz + a.chitau * vz + a.s * w2, a.L, a.halfL, a.invL);
            if (!DEP && a.zout != nullptr) {
                // keep the normals of this step for the reverse pass (adjoint recompute)
                const int nz6 = SCHEME == SIPF_STRANG ? 6 : 3;
                for (int q = 0; q < nz6; ++q) gp(a.zout + q * a.P + beg)[j] = zn[q];
            }
            if (!DEP && a.ox != nullptr) {
                // out of place (push-only passes): positions and ids to the output set
                gp(a.ox + beg)[j] = nx;
                gp(a.oy + beg)[j] = ny;
                gp(a.oz + beg)[j] = nz;
                gp(a.oid + beg)[j] = gp(iid)[j];
            } else {
                gp(a.x + beg)[j] = nx;
                gp(a.y + beg)[j] = ny;
                gp(a.z + beg)[j] = nz;
            }
            if (!(isfinite(nx) && isfinite(ny) && isfinite(nz))) atomicOr(a.err, 1);
            }
            tc_add(tc, a, valid, nx, ny, nz);
        }
    }
}

// Persistent over the work items listed by the last sort (header: next_item).
// Lane layout of an FP32 item of cnt particles: ppe = ceil(cnt / PT)
// particles per lane on lact = ceil(cnt / ppe) lanes; lane t holds the
// particles of ranks t ppe .. t ppe + ppe - 1 of the item, and rank
// s = t ppe + k is stored at column k, row t: position col(k) + t with
// col(k) = k lact - max(0, k - rlast), where rlast = cnt - (lact - 1) ppe is
// the length of the last lane's run (columns k >= rlast are one row short).
// Loads of one column are contiguous; a lane's ranks are consecutive.
struct ColLayout {
    int ppe, lact, rlast;
    __device__ __forceinline__ ColLayout(int cnt) {
        ppe = (cnt + PT - 1) / PT;
        lact = (cnt + ppe - 1) / ppe;
        rlast = cnt - (lact - 1) * ppe;
    }
    __device__ __forceinline__ int col(int k) const { return k * lact - max(0, k - rlast); }
    __device__ __forceinline__ bool valid(int t, int k) const {
        return k < ppe && t < lact && (t < lact - 1 || k < rlast);
    }
};

// The sorted FP32 pass accumulates its deposit window in fixed point with
// integer LDS atomics: on gfx950 a float LDS atomic add (ds_add_f32) issues
// about fifty times slower than the integer one.
using RunWin = int32_t;

// The 32 weights of eq. 4ord of one particle times the window scale 2^S,
// added to a run accumulator (slots in the order of flush_run4).
__device__ __forceinline__ void add_weights4(float* acc, const Axis4<float>& ax, const Axis4<float>& ay,
                                             const Axis4<float>& az, float S, float scale) {
    const float X[4] = {ax.wm * scale, ax.w0 * scale, ax.w1 * scale, ax.wp * scale};
    const float Y[4] = {ay.wm, ay.w0, ay.w1, ay.wp};
    const float Z[4] = {az.wm, az.w0, az.w1, az.wp};
    int q = 0;
#pragma unroll
    for (int j = 1; j <= 2; ++j)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            const float yz = Y[j] * Z[k];
            const float Syz = S * yz;
            acc[q] = fmaf(X[1], Syz, acc[q]); ++q;  // inner nodes (1, j, k), (2, j, k)
            acc[q] = fmaf(X[2], Syz, acc[q]); ++q;
            acc[q] = fmaf(X[0], yz, acc[q]); ++q;   // outer nodes on x: (0, j, k), (3, j, k)
            acc[q] = fmaf(X[3], yz, acc[q]); ++q;
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            const float xz = X[i] * Z[k];
            acc[q] = fmaf(Y[0], xz, acc[q]); ++q;   // outer nodes on y: (i, 0, k), (i, 3, k)
            acc[q] = fmaf(Y[3], xz, acc[q]); ++q;
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int j = 1; j <= 2; ++j) {
            const float xy = X[i] * Y[j];
            acc[q] = fmaf(Z[0], xy, acc[q]); ++q;   // outer nodes on z: (i, j, 0), (i, j, 3)
            acc[q] = fmaf(Z[3], xy, acc[q]); ++q;
        }
}

// Adds a run accumulator (already at the window scale 2^S), rounded to
// integers, to the fixed-point deposit window at the run's base node
// (cell - (1,1,1)); node (i, j, k) at (i D + j) D + k.
__device__ __forceinline__ void flush_run4(RunWin* win, int base, const float* acc) {
    constexpr int D = Win<float>::D;
    uint32_t* w = reinterpret_cast<uint32_t*>(win) + base;
#define SIPF_FL(q, i, j, k) atomicAdd(w + ((i) * D + (j)) * D + (k), (uint32_t)round_half_up(acc[q]))
    int q = 0;
#pragma unroll
    for (int j = 1; j <= 2; ++j)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            SIPF_FL(q, 1, j, k); ++q;
            SIPF_FL(q, 2, j, k); ++q;
            SIPF_FL(q, 0, j, k); ++q;
            SIPF_FL(q, 3, j, k); ++q;
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int k = 1; k <= 2; ++k) {
            SIPF_FL(q, i, 0, k); ++q;
            SIPF_FL(q, i, 3, k); ++q;
        }
#pragma unroll
    for (int i = 1; i <= 2; ++i)
#pragma unroll
        for (int j = 1; j <= 2; ++j) {
            SIPF_FL(q, i, j, 0); ++q;
            SIPF_FL(q, i, j, 3); ++q;
        }
#undef SIPF_FL
}

// Particles of an FP32 item in the lane layout, loaded into registers.
__device__ __forceinline__ void load_cols(const PartDesc<float>& a, int64_t beg, int cnt, float* px, float* py,
                                          float* pz, uint32_t* pid) {
    const ColLayout cl(cnt);
    const int tid = threadIdx.x;
    const float* ix = a.x + beg;
    const float* iy = a.y + beg;
    const float* iz = a.z + beg;
    const uint32_t* iid = a.id + beg;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t jj = (uint32_t)(cl.valid(tid, k) ? cl.col(k) + tid : 0);
        px[k] = gp(ix)[jj];
        py[k] = gp(iy)[jj];
        pz[k] = gp(iz)[jj];
        pid[k] = gp(iid)[jj];
    }
}

// Whether an FP32 item can take the sorted pass (its box is checked there).
__device__ __forceinline__ bool sorted_candidate(const PartDesc<float>& a, const WorkItem& w, int win_bytes) {
    return a.ox == nullptr && w.cnt >= MIN_WINDOW_ITEM && a.H > Win<float>::D && a.H > Win<float>::G &&
           win_bytes >= fused_bytes<float>();
}

// FP32 work item in one loop, with the item kept sorted by cell between
// steps.  The particles arrive in the lane layout above, sorted by cell by
// the previous step's write-out (in the order of the re-sort right after
// one).  Each particle deposits its position X^(n-1) (Algorithm 4 reads only
// the state after step n-1 in both branches, so the deposit and the push of a
// particle are independent and one pass serves both): a lane adds the
// weights of its consecutive particles into registers while they share a
// cell and adds each run to the deposit window once (one set of 32 LDS
// atomics per run instead of per particle; the lanes of a wave then work on
// neighbouring cells, so those atomics spread over the LDS banks).  The
// particle then draws its noise, gathers the gradient at Y from the gradient
// window (neighbouring lanes read neighbouring rows) and is pushed.  The
// pushed particles are counting-sorted by
// their new cell inside the item's box (cells that left it go last) and
// written back to the item's segment in the lane layout, which keeps the
// order for the next step.  Returns false, touching nothing, when the item
// does not fit the windows.
template <int SCHEME, bool P2>
__device__ __forceinline__ bool item_sorted(const PartDesc<float>& a, int64_t beg, int cnt, unsigned char* lds,
                                            int* sh, const TileCount& tc) {
    float px[PPT], py[PPT], pz[PPT];
    uint32_t pid[PPT];
    load_cols(a, beg, cnt, px, py, pz, pid);
    constexpr int D = Win<float>::D, G = Win<float>::G, G3 = G * G * G;
    const int tid = threadIdx.x;
    const int H = a.H, Hh = H / 2;
    const Wrap<P2> wr{H, H - 1};
    const float hl = a.hl;
    const ColLayout cl(cnt);
    // bounding box of the item's cells, relative to the cell of its first particle (thread 0, k = 0)
    if (tid < 3) sh[tid] = INT_MAX;
    else if (tid < 6) sh[tid] = INT_MIN;
    if (tid == 0) {
        sh[8] = wr(ifloor(px[0] * hl));
        sh[9] = wr(ifloor(py[0] * hl));
        sh[10] = wr(ifloor(pz[0] * hl));
    }
    tc_reference(tc, a, px[0], py[0], pz[0]);
    __syncthreads();
    const int rx = sh[8], ry = sh[9], rz = sh[10];
    {
        int mnx = INT_MAX, mny = INT_MAX, mnz = INT_MAX, mxx = INT_MIN, mxy = INT_MIN, mxz = INT_MIN;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cl.valid(tid, k)) {
                const int cx = wr(wr(ifloor(px[k] * hl)) - rx + Hh) - Hh;
                const int cy = wr(wr(ifloor(py[k] * hl)) - ry + Hh) - Hh;
                const int cz = wr(wr(ifloor(pz[k] * hl)) - rz + Hh) - Hh;
                mnx = min(mnx, cx); mxx = max(mxx, cx);
                mny = min(mny, cy); mxy = max(mxy, cy);
                mnz = min(mnz, cz); mxz = max(mxz, cz);
            }
        }
        mnx = wave_min(mnx); mny = wave_min(mny); mnz = wave_min(mnz);
        mxx = wave_max(mxx); mxy = wave_max(mxy); mxz = wave_max(mxz);
        if ((tid & 63) == 0) {
            atomicMin(&sh[0], mnx); atomicMin(&sh[1], mny); atomicMin(&sh[2], mnz);
            atomicMax(&sh[3], mxx); atomicMax(&sh[4], mxy); atomicMax(&sh[5], mxz);
        }
    }
    __syncthreads();
    const int bx0 = sh[0], by0 = sh[1], bz0 = sh[2];
    const int nbx = sh[3] - bx0 + 1, nby = sh[4] - by0 + 1, nbz = sh[5] - bz0 + 1;
    int m = a.gmargin;
    while (m >= 0 && (nbx + 1 + 2 * m > G || nby + 1 + 2 * m > G || nbz + 1 + 2 * m > G)) --m;
    if (nbx + 3 > D || nby + 3 > D || nbz + 3 > D || m < 0) {
        __syncthreads();  // sh is rewritten by the caller's fallback
        return false;
    }
    RunWin* win = reinterpret_cast<RunWin*>(lds);
    float* Gw = reinterpret_cast<float*>(lds + fused_dep_bytes<float>());
    uint32_t* cw = reinterpret_cast<uint32_t*>(lds + fused_win_bytes<float>());
    uint32_t* wtot = cw + SORT_WORDS_MAX;
    const int nkeys = nbx * nby * nbz + 1, nwords = (nkeys + 1) / 2;
    // deposit window: nodes -1..+2 around the box; sort counters
    const int dox = wr(rx + bx0 - 1), doy = wr(ry + by0 - 1), doz = wr(rz + bz0 - 1);
    {
        int i0, wj, wk, nrep;
        plane_map(nby + 3, nbz + 3, i0, wj, wk, nrep);
        for (int i = i0; i < nbx + 3; i += nrep) win[(i * D + wj) * D + wk] = (RunWin)0;
        for (int w = tid; w < nwords; w += PT) cw[w] = 0u;
    }
    // gradient window: the box, the W^- margin m and the trilinear reach
    const int gox = wr(rx + bx0 - m), goy = wr(ry + by0 - m), goz = wr(rz + bz0 - m);
    const int gWx = nbx + 1 + 2 * m, gWy = nby + 1 + 2 * m, gWz = nbz + 1 + 2 * m;
    {
        const int H3 = H * H * H;
        int i0, wj, wk, nrep;
        plane_map(gWy, gWz, i0, wj, wk, nrep);
        const int nyz = wr(goy + wj) * H + wr(goz + wk);
        for (int i = i0; i < gWx; i += nrep) {
            const int node = wr(gox + i) * H * H + nyz;
            const int o = (i * G + wj) * G + wk;
            Gw[o] = gp(a.G)[node];
            Gw[G3 + o] = gp(a.G)[H3 + node];
            Gw[2 * G3 + o] = gp(a.G)[2 * H3 + node];
        }
    }
    const int need = (11 * cnt + 7) / 8;
    const int S = min(Magic<float>::MAXS, Fixed<float>::BITS - (32 - __clz(need)));
    const float scale = ldexpf(1.0f, S);
    const uint32_t step_n = *a.step + 1u;
    const size_t H3 = (size_t)H * H * H;
    __syncthreads();

    float acc[32];
    int run = -1;  // window base node of the run in acc
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (!cl.valid(tid, k)) continue;
        const float x = px[k], y = py[k], z = pz[k];
        {
            const float sx = x * hl, sy = y * hl, sz = z * hl;
            const float fx = floorf(sx), fy = floorf(sy), fz = floorf(sz);
            const int base =
                mad24(mad24(wr((int)fx - 1 - dox), D, wr((int)fy - 1 - doy)), D, wr((int)fz - 1 - doz));
            if (base != run) {
                if (run >= 0) flush_run4(win, run, acc);
#pragma unroll
                for (int q = 0; q < 32; ++q) acc[q] = 0.0f;
                run = base;
            }
            const Axis4<float> ax = axis4(sx - fx), ay = axis4(sy - fy), az = axis4(sz - fz);
            add_weights4(acc, ax, ay, az, 1.0f + (ax.w0 * ax.w1 + ay.w0 * ay.w1 + az.w0 * az.w1) * 0.5f, scale);
        }
        float yx, yy, yz, w0, w1, w2;
        float zn[6];
        if (SCHEME == SIPF_STRANG) {
            noise6<3, float>(pid[k], step_n, a.inst, a.k0, a.k1, zn);
            yx = x + a.s * zn[0];
            yy = y + a.s * zn[1];
            yz = z + a.s * zn[2];
            w0 = zn[3];
            w1 = zn[4];
            w2 = zn[5];
        } else {
            noise6<2, float>(pid[k], step_n, a.inst, a.k0, a.k1, zn);
            w0 = zn[0];
            w1 = zn[1];
            w2 = zn[2];
            yx = x;
            yy = y;
            yz = z;
        }
        const float sx = yx * hl, sy = yy * hl, sz = yz * hl;
        const float fx = floorf(sx), fy = floorf(sy), fz = floorf(sz);
        const int gx = (int)fx, gy = (int)fy, gz = (int)fz;
        float vx, vy, vz;
        if (!gather_fast<float>(Gw, gx, gy, gz, sx - fx, sy - fy, sz - fz, wr, gox, goy, goz, gWx, gWy, gWz, vx,
                                vy, vz)) {
            const int jx[2] = {wr(gx), wr(gx + 1)};
            const int jy[2] = {wr(gy), wr(gy + 1)};
            const int jz[2] = {wr(gz), wr(gz + 1)};
            trilinear3<float>(gp(a.G), H3, H, H, jx, jy, jz, sx - fx, sy - fy, sz - fz, vx, vy, vz);
        }
        px[k] = wrap_box(yx + a.chitau * vx + a.s * w0, a.L, a.halfL, a.invL);
        py[k] = wrap_box(yy + a.chitau * vy + a.s * w1, a.L, a.halfL, a.invL);
        pz[k] = wrap_box(yz + a.chitau * vz + a.s * w2, a.L, a.halfL, a.invL);
        if (!(isfinite(px[k]) && isfinite(py[k]) && isfinite(pz[k]))) atomicOr(a.err, 1);
    }
    if (run >= 0) flush_run4(win, run, acc);
    // ranks of the pushed particles among those of the same new cell
    uint32_t kr[PPT];  // key << 16 | rank
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        kr[k] = 0u;
        if (!cl.valid(tid, k)) continue;
        const int cx = wr(wr(ifloor(px[k] * hl)) - rx + Hh) - Hh - bx0;
        const int cy = wr(wr(ifloor(py[k] * hl)) - ry + Hh) - Hh - by0;
        const int cz = wr(wr(ifloor(pz[k] * hl)) - rz + Hh) - Hh - bz0;
        const bool in = (unsigned)cx < (unsigned)nbx && (unsigned)cy < (unsigned)nby && (unsigned)cz < (unsigned)nbz;
        const uint32_t kk = in ? (uint32_t)mad24(mad24(cx, nby, cy), nbz, cz) : (uint32_t)(nkeys - 1);
        const uint32_t sft = 16u * (kk & 1u);
        kr[k] = (kk << 16) | ((atomicAdd(&cw[kk >> 1], 1u << sft) >> sft) & 0xFFFFu);
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) tc_add(tc, a, cl.valid(tid, k), px[k], py[k], pz[k]);
    __syncthreads();
    // the deposit window into the grid
    {
        const float back = a.wmass * ldexpf(1.0f, -S);
        int i0, wj, wk, nrep;
        plane_map(nby + 3, nbz + 3, i0, wj, wk, nrep);
        const int nyz = wr(doy + wj) * H + wr(doz + wk);
        for (int i = i0; i < nbx + 3; i += nrep) {
            const RunWin v = win[(i * D + wj) * D + wk];
            if (v != (RunWin)0) gatomic_add(a.phi + wr(dox + i) * H * H + nyz, (float)v * back);
        }
    }
    // exclusive scan of the counts: thread t owns words [t wp, t wp + wp)
    const int wp = (nwords + PT - 1) / PT;
    uint32_t loc = 0;
    for (int i = 0; i < wp; ++i) {
        const int w = tid * wp + i;
        if (w < nwords) {
            const uint32_t v = cw[w];
            loc += (v & 0xFFFFu) + (v >> 16);
        }
    }
    uint32_t incl = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(incl, off, 64);
        if ((tid & 63) >= off) incl += u;
    }
    if ((tid & 63) == 63) wtot[tid >> 6] = incl;
    __syncthreads();
    {
        uint32_t b = incl - loc;
        for (int w = 0; w < (tid >> 6); ++w) b += wtot[w];
        for (int i = 0; i < wp; ++i) {
            const int w = tid * wp + i;
            if (w < nwords) {
                const uint32_t v = cw[w], lo = v & 0xFFFFu;
                cw[w] = b | ((b + lo) << 16);
                b += lo + (v >> 16);
            }
        }
    }
    __syncthreads();
    // stage in the lane layout (over the dead windows), then write back
    float4* stg = reinterpret_cast<float4*>(lds);
    const float inv_ppe = 1.0f / (float)cl.ppe;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (!cl.valid(tid, k)) continue;
        const uint32_t kk = kr[k] >> 16, sft = 16u * (kk & 1u);
        const int s = (int)(((cw[kk >> 1] >> sft) & 0xFFFFu) + (kr[k] & 0xFFFFu));
        int t2, k2;
        divmod_small(s, cl.ppe, inv_ppe, t2, k2);
        stg[cl.col(k2) + t2] = make_float4(px[k], py[k], pz[k], __uint_as_float(pid[k]));
    }
    __syncthreads();
    for (int g = tid; g < cnt; g += PT) {
        const float4 v = stg[g];
        gp(a.x + beg)[g] = v.x;
        gp(a.y + beg)[g] = v.y;
        gp(a.z + beg)[g] = v.z;
        gp(a.id + beg)[g] = __float_as_uint(v.w);
    }
    return true;
}

// kcounts: the sort's tile counts of every instance (MAX_KEYS each) when this
// step takes them for the next sort (3-D deposit + push passes), else null.
// COUNT: the instantiation that takes the counts (the other one carries no
// counting code, so its registers are those of the plain pass).
template <typename T, bool DEP, bool PUSH, int SCHEME, bool P2, bool SORTED, bool COUNT>
__device__ __forceinline__ void particles_body(const PartDesc<T>* __restrict__ pds,
                                               const WorkItem* __restrict__ items, int* hdr, int win_bytes,
                                               unsigned char* smem_raw, int* sh, int* slot_p, uint32_t* kcounts,
                                               uint32_t* tslot, int* tref) {
    const int n = hdr[0];
    if (!COUNT) kcounts = nullptr;
    if (kcounts != nullptr)
        for (int i = threadIdx.x; i < TC_SLOTS; i += PT)
            ((LDS_AS uint32_t*)tslot)[i] = 0u;  // first read after the item's barriers
    for (int it = blockIdx.x; it < n; it = next_item(hdr, n, slot_p)) {
        const WorkItem w = items[it];
        const PartDesc<T>& a = pds[w.inst];
        const TileCount tc{kcounts != nullptr ? kcounts + (size_t)w.inst * MAX_KEYS : nullptr, tslot, tref};
        bool done = false;
        if constexpr (SORTED) done = sorted_candidate(a, w, win_bytes) && item_sorted<SCHEME, P2>(a, w.beg, w.cnt, smem_raw, sh, tc);
        if (!done) item_pass<T, DEP, PUSH, SCHEME, P2>(a, w.beg, w.cnt, smem_raw, win_bytes, sh, tc);
        tc_flush(tc, a);
    }
}

// Two-phase passes: FP64 deposit + push, and the deposit-only and push-only
// passes of both precisions.
template <typename T, bool DEP, bool PUSH, int SCHEME, bool P2, bool COUNT = false>
__global__ __launch_bounds__(PT) SIPF_PART_ATTR void k_particles(const PartDesc<T>* __restrict__ pds,
                                                  const WorkItem* __restrict__ items, int* hdr, int win_bytes,
                                                  uint32_t* kcounts) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int sh[8];
    __shared__ int slot;
    __shared__ uint32_t tslot[TC_SLOTS];
    __shared__ int tref[3];
    particles_body<T, DEP, PUSH, SCHEME, P2, false, COUNT>(pds, items, hdr, win_bytes, smem_raw, sh, &slot, kcounts,
                                                           tslot, tref);
}

// The FP32 two-phase deposit + push pass (items kept in tile order, not
// sorted by cell): one window at a time, so three workgroups fit a CU and the
// registers are budgeted for six waves per SIMD.
#ifndef SIPF_TWO_WAVES
#define SIPF_TWO_WAVES 6
#endif
template <int SCHEME, bool P2, bool COUNT = false>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(SIPF_TWO_WAVES))) void k_particles_two(
    const PartDesc<float>* __restrict__ pds, const WorkItem* __restrict__ items, int* hdr, int win_bytes,
    uint32_t* kcounts) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int sh[8];
    __shared__ int slot;
    __shared__ uint32_t tslot[TC_SLOTS];
    __shared__ int tref[3];
    particles_body<float, true, true, SCHEME, P2, false, COUNT>(pds, items, hdr, win_bytes, smem_raw, sh, &slot,
                                                                kcounts, tslot, tref);
}

// The fused deposit + push pass: its two windows (and, in FP32, the sort
// counters) allow two workgroups per CU, i.e. four waves per SIMD, so the
// registers are budgeted for four.
#ifndef SIPF_FUSED_WAVES
#define SIPF_FUSED_WAVES 4
#endif
template <typename T, int SCHEME, bool P2, bool COUNT = false>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(SIPF_FUSED_WAVES))) void k_particles_fused(
    const PartDesc<T>* __restrict__ pds, const WorkItem* __restrict__ items, int* hdr, int win_bytes,
    uint32_t* kcounts) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int sh[12];
    __shared__ int slot;
    __shared__ uint32_t tslot[TC_SLOTS];
    __shared__ int tref[3];
    particles_body<T, true, true, SCHEME, P2, true, COUNT>(pds, items, hdr, win_bytes, smem_raw, sh, &slot, kcounts,
                                                           tslot, tref);
}

// Workgroups of the fused particle pass that are resident on the whole device
// at once (occupancy from its registers and its LDS window): the persistent
// grid is sized to this, so that no workgroup waits for another to finish
// before it can start its share of the work items.
template <typename T> int particle_resident_blocks(int scheme, int win_bytes, bool sorted) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e;
    if constexpr (sizeof(T) == 4) {
        if (!sorted) {
            e = scheme == SIPF_STRANG ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                            &per_cu, (const void*)k_particles_two<SIPF_STRANG, true>, PT, win_bytes)
                                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                            &per_cu, (const void*)k_particles_two<SIPF_EM, true>, PT, win_bytes);
        } else {
            if (win_bytes < fused_bytes<T>()) win_bytes = fused_bytes<T>();
        e = scheme == SIPF_STRANG ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                        &per_cu, (const void*)k_particles_fused<T, SIPF_STRANG, true>, PT, win_bytes)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                        &per_cu, (const void*)k_particles_fused<T, SIPF_EM, true>, PT, win_bytes);
        }
    } else {
        e = scheme == SIPF_STRANG
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, (const void*)k_particles<T, true, true, SIPF_STRANG, true>, PT, win_bytes)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &per_cu, (const void*)k_particles<T, true, true, SIPF_EM, true>, PT, win_bytes);
    }
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || per_cu < 1 || cus < 1) {
        (void)hipGetLastError();
        return 1024;
    }
    return per_cu * cus;
}

template <typename T, bool P2>
static void particles_p2(const PartDesc<T>* pd, const WorkItem* items, int* nitems, dim3 g, bool deposit,
                         bool push, int scheme, int win_bytes, bool sorted, uint32_t* kcounts, hipStream_t s) {
    const dim3 b(PT);
    // tile counts are taken only by the deposit + push pass, in its COUNT instantiation
    const bool count = deposit && push && kcounts != nullptr;
    const bool strang = scheme == SIPF_STRANG;
    if (deposit && push) {
        if constexpr (sizeof(T) == 4) {
            if (!sorted) {
                const size_t shm = (size_t)win_bytes;
                if (count)
                    launch_kernel(strang ? k_particles_two<SIPF_STRANG, P2, true> : k_particles_two<SIPF_EM, P2, true>, g,
                                  b, shm, s, pd, items, nitems, win_bytes, kcounts);
                else
                    launch_kernel(strang ? k_particles_two<SIPF_STRANG, P2> : k_particles_two<SIPF_EM, P2>, g, b, shm, s,
                                  pd, items, nitems, win_bytes, (uint32_t*)nullptr);
                return;
            }
            // the sorted pass holds both windows and the sort counters at once
            if (win_bytes < fused_bytes<T>()) win_bytes = fused_bytes<T>();
            const size_t shm = (size_t)win_bytes;
            if (count)
                launch_kernel(strang ? k_particles_fused<T, SIPF_STRANG, P2, true> : k_particles_fused<T, SIPF_EM, P2, true>,
                              g, b, shm, s, pd, items, nitems, win_bytes, kcounts);
            else
                launch_kernel(strang ? k_particles_fused<T, SIPF_STRANG, P2> : k_particles_fused<T, SIPF_EM, P2>, g, b, shm,
                              s, pd, items, nitems, win_bytes, (uint32_t*)nullptr);
            return;
        }
    }
    const size_t shm = (size_t)win_bytes;
    if (deposit && push) {
        if constexpr (sizeof(T) == 8) {
            if (count)
                launch_kernel(strang ? k_particles<T, true, true, SIPF_STRANG, P2, true>
                                     : k_particles<T, true, true, SIPF_EM, P2, true>,
                              g, b, shm, s, pd, items, nitems, win_bytes, kcounts);
            else
                launch_kernel(strang ? k_particles<T, true, true, SIPF_STRANG, P2> : k_particles<T, true, true, SIPF_EM, P2>,
                              g, b, shm, s, pd, items, nitems, win_bytes, (uint32_t*)nullptr);
        }
    } else if (deposit) {
        launch_kernel((k_particles<T, true, false, SIPF_STRANG, P2>), g, b, shm, s, pd, items, nitems, win_bytes,
                      (uint32_t*)nullptr);
    } else if (push) {
        launch_kernel(strang ? k_particles<T, false, true, SIPF_STRANG, P2> : k_particles<T, false, true, SIPF_EM, P2>, g,
                      b, shm, s, pd, items, nitems, win_bytes, (uint32_t*)nullptr);
    }
}

template <typename T>
hipError_t launch_particles(const PartDesc<T>* pd, const WorkItem* items, int* nitems, int grid, bool deposit,
                            bool push, int scheme, int win_bytes, bool pow2, bool sorted, hipStream_t s,
                            uint32_t* kcounts) {
    if (grid <= 0) return hipSuccess;
    if (pow2) particles_p2<T, true>(pd, items, nitems, dim3(grid), deposit, push, scheme, win_bytes, sorted, kcounts, s);
    else particles_p2<T, false>(pd, items, nitems, dim3(grid), deposit, push, scheme, win_bytes, sorted, kcounts, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile sort: histogram, scan, combine, scatter -- for a group of instances
//
// The sort chunk table lists (instance, first particle) for every run of
// SORT_CHUNK particles of every instance.  Counts and cursors hold MAX_KEYS
// entries per instance.  The scan writes each instance's work items into its
// own segment; the combine pass concatenates the segments into one list that
// the (persistent) particle pass walks.
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(SORT_THREADS) void k_tile_hist(const PartDesc<T>* __restrict__ pds,
                                                            const SortChunk* __restrict__ chunks,
                                                            uint32_t* counts) {
    __shared__ uint32_t h[MAX_KEYS];
    const SortChunk ch = chunks[blockIdx.x];
    const PartDesc<T> a = pds[ch.inst];
    const int nk = a.nkeys;
    const int tid = threadIdx.x;
    const int64_t end = min(ch.beg + (int64_t)SORT_CHUNK, a.P);
    // all loads first (lanes past the end re-read the chunk's first particle),
    // so that the chunk costs one memory round trip, overlapped with the
    // clearing of the histogram
    T px[SORT_PER_THREAD], py[SORT_PER_THREAD], pz[SORT_PER_THREAD];
#pragma unroll
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const int64_t i = ch.beg + tid + (int64_t)k * SORT_THREADS;
        const int64_t j = i < end ? i : ch.beg;
        px[k] = gp(a.x)[j];
        py[k] = gp(a.y)[j];
        pz[k] = DIM == 3 ? gp(a.z)[j] : (T)0;
    }
    for (int i = tid; i < nk; i += SORT_THREADS) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const bool ok = ch.beg + tid + (int64_t)k * SORT_THREADS < end;
        const uint32_t key = ok ? key_of<T, DIM>(a, px[k], py[k], pz[k]) : 0xFFFFFFFFu;
        int head;
        const uint32_t len = lane_runs(key, head);
        if (ok && len) atomicAdd(&h[key], len);
    }
    __syncthreads();
    uint32_t* cnt = counts + (size_t)ch.inst * MAX_KEYS;
    for (int i = tid; i < nk; i += SORT_THREADS)
        if (h[i]) atomicAdd(&cnt[i], h[i]);
}

// Block-wide exclusive scans of NV values per thread (1024 threads = 16
// waves): inclusive scans inside each wave with lane shuffles, the wave
// totals through LDS (part: at least 16 NV words), one barrier between.
// totals[v] receives the block sum of value v.
template <int NV>
__device__ __forceinline__ void block_exclusive_scan_n(uint32_t* v, uint32_t* part, uint32_t* totals) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t inc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) inc[q] = v[q];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const uint32_t u = __shfl_up(inc[q], off, 64);
            if (lane >= off) inc[q] += u;
        }
    }
    __syncthreads();  // part may still be read by a previous scan
    if (lane == 63)
#pragma unroll
        for (int q = 0; q < NV; ++q) part[q * 16 + w] = inc[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        uint32_t before = 0, all = 0;
        for (int k = 0; k < 16; ++k) {
            const uint32_t t = part[q * 16 + k];
            before += k < w ? t : 0u;
            all += t;
        }
        totals[q] = all;
        v[q] = before + inc[q] - v[q];
    }
}

// Block-wide exclusive scan of one value per thread (1024 threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* part, uint32_t& total) {
    uint32_t x[1] = {v}, t[1];
    block_exclusive_scan_n<1>(x, part, t);
    total = t[0];
    return x[0];
}

// One workgroup per instance: exclusive scan of the tile counts into the
// cursors (tile starts) and the instance's work items (each non-empty tile
// split into ceil(count / chunk) contiguous items of near-equal size) into
// its segment of `seg`.  Items of at least chunk / 2 particles come first and
// the single items of sparser tiles last, so that the persistent passes, which
// draw items in list order, end on the small ones.  Clears the counts for the
// next sort.  DIRECT (a single instance): the segment is the item list itself
// and the scan writes its count, so no combine pass follows.
template <typename T, bool DIRECT>
__global__ __launch_bounds__(1024) void k_tile_scan(const PartDesc<T>* __restrict__ pds, uint32_t* counts,
                                                    uint32_t* cursor, WorkItem* seg, const int* __restrict__ seg_off,
                                                    int* seg_n, int chunk, int* nitems) {
    __shared__ uint32_t part[1024];
    const int inst = blockIdx.x;
    const int nk = pds[inst].nkeys;
    uint32_t* cnt = counts + (size_t)inst * MAX_KEYS;
    uint32_t* cur = cursor + (size_t)inst * MAX_KEYS;
    WorkItem* items = DIRECT ? seg : seg + seg_off[inst];
    const int tid = threadIdx.x;
    constexpr int PER = MAX_KEYS / 1024;  // keys per thread, consecutive in key order
    const uint32_t half = ((uint32_t)chunk + 1u) / 2u;
    static_assert(PER == 4, "one 16-byte load of counts per thread");
    uint32_t loc[PER], nit[PER];
    uint32_t sum = 0, ibig = 0, ismall = 0;
    // the instance's MAX_KEYS counts are 16-byte aligned: one load per thread
    const uint4 c4 = reinterpret_cast<const uint4*>(cnt)[tid];
    const uint32_t cv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = tid * PER + j;
        loc[j] = i < nk ? cv[j] : 0u;
        nit[j] = (loc[j] + chunk - 1) / chunk;
        sum += loc[j];
        if (loc[j] >= half) ibig += nit[j];
        else if (loc[j] > 0) ismall += 1u;
    }
    uint32_t sc[3] = {sum, ibig, ismall}, tot[3];
    block_exclusive_scan_n<3>(sc, part, tot);
    if (tot[0] != (uint32_t)pds[inst].P) {
        // the counts do not add up to the particle count: list no work items
        // (the scatter drops what would land outside the array) and flag it
        for (int j = 0; j < PER; ++j) {
            const int i = tid * PER + j;
            if (i < nk) {
                cur[i] = (uint32_t)pds[inst].P;  // every scatter target lands past the end
                cnt[i] = 0u;
            }
        }
        if (tid == 0) {
            seg_n[inst] = 0;
            if constexpr (DIRECT) nitems[0] = 0;
            atomicOr(pds[inst].err, 4);
        }
        return;
    }
    const uint32_t tbig = tot[1], tsmall = tot[2];
    uint32_t run = sc[0];
    uint32_t rbig = sc[1];
    uint32_t rsmall = tbig + sc[2];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = tid * PER + j;
        if (i < nk) {
            cur[i] = run;
            cnt[i] = 0u;
            if (nit[j] > 0) {
                // nit items: the first rem of base + 1 particles, the rest of base
                const uint32_t base = loc[j] / nit[j], rem = loc[j] - base * nit[j];
                const bool big = loc[j] >= half;
                const uint32_t at = big ? rbig : rsmall;
                uint32_t b = run;
                for (uint32_t k = 0; k < nit[j]; ++k) {
                    const uint32_t c = base + (k < rem ? 1u : 0u);
                    WorkItem w;
                    w.beg = (int64_t)b;
                    w.cnt = (int32_t)c;
                    w.inst = inst;
                    items[at + k] = w;
                    b += c;
                }
                if (big) rbig += nit[j];
                else rsmall += 1u;
            }
        }
        run += loc[j];
    }
    if (tid == 0) {
        seg_n[inst] = (int)(tbig + tsmall);
        if constexpr (DIRECT) nitems[0] = (int)(tbig + tsmall);
    }
}

// Concatenate the instances' item segments into one list (one workgroup):
// list entry k belongs to the last instance whose start is <= k (binary
// search over the starts in LDS), so every copy is independent of the others.
__global__ __launch_bounds__(1024) void k_items_combine(const WorkItem* __restrict__ seg,
                                                        const int* __restrict__ seg_off, const int* __restrict__ seg_n,
                                                        int ninst, WorkItem* items, int* nitems) {
    __shared__ uint32_t part[1024];
    __shared__ int start[1024];
    __shared__ int from[1024];
    const int tid = threadIdx.x;
    const uint32_t v = tid < ninst ? (uint32_t)seg_n[tid] : 0u;
    const int o = tid < ninst ? seg_off[tid] : 0;
    uint32_t total;
    const uint32_t off = block_exclusive_scan(v, part, total);
    if (tid < ninst) {
        start[tid] = (int)off;
        from[tid] = o;
    }
    __syncthreads();
    for (int k = tid; k < (int)total; k += 1024) {
        int lo = 0, hi = ninst - 1;  // start[lo] <= k always holds (start[0] = 0)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        items[k] = seg[from[lo] + (k - start[lo])];
    }
    if (tid == 0) *nitems = (int)total;
}

template <typename T, int DIM>
__global__ __launch_bounds__(SORT_THREADS) void k_tile_scatter(const PartDesc<T>* __restrict__ src,
                                                               const PartDesc<T>* __restrict__ dst,
                                                               const SortChunk* __restrict__ chunks,
                                                               uint32_t* cursor) {
    __shared__ uint32_t lc[MAX_KEYS];  // counts of the chunk's keys, then their first slots
    const SortChunk ch = chunks[blockIdx.x];
    const PartDesc<T> a = src[ch.inst];
    const PartDesc<T> b = dst[ch.inst];
    const int nk = a.nkeys;
    uint32_t* cur = cursor + (size_t)ch.inst * MAX_KEYS;
    const int tid = threadIdx.x;
    T px[SORT_PER_THREAD], py[SORT_PER_THREAD], pz[SORT_PER_THREAD];
    uint32_t pid[SORT_PER_THREAD], key[SORT_PER_THREAD], rank[SORT_PER_THREAD];
    const int lane = tid & 63;
    const int64_t end = min(ch.beg + (int64_t)SORT_CHUNK, a.P);
    // all loads first (lanes past the end re-read the chunk's first particle)
#pragma unroll
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const int64_t i = ch.beg + tid + (int64_t)k * SORT_THREADS;
        const int64_t j = i < end ? i : ch.beg;
        px[k] = gp(a.x)[j];
        py[k] = gp(a.y)[j];
        pz[k] = DIM == 3 ? gp(a.z)[j] : (T)0;
        pid[k] = gp(a.id)[j];
    }
    for (int i = tid; i < nk; i += SORT_THREADS) lc[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        const bool ok = ch.beg + tid + (int64_t)k * SORT_THREADS < end;
        key[k] = ok ? key_of<T, DIM>(a, px[k], py[k], pz[k]) : 0xFFFFFFFFu;
        // rank inside the chunk's tile: one LDS atomic per run of equal keys
        int head;
        const uint32_t len = lane_runs(key[k], head);
        uint32_t base = 0u;
        if (ok && len) base = atomicAdd(&lc[key[k]], len);
        rank[k] = (uint32_t)__shfl((int)base, head, 64) + (uint32_t)(lane - head);
    }
    __syncthreads();
    for (int i = tid; i < nk; i += SORT_THREADS)
        if (lc[i]) lc[i] = atomicAdd(&cur[i], lc[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_PER_THREAD; ++k) {
        if (ch.beg + tid + (int64_t)k * SORT_THREADS < end) {
            const uint32_t d = lc[key[k]] + rank[k];
            if (d < (uint32_t)b.P) {
                gp(b.x)[d] = px[k];
                gp(b.y)[d] = py[k];
                if constexpr (DIM == 3) gp(b.z)[d] = pz[k];
                gp(b.id)[d] = pid[k];
            } else {
                atomicOr(b.err, 4);
            }
        }
    }
}

int sort_chunk() { return SORT_CHUNK; }

template <typename T>
hipError_t launch_sort(int dim, const PartDesc<T>* src, const PartDesc<T>* dst, const SortChunk* chunks, int nchunks,
                       int ninst, uint32_t* counts, uint32_t* cursor, WorkItem* seg, const int* seg_off, int* seg_n,
                       WorkItem* items, int* nitems, int chunk, hipStream_t s, bool counted) {
    if (chunk <= 0 || chunk > CH) chunk = CH;
    if (ninst < 1 || ninst > 1024 || (dim != 2 && dim != 3)) return hipErrorInvalidValue;
    if (!counted) {
        if (dim == 3) launch_kernel((k_tile_hist<T, 3>), dim3(nchunks), dim3(SORT_THREADS), 0, s, src, chunks, counts);
        else launch_kernel((k_tile_hist<T, 2>), dim3(nchunks), dim3(SORT_THREADS), 0, s, src, chunks, counts);
    }
    if (ninst == 1) {
        launch_kernel((k_tile_scan<T, true>), dim3(1), dim3(1024), 0, s, src, counts, cursor, items, seg_off, seg_n,
                      chunk, nitems);
    } else {
        launch_kernel((k_tile_scan<T, false>), dim3(ninst), dim3(1024), 0, s, src, counts, cursor, seg, seg_off,
                      seg_n, chunk, nitems);
        launch_kernel(k_items_combine, dim3(1), dim3(1024), 0, s, seg, seg_off, seg_n, ninst, items, nitems);
    }
    if (dim == 3)
        launch_kernel((k_tile_scatter<T, 3>), dim3(nchunks), dim3(SORT_THREADS), 0, s, src, dst, chunks, cursor);
    else
        launch_kernel((k_tile_scatter<T, 2>), dim3(nchunks), dim3(SORT_THREADS), 0, s, src, dst, chunks, cursor);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small kernels: layout conversion, test entry points
// ---------------------------------------------------------------------------
// P x DIM positions (row-major) -> SoA, wrapped into the box, ids 0..P-1
template <typename T, int DIM>
__global__ void k_load_positions(const T* __restrict__ xyz, int64_t P, T L, T halfL, T invL, T* x, T* y, T* z,
                                 uint32_t* id, int* err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const T a = xyz[DIM * i], b = xyz[DIM * i + 1];
    const T c = DIM == 3 ? xyz[DIM * i + 2] : (T)0;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(err, 2);
    x[i] = wrap_box(a, L, halfL, invL);
    y[i] = wrap_box(b, L, halfL, invL);
    if constexpr (DIM == 3) z[i] = wrap_box(c, L, halfL, invL);
    id[i] = (uint32_t)i;
}

template <typename T>
hipError_t launch_load_positions(const T* xyz, int64_t P, T L, PartDesc<T> pd, int* err, hipStream_t s) {
    const int nb = (int)((P + 255) / 256);
    if (pd.dim == 2)
        hipLaunchKernelGGL((k_load_positions<T, 2>), dim3(nb), dim3(256), 0, s, xyz, P, L, L / 2, (T)1 / L, pd.x,
                           pd.y, pd.z, pd.id, err);
    else
        hipLaunchKernelGGL((k_load_positions<T, 3>), dim3(nb), dim3(256), 0, s, xyz, P, L, L / 2, (T)1 / L, pd.x,
                           pd.y, pd.z, pd.id, err);
    return hipGetLastError();
}

// SoA in sorted order -> P x DIM row-major in original particle order
template <typename T, int DIM>
__global__ void k_unsort(const T* __restrict__ x, const T* __restrict__ y, const T* __restrict__ z,
                         const uint32_t* __restrict__ id, int64_t P, T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int64_t j = id[i];
    out[DIM * j] = x[i];
    out[DIM * j + 1] = y[i];
    if constexpr (DIM == 3) out[DIM * j + 2] = z[i];
}

template <typename T> hipError_t launch_unsort(const PartDesc<T>* pd, T* out, hipStream_t s) {
    const int nb = (int)((pd->P + 255) / 256);
    if (pd->dim == 2)
        hipLaunchKernelGGL((k_unsort<T, 2>), dim3(nb), dim3(256), 0, s, pd->x, pd->y, pd->z, pd->id, pd->P, out);
    else
        hipLaunchKernelGGL((k_unsort<T, 3>), dim3(nb), dim3(256), 0, s, pd->x, pd->y, pd->z, pd->id, pd->P, out);
    return hipGetLastError();
}

template <typename T> __global__ void k_fill(T* p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
template <typename T> hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nbl = (n + 255) / 256;
    const int nb = (int)(nbl < 4096 ? nbl : 4096);
    hipLaunchKernelGGL((k_fill<T>), dim3(nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename T>
__global__ void k_cells(const T* __restrict__ X, int64_t n, T hl, int32_t* cells) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 3; ++d) cells[3 * i + d] = ifloor(X[3 * i + d] * hl);
}
template <typename T> hipError_t launch_cells(const T* X, int64_t n, int, T hl, int32_t* cells, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_cells<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, hl, cells);
    return hipGetLastError();
}

template <typename T>
__global__ void k_philox_dbg(uint32_t k0, uint32_t k1, int64_t n, const uint32_t* __restrict__ ctr,
                             uint32_t* __restrict__ raw, T* __restrict__ normals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u32x4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    const u32x4 r = philox4x32_10(c, k0, k1);
    if (raw) {
        raw[4 * i] = r.v0;
        raw[4 * i + 1] = r.v1;
        raw[4 * i + 2] = r.v2;
        raw[4 * i + 3] = r.v3;
    }
    if (normals) {
        T z[6];
        normals6<3>(r, z);
        for (int j = 0; j < 6; ++j) normals[6 * i + j] = z[j];
    }
}
template <typename T>
hipError_t launch_philox_dbg(uint64_t seed, int64_t n, const uint32_t* ctr, uint32_t* raw, T* normals, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_philox_dbg<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t)seed,
                       (uint32_t)(seed >> 32), n, ctr, raw, normals);
    return hipGetLastError();
}

#define SIPF_INST(T)                                                                                              \
    template int particle_resident_blocks<T>(int, int, bool);                                                     \
    template hipError_t launch_particles<T>(const PartDesc<T>*, const WorkItem*, int*, int, bool, bool, int, \
                                            int, bool, bool, hipStream_t, uint32_t*);                             \
    template hipError_t launch_sort<T>(int, const PartDesc<T>*, const PartDesc<T>*, const SortChunk*, int, int,   \
                                       uint32_t*, uint32_t*, WorkItem*, const int*, int*, WorkItem*, int*, int,    \
                                       hipStream_t, bool);                                                         \
    template hipError_t launch_load_positions<T>(const T*, int64_t, T, PartDesc<T>, int*, hipStream_t);          \
    template hipError_t launch_unsort<T>(const PartDesc<T>*, T*, hipStream_t);                                    \
    template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                                              \
    template hipError_t launch_cells<T>(const T*, int64_t, int, T, int32_t*, hipStream_t);                        \
    template hipError_t launch_philox_dbg<T>(uint64_t, int64_t, const uint32_t*, uint32_t*, T*, hipStream_t);

SIPF_INST(float)
SIPF_INST(double)
template hipError_t launch_fill<int>(int*, int64_t, int, hipStream_t);

}  // namespace sipf
