// Particle pass of the two-dimensional step (the 2-D runs of Sec. 5.2): the
// 12-node fourth-order deposit of X^(n-1) (the construction of eq. 4ord with
// d = 2), the bilinear gather of grad c^(n-1) at Y = X + W^- and the split
// push (Algorithm 4), or the Euler-Maruyama push (eq. rho_hat_update).
//
// Same organisation as the 3-D pass: the tile sort (particles.hip, T^2-cell
// tiles) hands out work items of up to 4096 consecutive particles; a
// workgroup measures the item's bounding box of cells, deposits into an LDS
// window in fixed point with integer atomics and adds the window to the grid
// once, stages the gradient around the box (plus the W^- margin) in LDS, and
// pushes.  Items whose windows do not fit use the global grids directly.
//
// Noise: the Philox block of (id, n, 0, instance); split step W^- from
// (z0, z1) and W^+ from (z2, z3), Euler-Maruyama W from (z0, z1).
#include <climits>

#include "internal.h"
#include "pass_common.h"
#include "sipf.h"

namespace sipf {

constexpr int PT2 = 512;                 // threads per workgroup
constexpr int PPT2 = 8;                  // particles per thread; items hold at most PT2 * PPT2
constexpr int MIN_WINDOW_ITEM2 = 64;     // smaller items use the global grids

// the 12 nodes of the 2-D fourth-order stencil; sink(index, F) with
// index = row * Wy + column relative to the window origin (ox, oy)
template <typename T, typename Sink>
__device__ __forceinline__ void deposit2_one(Sink& sink, T x, T y, T hl, int Hm, int ox, int oy, int Wy) {
    const T sx = x * hl, sy = y * hl;
    const T fx = floor(sx), fy = floor(sy);
    const int gx = (int)fx, gy = (int)fy;
    const Axis4<T> ax = axis4(sx - fx), ay = axis4(sy - fy);
    const T S = (T)1 + (ax.w0 * ax.w1 + ay.w0 * ay.w1) * (T)0.5;
    int cx[4], cy[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        cx[j] = ((gx - 1 + j - ox) & Hm) * Wy;
        cy[j] = (gy - 1 + j - oy) & Hm;
    }
    const T wx[2] = {ax.w0, ax.w1}, wy[2] = {ay.w0, ay.w1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        // inner nodes (a, 0) and (a, 1)
        sink(cx[1 + a] + cy[1], wx[a] * wy[0] * S);
        sink(cx[1 + a] + cy[2], wx[a] * wy[1] * S);
        // outer nodes on x: (-1, a) and (2, a)
        sink(cx[0] + cy[1 + a], ax.wm * wy[a]);
        sink(cx[3] + cy[1 + a], ax.wp * wy[a]);
        // outer nodes on y: (a, -1) and (a, 2)
        sink(cx[1 + a] + cy[0], wx[a] * ay.wm);
        sink(cx[1 + a] + cy[3], wx[a] * ay.wp);
    }
}

template <typename T> struct LdsSink2 {
    typename Fixed<T>::I* win;
    T scale;
    __device__ __forceinline__ void operator()(int idx, T F) const {
        atomicAdd(reinterpret_cast<typename Fixed<T>::U*>(win + idx), (typename Fixed<T>::U)Fixed<T>::quant(F * scale));
    }
};
template <typename T> struct GlobalSink2 {
    T* phi;
    T m;
    __device__ __forceinline__ void operator()(int idx, T F) const { gatomic_add(phi + idx, F * m); }
};

// bilinear interpolation of two planar grids of node pitch n2 and row stride Wy
template <typename T, typename Ptr>
__device__ __forceinline__ void bilinear2(Ptr G, size_t n2, int Wy, const int* ix, const int* iy, T lx, T ly, T& vx,
                                          T& vy) {
    const T wx[2] = {(T)1 - lx, lx}, wy[2] = {(T)1 - ly, ly};
    vx = (T)0;
    vy = (T)0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const size_t node = (size_t)ix[a] * Wy + iy[b];
            const T w = wx[a] * wy[b];
            vx += w * G[node];
            vy += w * G[n2 + node];
        }
}

template <typename T, bool DEP, bool PUSH, int SCHEME>
__device__ __forceinline__ void item_pass2(const PartDesc<T>& a, int64_t beg, int cnt, unsigned char* lds,
                                           int win_bytes, int* sh) {
    using I = typename Fixed<T>::I;
    const int tid = threadIdx.x;
    const int H = a.H, Hm = H - 1, Hh = H / 2;
    const T hl = a.hl;
    const T* ix = a.x + beg;
    const T* iy = a.y + beg;
    const uint32_t* iid = a.id + beg;
    T px[PPT2], py[PPT2];
#pragma unroll
    for (int k = 0; k < PPT2; ++k) {
        const int j = tid + k * PT2;
        const uint32_t jj = (uint32_t)(j < cnt ? j : cnt - 1);
        px[k] = gp(ix)[jj];
        py[k] = gp(iy)[jj];
    }
    const bool windows = cnt >= MIN_WINDOW_ITEM2;
    int rx = 0, ry = 0;
    if (windows) {
        // bounding box of the item's cells, relative to the first particle's cell
        if (tid < 2) sh[tid] = INT_MAX;
        else if (tid < 4) sh[tid] = INT_MIN;
        __syncthreads();
        rx = ifloor(gp(a.x)[beg] * hl) & Hm;
        ry = ifloor(gp(a.y)[beg] * hl) & Hm;
        int mnx = INT_MAX, mny = INT_MAX, mxx = INT_MIN, mxy = INT_MIN;
#pragma unroll
        for (int k = 0; k < PPT2; ++k) {
            if (tid + k * PT2 < cnt) {
                const int cx = (((ifloor(px[k] * hl) & Hm) - rx + Hh) & Hm) - Hh;
                const int cy = (((ifloor(py[k] * hl) & Hm) - ry + Hh) & Hm) - Hh;
                mnx = min(mnx, cx);
                mxx = max(mxx, cx);
                mny = min(mny, cy);
                mxy = max(mxy, cy);
            }
        }
        mnx = wave_min(mnx);
        mny = wave_min(mny);
        mxx = wave_max(mxx);
        mxy = wave_max(mxy);
        if ((tid & 63) == 0) {
            atomicMin(&sh[0], mnx);
            atomicMin(&sh[1], mny);
            atomicMax(&sh[2], mxx);
            atomicMax(&sh[3], mxy);
        }
        __syncthreads();
    }

    if (DEP) {
        int ox = 0, oy = 0, Wx = H, Wy = H;
        bool use_win = false;
        if (windows) {
            // nodes -1..+2 around every cell of the box
            axis_window(rx, sh[0] - 1, sh[2] + 2, H, ox, Wx);
            axis_window(ry, sh[1] - 1, sh[3] + 2, H, oy, Wy);
            use_win = (int64_t)Wx * Wy * (int64_t)sizeof(I) <= win_bytes;
        }
        if (use_win) {
            I* win = reinterpret_cast<I*>(lds);
            const int nw = Wx * Wy;
            for (int e = tid; e < nw; e += PT2) win[e] = 0;
            // 2^S with S = BITS - bitlength(ceil(11 cnt / 8)): |sum of F| <= 1.375 cnt per node
            const int need = (11 * cnt + 7) / 8;
            const int S = Fixed<T>::BITS - (32 - __clz(need));
            const T scale = (T)ldexp(1.0, S);
            __syncthreads();
            LdsSink2<T> sink{win, scale};
#pragma unroll
            for (int k = 0; k < PPT2; ++k)
                if (tid + k * PT2 < cnt) deposit2_one(sink, px[k], py[k], hl, Hm, ox, oy, Wy);
            __syncthreads();
            const T back = a.wmass * (T)ldexp(1.0, -S);
            for (int e = tid; e < nw; e += PT2) {
                const I v = win[e];
                if (v != 0) {
                    const int ex = e / Wy, ey = e - ex * Wy;
                    gatomic_add(a.phi + (size_t)((ox + ex) & Hm) * H + ((oy + ey) & Hm), (T)v * back);
                }
            }
            __syncthreads();  // the window memory is reused below
        } else {
            GlobalSink2<T> sink{a.phi, a.wmass};
#pragma unroll
            for (int k = 0; k < PPT2; ++k)
                if (tid + k * PT2 < cnt) deposit2_one(sink, px[k], py[k], hl, Hm, 0, 0, H);
        }
    }

    if (PUSH) {
        // gradient window: cells of the box (+ margin for the W^- displacement) and +1 for the bilinear reach
        int ox = 0, oy = 0, Wx = H, Wy = H;
        bool use_win = false;
        size_t n2 = 0;
        if (windows) {
            for (int m = a.gmargin; m >= 0 && !use_win; --m) {
                axis_window(rx, sh[0] - m, sh[2] + 1 + m, H, ox, Wx);
                axis_window(ry, sh[1] - m, sh[3] + 1 + m, H, oy, Wy);
                use_win = 2 * (int64_t)Wx * Wy * (int64_t)sizeof(T) <= win_bytes;
            }
            if (use_win) {
                T* Gw = reinterpret_cast<T*>(lds);
                const int nw = Wx * Wy;
                n2 = (size_t)nw;
                const size_t HH2 = (size_t)H * H;
                for (int e = tid; e < nw; e += PT2) {
                    const int ex = e / Wy, ey = e - ex * Wy;
                    const size_t node = (size_t)((ox + ex) & Hm) * H + ((oy + ey) & Hm);
                    Gw[e] = gp(a.G)[node];
                    Gw[nw + e] = gp(a.G)[HH2 + node];
                }
                __syncthreads();
            }
        }
        const T* Gl = reinterpret_cast<const T*>(lds);
        const uint32_t n = *a.step + 1u;
        const size_t HH2 = (size_t)H * H;
#pragma unroll 4
        for (int k = 0; k < PPT2; ++k) {
            const int j = tid + k * PT2;
            if (j >= cnt) continue;
            const T x = gp(ix)[j], y = gp(iy)[j];
            const uint32_t idk = gp(iid)[j];
            T yx, yy, w0, w1;
            T zn[6];
            if (SCHEME == SIPF_STRANG) {
                noise6<2, T>(idk, n, a.inst, a.k0, a.k1, zn);
                yx = x + a.s * zn[0];
                yy = y + a.s * zn[1];
                w0 = zn[2];
                w1 = zn[3];
            } else {
                noise6<1, T>(idk, n, a.inst, a.k0, a.k1, zn);
                w0 = zn[0];
                w1 = zn[1];
                yx = x;
                yy = y;
            }
            const T sx = yx * hl, sy = yy * hl;
            const T fx = floor(sx), fy = floor(sy);
            const int gx = (int)fx, gy = (int)fy;
            int cxs[2] = {(gx - ox) & Hm, (gx + 1 - ox) & Hm};
            int cys[2] = {(gy - oy) & Hm, (gy + 1 - oy) & Hm};
            T vx, vy;
            const bool inside = use_win && (Wx == H || cxs[0] <= Wx - 2) && (Wy == H || cys[0] <= Wy - 2);
            if (inside) {
                bilinear2<T>(Gl, n2, Wy, cxs, cys, sx - fx, sy - fy, vx, vy);
            } else {
                cxs[0] = gx & Hm;
                cxs[1] = (gx + 1) & Hm;
                cys[0] = gy & Hm;
                cys[1] = (gy + 1) & Hm;
                bilinear2<T>(gp(a.G), HH2, H, cxs, cys, sx - fx, sy - fy, vx, vy);
            }
            const T nx = wrap_box(yx + a.chitau * vx + a.s * w0, a.L, a.halfL, a.invL);
            const T ny = wrap_box(yy + a.chitau * vy + a.s * w1, a.L, a.halfL, a.invL);
            gp(a.x + beg)[j] = nx;
            gp(a.y + beg)[j] = ny;
            if (!(isfinite(nx) && isfinite(ny))) atomicOr(a.err, 1);
        }
    }
}

// Persistent over the work items listed by the last sort (header: next_item).
template <typename T, bool DEP, bool PUSH, int SCHEME>
__global__ __launch_bounds__(PT2) void k_particles2(const PartDesc<T>* __restrict__ pds,
                                                    const WorkItem* __restrict__ items, int* hdr, int win_bytes) {
    extern __shared__ __align__(16) unsigned char smem_raw2[];
    __shared__ int sh[4];
    __shared__ int slot;
    const int n = hdr[0];
    for (int it = blockIdx.x; it < n; it = next_item(hdr, n, &slot)) {
        const WorkItem w = items[it];
        item_pass2<T, DEP, PUSH, SCHEME>(pds[w.inst], w.beg, w.cnt, smem_raw2, win_bytes, sh);
    }
}

template <typename T> int particle_resident_blocks2(int scheme, int win_bytes) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = scheme == SIPF_STRANG
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, (const void*)k_particles2<T, true, true, SIPF_STRANG>, PT2, win_bytes)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, (const void*)k_particles2<T, true, true, SIPF_EM>, PT2, win_bytes);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || per_cu < 1 || cus < 1) {
        (void)hipGetLastError();
        return 1024;
    }
    return per_cu * cus;
}

template <typename T>
hipError_t launch_particles2(const PartDesc<T>* pd, const WorkItem* items, int* nitems, int grid, bool deposit,
                             bool push, int scheme, int win_bytes, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    const size_t shm = (size_t)win_bytes;
    const dim3 g(grid), b(PT2);
    if (deposit && push) {
        if (scheme == SIPF_STRANG)
            launch_kernel((k_particles2<T, true, true, SIPF_STRANG>), g, b, shm, s, pd, items, nitems, win_bytes);
        else
            launch_kernel((k_particles2<T, true, true, SIPF_EM>), g, b, shm, s, pd, items, nitems, win_bytes);
    } else if (deposit) {
        launch_kernel((k_particles2<T, true, false, SIPF_STRANG>), g, b, shm, s, pd, items, nitems, win_bytes);
    } else if (push) {
        if (scheme == SIPF_STRANG)
            launch_kernel((k_particles2<T, false, true, SIPF_STRANG>), g, b, shm, s, pd, items, nitems, win_bytes);
        else
            launch_kernel((k_particles2<T, false, true, SIPF_EM>), g, b, shm, s, pd, items, nitems, win_bytes);
    }
    return hipGetLastError();
}

template int particle_resident_blocks2<float>(int, int);
template int particle_resident_blocks2<double>(int, int);
template hipError_t launch_particles2<float>(const PartDesc<float>*, const WorkItem*, int*, int, bool, bool, int,
                                             int, hipStream_t);
template hipError_t launch_particles2<double>(const PartDesc<double>*, const WorkItem*, int*, int, bool, bool,
                                              int, int, hipStream_t);

}  // namespace sipf
