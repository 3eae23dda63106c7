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
#include <climits>

#include "internal.h"
#include "pass_common.h"
#include "sipf.h"

namespace sipf {

// sum over the 32 nodes of Gamma_4 of phibar[node] * dF/dlambda (eq. 4ord)
// Nodes are read from P at ((i - ox) mod H, (j - oy) mod H, (k - oz) mod H) with
// row strides (Wy, Wz): the whole grid for o = 0, W = H, or a window of it.
template <typename T>
__device__ __forceinline__ void deposit_grad(const T* __restrict__ phibar, T x, T y, T z, T hl, int H, T& gx_, T& gy_,
                                             T& gz_, int ox = 0, int oy = 0, int oz = 0, int Wy = 0, int Wz = 0) {
    const int Hm = H - 1;
    if (Wy == 0) {
        Wy = H;
        Wz = H;
    }
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
        const int ix = (g[0] - 1 + i - ox) & Hm, iy = (g[1] - 1 + j - oy) & Hm, iz = (g[2] - 1 + k - oz) & Hm;
        return phibar[((size_t)ix * Wy + iy) * Wz + iz];
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

// ---------------------------------------------------------------------------
// Reverse particle pass over the work items of a tile sort (one item = up to
// AdjShape<T>::PT x PPT particles of one tile, consecutive in the segment's order).  Per item,
// the cells of X bound a window of the grid that covers the trilinear stencil
// at Y = X + W^- (margin gmargin):
//   G window     the gradient grids, staged once from HBM (gather of v, J);
//   Gbar window  fixed-point accumulators of the transpose of the gather,
//                added to the grid once per item instead of once per particle;
//   phibar window the deposit cotangent.
// A particle whose Y cell leaves the window, or an item whose window does not
// fit, goes straight to HBM (gathers, float atomics).  The transpose of the
// deposit at X gathers the deposit cotangent from a third window (order-4
// stencil around the cells of X).
// ---------------------------------------------------------------------------
// Launch shape per precision: threads per workgroup and particles per thread
// (an item holds up to PT x PPT particles).  The pass needs ~166 VGPRs: one
// 768-thread workgroup is three waves per SIMD (measured FP32 forward +
// adjoint 37.6 against 38.7 ms with 512 threads); FP64 at 768 threads would
// spill, so it keeps 512 (two waves per SIMD).
template <typename T> struct AdjShape;
template <> struct AdjShape<float> { static constexpr int PT = 768, PPT = 6; };
template <> struct AdjShape<double> { static constexpr int PT = 512, PPT = 8; };
#ifndef ADJ_UNROLL
#define ADJ_UNROLL 1
#endif
#ifndef ADJ_BATCH
#define ADJ_BATCH 4
#endif

// Gbar accumulator: a term t (already scaled by 2^S) is added as round(t); S is
// chosen per item so that every node sum stays below 2^E in magnitude.
template <typename T> struct AdjFixed;
template <> struct AdjFixed<float> {
    using I = int32_t;
    using U = uint32_t;
    static constexpr int E = 30;
    __device__ static U q(float t) { return (U)(int32_t)rintf(t); }
};
template <> struct AdjFixed<double> {
    using I = long long;
    using U = unsigned long long;
    static constexpr int E = 50;
    __device__ static U q(double t) { return (U)Magic<double>::take(t + Magic<double>::M); }
};

int adj_window_bytes(bool fp64) { return fp64 ? 150 * 1024 : 76 * 1024; }

template <typename T, int SCHEME>
__device__ __forceinline__ void adj_item(const AdjDesc<T>& a, int64_t beg, int cnt, unsigned char* lds, int lds_bytes,
                                         int* sh, double& chib, double& sb) {
    using I = typename AdjFixed<T>::I;
    using U = typename AdjFixed<T>::U;
    constexpr int APT = AdjShape<T>::PT, APPT = AdjShape<T>::PPT;
    const int tid = threadIdx.x;
    const int H = a.H, Hm = H - 1, Hh = H / 2;
    const T hl = a.hl;
    const size_t H3 = (size_t)H * H * H;
    // the load phase keeps the particles only long enough for the bounding box
    // and the cotangent bound; the main loop re-reads each one from L2
    if (tid < 3) sh[tid] = INT_MAX;
    else if (tid < 6) sh[tid] = INT_MIN;
    else if (tid == 6) sh[6] = 0;
    __syncthreads();
    const int rx = ifloor(a.x[beg] * hl) & Hm, ry = ifloor(a.y[beg] * hl) & Hm, rz = ifloor(a.z[beg] * hl) & Hm;
    int mnx = INT_MAX, mny = INT_MAX, mnz = INT_MAX, mxx = INT_MIN, mxy = INT_MIN, mxz = INT_MIN;
    float bmax = 0.f;
    // in batches of ADJ_BATCH particles per thread, to bound the registers held
    constexpr int NB = APPT < ADJ_BATCH ? APPT : ADJ_BATCH;
#pragma unroll
    for (int k0 = 0; k0 < APPT; k0 += NB) {
        T px[NB], py[NB], pz[NB], qx[NB], qy[NB], qz[NB];
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
            const int j = tid + (k0 + kk) * APT;
            const uint32_t jj = (uint32_t)(j < cnt ? j : cnt - 1);  // in-item index for every lane: branch-free loads
            px[kk] = gp(a.x + beg)[jj];
            py[kk] = gp(a.y + beg)[jj];
            pz[kk] = gp(a.z + beg)[jj];
            qx[kk] = gp(a.xbx + beg)[jj];
            qy[kk] = gp(a.xby + beg)[jj];
            qz[kk] = gp(a.xbz + beg)[jj];
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
            const int j = tid + (k0 + kk) * APT;
            if (j < cnt) {
                const int cx = (((ifloor(px[kk] * hl) & Hm) - rx + Hh) & Hm) - Hh;
                const int cy = (((ifloor(py[kk] * hl) & Hm) - ry + Hh) & Hm) - Hh;
                const int cz = (((ifloor(pz[kk] * hl) & Hm) - rz + Hh) & Hm) - Hh;
                mnx = min(mnx, cx); mxx = max(mxx, cx);
                mny = min(mny, cy); mxy = max(mxy, cy);
                mnz = min(mnz, cz); mxz = max(mxz, cz);
                // |x| rounded up to float (values beyond float range give +inf)
                const float m3 =
                    (float)fmax(fmax(fabs((double)qx[kk]), fabs((double)qy[kk])), fabs((double)qz[kk]));
                bmax = fmaxf(bmax, m3 * 1.0000002f);
            }
        }
    }
    mnx = wave_min(mnx); mny = wave_min(mny); mnz = wave_min(mnz);
    mxx = wave_max(mxx); mxy = wave_max(mxy); mxz = wave_max(mxz);
    int bm = __float_as_int(bmax);  // non-negative floats order like their bit patterns
    bm = wave_max(bm);
    if ((tid & 63) == 0) {
        atomicMin(&sh[0], mnx); atomicMin(&sh[1], mny); atomicMin(&sh[2], mnz);
        atomicMax(&sh[3], mxx); atomicMax(&sh[4], mxy); atomicMax(&sh[5], mxz);
        atomicMax(&sh[6], bm);
    }
    __syncthreads();

    // window geometry (uniform across the workgroup)
    const double bound = (double)cnt * (double)a.chitau * (double)__int_as_float(sh[6]);
    int gox = 0, goy = 0, goz = 0, gWx = H, gWy = H, gWz = H;
    bool gwin = false;
    if (bound < 1e300) {
        for (int m = a.gmargin; m >= 0 && !gwin; --m) {
            axis_window(rx, sh[0] - m, sh[3] + 1 + m, H, gox, gWx);
            axis_window(ry, sh[1] - m, sh[4] + 1 + m, H, goy, gWy);
            axis_window(rz, sh[2] - m, sh[5] + 1 + m, H, goz, gWz);
            gwin = 3 * (int64_t)gWx * gWy * gWz * (int64_t)(sizeof(I) + sizeof(T)) <= lds_bytes;
        }
    }
    const int gn = gwin ? gWx * gWy * gWz : 0;
    I* Gb = reinterpret_cast<I*>(lds);
    T* Gw = reinterpret_cast<T*>(lds + (size_t)3 * gn * sizeof(I));
    // deposit-cotangent window: the order-4 stencil (-1 .. +2) around the cells of X
    const size_t used = (size_t)3 * gn * (sizeof(I) + sizeof(T));
    int dox = 0, doy = 0, doz = 0, dWx = H, dWy = H, dWz = H;
    bool dwin = false;
    if (a.phibar != nullptr) {
        axis_window(rx, sh[0] - 1, sh[3] + 2, H, dox, dWx);
        axis_window(ry, sh[1] - 1, sh[4] + 2, H, doy, dWy);
        axis_window(rz, sh[2] - 1, sh[5] + 2, H, doz, dWz);
        dwin = used + (size_t)dWx * dWy * dWz * sizeof(T) <= (size_t)lds_bytes;
    }
    T* Pw = reinterpret_cast<T*>(lds + used);
    if (dwin) {
        const int dn = dWx * dWy * dWz;
        const float inv_y = 1.0f / (float)dWy, inv_z = 1.0f / (float)dWz;
        for (int e = tid; e < dn; e += APT) {
            int i, j, k;
            unflatten3(e, dWy, dWz, inv_z, inv_y, i, j, k);
            Pw[e] = gp(a.phibar)[((size_t)((dox + i) & Hm) * H + ((doy + j) & Hm)) * H + ((doz + k) & Hm)];
        }
    }
    const T cdep = a.wmass * hl;
    if (gwin) {
        const float inv_y = 1.0f / (float)gWy, inv_z = 1.0f / (float)gWz;
        for (int e = tid; e < gn; e += APT) {
            int i, j, k;
            unflatten3(e, gWy, gWz, inv_z, inv_y, i, j, k);
            const size_t node = ((size_t)((gox + i) & Hm) * H + ((goy + j) & Hm)) * H + ((goz + k) & Hm);
            Gw[e] = gp(a.G)[node];
            Gw[gn + e] = gp(a.G)[H3 + node];
            Gw[2 * gn + e] = gp(a.G)[2 * H3 + node];
            Gb[e] = 0;
            Gb[gn + e] = 0;
            Gb[2 * gn + e] = 0;
        }
    }
    int e2 = 0;
    if (bound > 0 && gwin) (void)frexp(bound, &e2);  // bound < 2^e2
    const T scale = (T)ldexp(1.0, AdjFixed<T>::E - e2);
    const T back = (T)ldexp(1.0, e2 - AdjFixed<T>::E);
    __syncthreads();

#pragma unroll ADJ_UNROLL
    for (int k = 0; k < APPT; ++k) {
        const int j = tid + k * APT;
        if (j >= cnt) continue;
        const T X[3] = {gp(a.x + beg)[j], gp(a.y + beg)[j], gp(a.z + beg)[j]};
        const T xb[3] = {gp(a.xbx + beg)[j], gp(a.xby + beg)[j], gp(a.xbz + beg)[j]};
        const uint32_t pidk = gp(a.id + beg)[j];
        T zm[3], zp[3], Y[3], zn[6];
        if (a.zin != nullptr) {
            // the normals kept by the segment's forward recompute
#pragma unroll
            for (int q = 0; q < 6; ++q)
                zn[q] = (SCHEME == SIPF_STRANG || q < 3) ? gp(a.zin + q * a.P + beg)[j] : (T)0;
        } else if (SCHEME == SIPF_STRANG) {
            noise6<3, T>(pidk, a.n, a.inst, a.k0, a.k1, zn);
        } else {
            noise6<2, T>(pidk, a.n, a.inst, a.k0, a.k1, zn);
        }
        if (SCHEME == SIPF_STRANG) {
            for (int d = 0; d < 3; ++d) {
                zm[d] = zn[d];
                zp[d] = zn[3 + d];
                Y[d] = X[d] + a.s * zm[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                zp[d] = zn[d];
                zm[d] = 0;
                Y[d] = X[d];
            }
        }
        int gc[3];
        T w[3][2];
        for (int d = 0; d < 3; ++d) {
            const T sv = Y[d] * hl;
            const T f = floor(sv);
            gc[d] = (int)f;
            w[d][1] = sv - f;
            w[d][0] = (T)1 - w[d][1];
        }
        const int i0 = (gc[0] - gox) & Hm, j0 = (gc[1] - goy) & Hm, k0 = (gc[2] - goz) & Hm;
        const bool inside = gwin && (gWx == H || i0 <= gWx - 2) && (gWy == H || j0 <= gWy - 2) &&
                            (gWz == H || k0 <= gWz - 2);
        // node offsets: in the window, or in the whole grid
        int off[8];
        {
            int q = 0;
            for (int ia = 0; ia < 2; ++ia)
                for (int ib = 0; ib < 2; ++ib)
                    for (int ic = 0; ic < 2; ++ic, ++q) {
                        if (inside)
                            off[q] = (((gc[0] + ia - gox) & Hm) * gWy + ((gc[1] + ib - goy) & Hm)) * gWz +
                                     ((gc[2] + ic - goz) & Hm);
                        else
                            off[q] = (((gc[0] + ia) & Hm) * H + ((gc[1] + ib) & Hm)) * H + ((gc[2] + ic) & Hm);
                    }
        }
        // gradient values at the 8 nodes: from the LDS window or from HBM (two
        // explicit paths, so that LDS reads stay ds_read instructions)
        T gv[3][8];
        if (inside) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int d = 0; d < 3; ++d) gv[d][q] = Gw[d * gn + off[q]];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int d = 0; d < 3; ++d) gv[d][q] = gp(a.G)[d * H3 + off[q]];
        }
        T v[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, wt[8];
        {
            int q = 0;
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                    for (int ic = 0; ic < 2; ++ic, ++q) {
                        const T wyz = w[1][ib] * w[2][ic], wxz = w[0][ia] * w[2][ic], wxy = w[0][ia] * w[1][ib];
                        wt[q] = w[0][ia] * wyz;
                        const T dx = (ia ? hl : -hl) * wyz;
                        const T dy = (ib ? hl : -hl) * wxz;
                        const T dz = (ic ? hl : -hl) * wxy;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            v[d] += wt[q] * gv[d][q];
                            J[d][0] += dx * gv[d][q];
                            J[d][1] += dy * gv[d][q];
                            J[d][2] += dz * gv[d][q];
                        }
                    }
        }
        chib += (double)(a.tau * (xb[0] * v[0] + xb[1] * v[1] + xb[2] * v[2]));
        T vb[3], yb[3];
        for (int d = 0; d < 3; ++d) vb[d] = a.chitau * xb[d];
        for (int e = 0; e < 3; ++e) yb[e] = xb[e] + vb[0] * J[0][e] + vb[1] * J[1][e] + vb[2] * J[2][e];
        if (SCHEME == SIPF_STRANG)
            sb += (double)(xb[0] * zp[0] + xb[1] * zp[1] + xb[2] * zp[2] + yb[0] * zm[0] + yb[1] * zm[1] +
                           yb[2] * zm[2]);
        else
            sb += (double)(xb[0] * zp[0] + xb[1] * zp[1] + xb[2] * zp[2]);
        // transpose of the gather: vbar spread with the trilinear weights at Y
        if (inside) {
            const T vs[3] = {vb[0] * scale, vb[1] * scale, vb[2] * scale};
            for (int q = 0; q < 8; ++q)
                for (int d = 0; d < 3; ++d)
                    atomicAdd(reinterpret_cast<U*>(Gb + d * gn + off[q]), AdjFixed<T>::q(wt[q] * vs[d]));
        } else {
            for (int q = 0; q < 8; ++q)
                for (int d = 0; d < 3; ++d) gatomic_add(a.Gbar + d * H3 + off[q], wt[q] * vb[d]);
        }
        // transpose of the deposit at X
        if (a.phibar != nullptr) {
            T gx, gy, gz;
            if (dwin) deposit_grad(Pw, X[0], X[1], X[2], hl, H, gx, gy, gz, dox, doy, doz, dWy, dWz);
            else deposit_grad(a.phibar, X[0], X[1], X[2], hl, H, gx, gy, gz);
            yb[0] += cdep * gx;
            yb[1] += cdep * gy;
            yb[2] += cdep * gz;
        }
        gp(a.xbx + beg)[j] = yb[0];
        gp(a.xby + beg)[j] = yb[1];
        gp(a.xbz + beg)[j] = yb[2];
    }
    __syncthreads();
    if (gwin) {
        const float inv_y = 1.0f / (float)gWy, inv_z = 1.0f / (float)gWz;
        for (int e = tid; e < 3 * gn; e += APT) {
            const I val = Gb[e];
            if (val != 0) {
                const int d = e >= 2 * gn ? 2 : (e >= gn ? 1 : 0);
                int i, j, k;
                unflatten3(e - d * gn, gWy, gWz, inv_z, inv_y, i, j, k);
                const size_t node = ((size_t)((gox + i) & Hm) * H + ((goy + j) & Hm)) * H + ((goz + k) & Hm);
                gatomic_add(a.Gbar + d * H3 + node, (T)val * back);
            }
        }
    }
}

__device__ __forceinline__ double block_sum_n(double v, double* sh, int nthreads) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nthreads / 64; ++i) t += sh[i];
    return t;
}

// Register budget of the reverse pass: waves per SIMD to leave room for (0: the
// compiler's choice).
#ifndef ADJ_WAVES
#define ADJ_WAVES 0
#endif
#if ADJ_WAVES > 0
#define ADJ_ATTR __attribute__((amdgpu_waves_per_eu(ADJ_WAVES)))
#else
#define ADJ_ATTR
#endif
template <typename T, int SCHEME>
__global__ __launch_bounds__(AdjShape<T>::PT) ADJ_ATTR void k_adj_items(AdjDesc<T> a,
                                                                      const WorkItem* __restrict__ items, int* hdr,
                                                                      int lds_bytes) {
    constexpr int APT = AdjShape<T>::PT;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int sh[8];
    __shared__ int slot;
    __shared__ double shd[APT / 64];
    const int n = hdr[0];
    double chib = 0, sb = 0;
    for (int it = blockIdx.x; it < n; it = next_item(hdr, n, &slot)) {
        const WorkItem w = items[it];
        adj_item<T, SCHEME>(a, w.beg, w.cnt, lds, lds_bytes, sh, chib, sb);
    }
    __syncthreads();
    const double tc = block_sum_n(chib, shd, APT);
    const double ts = block_sum_n(sb, shd, APT);
    if (threadIdx.x == 0) {
        atomicAdd(a.acc, tc);
        atomicAdd(a.acc + 1, ts);
    }
}

template <typename T>
__global__ void k_copy_positions(T* x, T* y, T* z, uint32_t* id, const T* __restrict__ sx, const T* __restrict__ sy,
                                 const T* __restrict__ sz, const uint32_t* __restrict__ sid, int64_t P) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = sx[i];
        y[i] = sy[i];
        z[i] = sz[i];
        id[i] = sid[i];
    }
}

template <typename T>
__global__ void k_xbar_order(T* xbar, T* bx, T* by, T* bz, const uint32_t* __restrict__ id, int64_t P, int to_order) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const size_t p = id[i];
        if (to_order) {
            bx[i] = xbar[3 * p];
            by[i] = xbar[3 * p + 1];
            bz[i] = xbar[3 * p + 2];
        } else {
            xbar[3 * p] = bx[i];
            xbar[3 * p + 1] = by[i];
            xbar[3 * p + 2] = bz[i];
        }
    }
}

__global__ void k_iota_u32(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
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
template <typename T>
hipError_t launch_adj_items(const AdjDesc<T>& a, const WorkItem* items, int* nitems, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    constexpr int APT = AdjShape<T>::PT;
    if (particle_chunk() > APT * AdjShape<T>::PPT) return hipErrorInvalidValue;  // an item must fit one workgroup
    const int lds = adj_window_bytes(sizeof(T) == 8);
    if (a.scheme == SIPF_STRANG) {
        (void)hipFuncSetAttribute((const void*)k_adj_items<T, SIPF_STRANG>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        hipLaunchKernelGGL((k_adj_items<T, SIPF_STRANG>), dim3(grid), dim3(APT), lds, s, a, items, nitems, lds);
    } else {
        (void)hipFuncSetAttribute((const void*)k_adj_items<T, SIPF_EM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  lds);
        hipLaunchKernelGGL((k_adj_items<T, SIPF_EM>), dim3(grid), dim3(APT), lds, s, a, items, nitems, lds);
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_copy_positions(T* x, T* y, T* z, uint32_t* id, const T* sx, const T* sy, const T* sz,
                                 const uint32_t* sid, int64_t P, hipStream_t s) {
    hipLaunchKernelGGL((k_copy_positions<T>), dim3(grid_for(P)), dim3(256), 0, s, x, y, z, id, sx, sy, sz, sid, P);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_xbar_order(T* xbar, T* bx, T* by, T* bz, const uint32_t* id, int64_t P, bool to_order,
                             hipStream_t s) {
    hipLaunchKernelGGL((k_xbar_order<T>), dim3(grid_for(P)), dim3(256), 0, s, xbar, bx, by, bz, id, P,
                       to_order ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n);
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
    template hipError_t launch_adj_items<T>(const AdjDesc<T>&, const WorkItem*, int*, int, hipStream_t); \
    template hipError_t launch_copy_positions<T>(T*, T*, T*, uint32_t*, const T*, const T*, const T*,          \
                                                 const uint32_t*, int64_t, hipStream_t);                       \
    template hipError_t launch_xbar_order<T>(T*, T*, T*, T*, const uint32_t*, int64_t, bool, hipStream_t);     \
    template hipError_t launch_dot<T>(const T*, const T*, int64_t, double*, hipStream_t); \
    template hipError_t launch_axpby<T>(T*, const T*, T, T, int64_t, hipStream_t);
SIPF_ADJ_INST(float)
SIPF_ADJ_INST(double)

}  // namespace sipf
