// In-place LDS FFT building blocks shared by the 3-D and 2-D field passes.
//
// Length N = N1 * N2 (N1, N2 <= 23): a stage of N1-point register DFTs with
// twiddles, then a stage of N2-point register DFTs.  The forward transform
// takes natural order and leaves frequency k at position
// (k mod N1) * N2 + k div N1; the inverse takes that order and returns
// natural order.  A register DFT of even length splits into two halves
// (radix 2); one of odd length is summed directly, pairing the terms j and
// R - j, with cosines and sines fixed at compile time.  Lengths with odd
// factors (12, 22, 46, 90 and their halves) serve grids that are not powers
// of two.
//
// Lengths 512 .. 4096 (N = 16 M, M <= 256) add a first stage: 16-point DFTs
// across the 16 blocks of M elements with twiddles w_N^(m k1), then the
// M-point two-stage transform of every block; frequency k1 + 16 k' sits at
// position k1 M + pos_M(k').  The inverse runs the stages in reverse order.
#pragma once

#include "common.h"

namespace sipf {

template <int N> struct Split;
template <> struct Split<4>   { static constexpr int N1 = 4,  N2 = 1; };
template <> struct Split<8>   { static constexpr int N1 = 8,  N2 = 1; };
template <> struct Split<16>  { static constexpr int N1 = 16, N2 = 1; };
template <> struct Split<32>  { static constexpr int N1 = 8,  N2 = 4; };
template <> struct Split<64>  { static constexpr int N1 = 8,  N2 = 8; };
template <> struct Split<128> { static constexpr int N1 = 16, N2 = 8; };
template <> struct Split<256> { static constexpr int N1 = 16, N2 = 16; };
// lengths with odd factors
template <> struct Split<3>   { static constexpr int N1 = 3,  N2 = 1; };
template <> struct Split<5>   { static constexpr int N1 = 5,  N2 = 1; };
template <> struct Split<6>   { static constexpr int N1 = 6,  N2 = 1; };
template <> struct Split<11>  { static constexpr int N1 = 11, N2 = 1; };
template <> struct Split<12>  { static constexpr int N1 = 12, N2 = 1; };
template <> struct Split<22>  { static constexpr int N1 = 11, N2 = 2; };
template <> struct Split<23>  { static constexpr int N1 = 23, N2 = 1; };
template <> struct Split<45>  { static constexpr int N1 = 9,  N2 = 5; };
template <> struct Split<46>  { static constexpr int N1 = 23, N2 = 2; };
template <> struct Split<90>  { static constexpr int N1 = 10, N2 = 9; };

// cos and sin of 2 pi m / R at compile time: the angle is reduced exactly to
// the nearest quarter turn q, leaving x = 2 pi (4m - qR) / (4R) with
// |x| <= pi / 4, where the Taylor series of cos and sin is summed far below
// double rounding (the 14th term is under 1e-30); then rotated by q quarters.
struct TrigC {
    static constexpr double PI = 3.14159265358979323846264338327950288;
    static constexpr double cos_s(double x) {
        double t = 1.0, r = 1.0;
        for (int n = 1; n < 14; ++n) {
            t *= -x * x / (double)((2 * n - 1) * (2 * n));
            r += t;
        }
        return r;
    }
    static constexpr double sin_s(double x) {
        double t = x, r = x;
        for (int n = 1; n < 14; ++n) {
            t *= -x * x / (double)((2 * n) * (2 * n + 1));
            r += t;
        }
        return r;
    }
    // want_sin ? sin : cos of 2 pi m / R
    static constexpr double cs(int m, int R, bool want_sin) {
        m %= R;
        if (m < 0) m += R;
        const int q = (8 * m + R) / (2 * R);  // nearest quarter, round(4m / R)
        const double x = 2.0 * PI * (double)(4 * m - q * R) / (4.0 * (double)R);
        const double c = cos_s(x), s = sin_s(x);
        switch (q & 3) {
            case 0: return want_sin ? s : c;
            case 1: return want_sin ? c : -s;
            case 2: return want_sin ? -s : -c;
            default: return want_sin ? -c : s;
        }
    }
};


// cos and sin of 2 pi j / 16, j = 0..7
struct Tw16 {
    static constexpr double c[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
    static constexpr double s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
};

// v * exp(DIR 2 pi i k / R)
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ cplx_t<T> twiddle(cplx_t<T> v) {
    using V = cplx_t<T>;
    if constexpr (K == 0) {
        return v;
    } else if constexpr (4 * K == R) {
        return DIR > 0 ? cmake<V, T>(-v.y, v.x) : cmake<V, T>(v.y, -v.x);
    } else if constexpr (16 % R == 0) {
        constexpr int j = K * (16 / R);
        const T c = (T)Tw16::c[j];
        const T s = (T)(DIR * Tw16::s[j]);
        return cmake<V, T>(v.x * c - v.y * s, v.x * s + v.y * c);
    } else {
        constexpr double cd = TrigC::cs(K, R, false), sd = TrigC::cs(K, R, true);
        const T c = (T)cd;
        const T s = (T)(DIR * sd);
        return cmake<V, T>(v.x * c - v.y * s, v.x * s + v.y * c);
    }
}

// compile-time table of cos and sin of 2 pi m / R, m = 0 .. R - 1
template <int R> struct TrigTab {
    double c[R], s[R];
    constexpr TrigTab() : c(), s() {
        for (int m = 0; m < R; ++m) {
            c[m] = TrigC::cs(m, R, false);
            s[m] = TrigC::cs(m, R, true);
        }
    }
};

// In-register DFT of length R, natural order in and out: X_k = sum_j x_j
// exp(DIR 2 pi i j k / R).
template <typename T, int R, int DIR, bool EVEN = (R % 2 == 0)> struct Dft;

// odd R: X_0 = sum_j x_j; for 0 < k <= (R - 1) / 2, with a_j = x_j + x_{R-j}
// and b_j = x_j - x_{R-j},
//   X_k, X_{R-k} = x_0 + sum_j a_j cos(2 pi j k / R) +- DIR i sum_j b_j sin(2 pi j k / R)
template <typename T, int R, int DIR> struct Dft<T, R, DIR, false> {
    using V = cplx_t<T>;
    __device__ __forceinline__ static void run(V* x) {
        if constexpr (R > 1) {
            constexpr int Q = (R - 1) / 2;
            constexpr TrigTab<R> tab{};
            V a[Q], b[Q];
            const V x0 = x[0];
            V sum = x0;
#pragma unroll
            for (int j = 1; j <= Q; ++j) {
                a[j - 1] = cadd(x[j], x[R - j]);
                b[j - 1] = csub(x[j], x[R - j]);
                sum = cadd(sum, a[j - 1]);
            }
            x[0] = sum;
#pragma unroll
            for (int k = 1; k <= Q; ++k) {
                T sr = x0.x, si = x0.y, dr = 0, di = 0;
#pragma unroll
                for (int j = 1; j <= Q; ++j) {
                    const int m = (j * k) % R;
                    const T c = (T)tab.c[m], sn = (T)tab.s[m];
                    sr += a[j - 1].x * c;
                    si += a[j - 1].y * c;
                    dr += b[j - 1].x * sn;
                    di += b[j - 1].y * sn;
                }
                // DIR i (dr + i di) = DIR (-di + i dr)
                const T ir = (T)(-DIR) * di, ii = (T)DIR * dr;
                x[k] = cmake<V, T>(sr + ir, si + ii);
                x[R - k] = cmake<V, T>(sr - ir, si - ii);
            }
        }
    }
};

// even R: radix 2 over the even and odd samples
template <typename T, int R, int DIR> struct Dft<T, R, DIR, true> {
    using V = cplx_t<T>;
    template <int K>
    __device__ __forceinline__ static void combine(V* x, const V* e, const V* o) {
        if constexpr (K < R / 2) {
            const V t = twiddle<T, R, DIR, K>(o[K]);
            x[K] = cadd(e[K], t);
            x[K + R / 2] = csub(e[K], t);
            combine<K + 1>(x, e, o);
        }
    }
    __device__ __forceinline__ static void run(V* x) {
        V e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = x[2 * i];
            o[i] = x[2 * i + 1];
        }
        Dft<T, R / 2, DIR>::run(e);
        Dft<T, R / 2, DIR>::run(o);
        combine<0>(x, e, o);
    }
};

// count independent length-N transforms; element e of transform b at
// buf[b * bs + e * es].  tw[m] = exp(-2 pi i m / N).  Caller synchronises
// before and after.
template <typename T, int N, int DIR>
__device__ __forceinline__ void lds_fft(cplx_t<T>* buf, int count, int bs, int es, const cplx_t<T>* tw) {
    using V = cplx_t<T>;
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    const int tid = threadIdx.x, nt = blockDim.x;
    if constexpr (DIR < 0) {
        for (int u = tid; u < count * N2; u += nt) {
            const int b = u % count, n2 = u / count;
            V* p = buf + b * bs + n2 * es;
            V r[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) r[i] = p[i * N2 * es];
            Dft<T, N1, -1>::run(r);
            if constexpr (N2 > 1) {
#pragma unroll
                for (int k1 = 1; k1 < N1; ++k1) r[k1] = cmul(r[k1], tw[n2 * k1]);
            }
#pragma unroll
            for (int i = 0; i < N1; ++i) p[i * N2 * es] = r[i];
        }
        if constexpr (N2 > 1) {
            __syncthreads();
            for (int u = tid; u < count * N1; u += nt) {
                const int b = u % count, k1 = u / count;
                V* p = buf + b * bs + k1 * N2 * es;
                V r[N2];
#pragma unroll
                for (int i = 0; i < N2; ++i) r[i] = p[i * es];
                Dft<T, N2, -1>::run(r);
#pragma unroll
                for (int i = 0; i < N2; ++i) p[i * es] = r[i];
            }
        }
    } else {
        if constexpr (N2 > 1) {
            for (int u = tid; u < count * N1; u += nt) {
                const int b = u % count, k1 = u / count;
                V* p = buf + b * bs + k1 * N2 * es;
                V r[N2];
#pragma unroll
                for (int i = 0; i < N2; ++i) r[i] = p[i * es];
                Dft<T, N2, +1>::run(r);
#pragma unroll
                for (int n2 = 1; n2 < N2; ++n2) r[n2] = cmul(r[n2], cconj(tw[n2 * k1]));
#pragma unroll
                for (int i = 0; i < N2; ++i) p[i * es] = r[i];
            }
            __syncthreads();
        }
        for (int u = tid; u < count * N2; u += nt) {
            const int b = u % count, n2 = u / count;
            V* p = buf + b * bs + n2 * es;
            V r[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) r[i] = p[i * N2 * es];
            Dft<T, N1, +1>::run(r);
#pragma unroll
            for (int i = 0; i < N1; ++i) p[i * N2 * es] = r[i];
        }
    }
}

template <int N> __device__ __forceinline__ int perm_pos(int k) {
    return (k % Split<N>::N1) * Split<N>::N2 + k / Split<N>::N1;
}
template <int N> __device__ __forceinline__ int perm_freq(int pos) {
    return pos / Split<N>::N2 + Split<N>::N1 * (pos % Split<N>::N2);
}

template <typename T, int N>
__device__ __forceinline__ void make_twiddles(cplx_t<T>* tw) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)m / (double)N, &s, &c);
        tw[m] = cmake<cplx_t<T>, T>((T)c, (T)(-s));
    }
}


// ---------------------------------------------------------------------------
// General form: ntr transforms, transform t at
// buf + (t / inner) * bs + (t % inner) * is, element stride es; the N-point
// twiddle w_N^j = exp(-2 pi i j / N) is tw[j * tws].
// ---------------------------------------------------------------------------
template <typename T, int N1, int N2, int DIR>
__device__ __forceinline__ void fft_2s(cplx_t<T>* buf, int ntr, int inner, int bs, int is, int es,
                                       const cplx_t<T>* tw, int tws) {
    using V = cplx_t<T>;
    const int tid = threadIdx.x, nt = blockDim.x;
    if constexpr (DIR < 0) {
        for (int u = tid; u < ntr * N2; u += nt) {
            const int t = u % ntr, n2 = u / ntr;
            V* p = buf + (t / inner) * bs + (t % inner) * is + n2 * es;
            V r[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) r[i] = p[i * N2 * es];
            Dft<T, N1, -1>::run(r);
            if constexpr (N2 > 1) {
#pragma unroll
                for (int k1 = 1; k1 < N1; ++k1) r[k1] = cmul(r[k1], tw[n2 * k1 * tws]);
            }
#pragma unroll
            for (int i = 0; i < N1; ++i) p[i * N2 * es] = r[i];
        }
        if constexpr (N2 > 1) {
            __syncthreads();
            for (int u = tid; u < ntr * N1; u += nt) {
                const int t = u % ntr, k1 = u / ntr;
                V* p = buf + (t / inner) * bs + (t % inner) * is + k1 * N2 * es;
                V r[N2];
#pragma unroll
                for (int i = 0; i < N2; ++i) r[i] = p[i * es];
                Dft<T, N2, -1>::run(r);
#pragma unroll
                for (int i = 0; i < N2; ++i) p[i * es] = r[i];
            }
        }
    } else {
        if constexpr (N2 > 1) {
            for (int u = tid; u < ntr * N1; u += nt) {
                const int t = u % ntr, k1 = u / ntr;
                V* p = buf + (t / inner) * bs + (t % inner) * is + k1 * N2 * es;
                V r[N2];
#pragma unroll
                for (int i = 0; i < N2; ++i) r[i] = p[i * es];
                Dft<T, N2, +1>::run(r);
#pragma unroll
                for (int n2 = 1; n2 < N2; ++n2) r[n2] = cmul(r[n2], cconj(tw[n2 * k1 * tws]));
#pragma unroll
                for (int i = 0; i < N2; ++i) p[i * es] = r[i];
            }
            __syncthreads();
        }
        for (int u = tid; u < ntr * N2; u += nt) {
            const int t = u % ntr, n2 = u / ntr;
            V* p = buf + (t / inner) * bs + (t % inner) * is + n2 * es;
            V r[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) r[i] = p[i * N2 * es];
            Dft<T, N1, +1>::run(r);
#pragma unroll
            for (int i = 0; i < N1; ++i) p[i * N2 * es] = r[i];
        }
    }
}

// first stage of N = 16 M: 16-point DFTs across the blocks (forward: then the
// twiddles; inverse: the conjugate twiddles first)
template <typename T, int M, int DIR>
__device__ __forceinline__ void fft_stage16(cplx_t<T>* buf, int count, int bs, int es, const cplx_t<T>* tw,
                                            int tws) {
    using V = cplx_t<T>;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int u = tid; u < count * M; u += nt) {
        const int b = u % count, m = u / count;
        V* p = buf + b * bs + m * es;
        V r[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = p[i * M * es];
        if constexpr (DIR > 0) {
#pragma unroll
            for (int k1 = 1; k1 < 16; ++k1) r[k1] = cmul(r[k1], cconj(tw[m * k1 * tws]));
        }
        Dft<T, 16, DIR>::run(r);
        if constexpr (DIR < 0) {
#pragma unroll
            for (int k1 = 1; k1 < 16; ++k1) r[k1] = cmul(r[k1], tw[m * k1 * tws]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) p[i * M * es] = r[i];
    }
}

// count transforms of length N (4 .. 4096) at buf + b * bs, element stride es
template <typename T, int N, int DIR>
__device__ __forceinline__ void lds_fft_g(cplx_t<T>* buf, int count, int bs, int es, const cplx_t<T>* tw, int tws) {
    if constexpr (N <= 256) {
        fft_2s<T, Split<N>::N1, Split<N>::N2, DIR>(buf, count, 1, bs, 0, es, tw, tws);
    } else {
        constexpr int M = N / 16;
        if constexpr (DIR < 0) {
            fft_stage16<T, M, -1>(buf, count, bs, es, tw, tws);
            __syncthreads();
            fft_2s<T, Split<M>::N1, Split<M>::N2, -1>(buf, count * 16, 16, bs, M * es, es, tw, tws * 16);
        } else {
            fft_2s<T, Split<M>::N1, Split<M>::N2, +1>(buf, count * 16, 16, bs, M * es, es, tw, tws * 16);
            __syncthreads();
            fft_stage16<T, M, +1>(buf, count, bs, es, tw, tws);
        }
    }
}

template <int N> __device__ __forceinline__ int perm_pos_g(int k) {
    if constexpr (N <= 256) {
        return perm_pos<N>(k);
    } else {
        constexpr int M = N / 16;
        return (k % 16) * M + perm_pos<M>(k / 16);
    }
}
template <int N> __device__ __forceinline__ int perm_freq_g(int pos) {
    if constexpr (N <= 256) {
        return perm_freq<N>(pos);
    } else {
        constexpr int M = N / 16;
        return pos / M + 16 * perm_freq<M>(pos % M);
    }
}

}  // namespace sipf
