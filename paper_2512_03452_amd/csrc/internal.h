// Internal interfaces between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sipf {

// Phase timing: while a LaunchTiming is installed on the calling thread, the
// step's launches carry its events in their dispatch (the first launch records
// `start` as it begins, every launch records `stop` as it ends), so the timed
// interval holds the kernels and nothing else.
struct LaunchTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    bool started = false;
};
extern thread_local LaunchTiming* g_launch_timing;

template <typename F, typename... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args) {
    LaunchTiming* t = g_launch_timing;
    if (t) {
        hipEvent_t first = t->started ? nullptr : t->start;
        t->started = true;
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, first, t->stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

// Everything the field passes (FFT, mode update, gradient) need for one
// instance.  3-D: spectral arrays are Hermitian half spectra H x H x (H/2+1)
// whose kx and ky indices are stored in the digit-permuted order of the LDS
// FFT (see fft.hip); grids are H^3 row-major; G holds the three gradient
// components one after another (d-major).  2-D (field2d.hip): spectra are
// (H/2+1) x H, ky-major (ky = 0..H/2), kx in the digit-permuted order; grids
// H^2 row-major; G holds two components.
template <typename T> struct FieldDesc {
    T* phi;                 // deposit accumulator (mass units); zeroed by the forward pass
    cplx_t<T>* B1;          // yz-plane pass output (x not yet transformed)
    cplx_t<T>* alpha;       // alpha^(n), permuted (kx, ky)
    cplx_t<T>* gspec;       // gradient spectra after the x inverse pass
    T* G;                   // gradient grids, one per axis
    uint32_t* step;         // completed-step counter, incremented by the forward pass
    T dt_over_eps;          // tau / eps (0 when elliptic)
    T eps_over_dt;          // eps / tau
    T k2;                   // k^2
    T inv_Ld;               // L^-d (F_H normalisation, Sec. 3.1)
    T two_pi_over_L;        // xi = 2 pi q / L
    T filt;                 // 2 pi^2 / H0^2, or 0 (no filter)
    int elliptic;           // eps = 0: A = 0, B = 1/(|xi|^2 + k^2), B = 0 where that vanishes
    int expo;               // exponential propagator (Sec. 3.4): A = exp(-tau s / eps), B = A tau / eps
};

// Mode factors of the implicit update (eq. alpha_hat_update) for
// s = |xi|^2 + k^2, of the exponential propagator of Sec. 3.4 (source weight
// tau/eps, as in the implicit form), or the elliptic limit when eps = 0.
template <typename T> __device__ __forceinline__ void mode_ab(const FieldDesc<T>& fd, T s, T& A, T& B) {
    if (fd.elliptic) {
        A = (T)0;
        B = s > (T)0 ? (T)1 / s : (T)0;
    } else if (fd.expo) {
        A = exp(-fd.dt_over_eps * s);
        B = A * fd.dt_over_eps;
    } else {
        A = (T)1 / ((T)1 + fd.dt_over_eps * s);
        B = (T)1 / (s + fd.eps_over_dt);
    }
}

// One instance of the particle pass.  Particles are stored SoA and kept
// approximately sorted by tile; id is the original particle index.
template <typename T> struct PartDesc {
    T* x;
    T* y;
    T* z;
    uint32_t* id;
    int64_t P;
    T* phi;                 // deposit target (H^3)
    const T* G;             // gradient grids (3 x H^3)
    const uint32_t* step;   // completed steps; this step is *step + 1
    int* err;               // device error flags (bit 0: non-finite position, bit 1: non-finite input, bit 2: sort counts inconsistent)
    int H;
    int dim;                // 2 or 3 (z unused in 2-D)
    int scheme;             // SIPF_STRANG or SIPF_EM
    T hl;                   // H / L
    T L;
    T halfL;
    T invL;
    T wmass;                // M0 / P
    T chitau;               // chi * tau
    T s;                    // noise scale: sqrt(mu tau) (split) or sqrt(2 mu tau) (EM)
    uint32_t k0, k1;        // Philox key
    uint32_t inst;          // fourth counter word
    int gmargin;            // cells the W^- displacement can reach (gradient window margin)
    int tshift;             // log2 of the sort tile side, or -1 when the side is not a power of two
    int tile;               // sort tile side (cells)
    int nkeys;              // Morton keys: (H / tile)^dim, or with ceil(H / tile) rounded up to a power of two
    T* ox;                  // push-only passes: positions out (null: in place), ids copied to oid
    T* oy;
    T* oz;
    uint32_t* oid;
    T* zout;                // push-only passes: the step's normals out (SoA, 6 x P in particle order), or null
};

// A run of sort-chunk particles of one instance (sort kernels).
struct SortChunk {
    int64_t beg;
    int32_t inst;
    int32_t pad;
};

// One reverse step of the particle branch (adjoint.hip).
template <typename T> struct AdjDesc {
    const T* x;             // X^(n-1), any order
    const T* y;
    const T* z;
    const uint32_t* id;
    int64_t P;
    const T* G;             // gradient grids of alpha^(n-1)
    const T* phibar;        // cotangent of the deposit of X^(n-1), or null
    T* xbar;                // P x 3 by particle id (seed kernel output)
    T* xbx;                 // cotangents in the order of x/y/z (SoA): in Xbar^(n), out Xbar^(n-1)
    T* xby;
    T* xbz;
    T* Gbar;                // 3 x H^3 cotangent of G (accumulated)
    double* acc;            // [0] chibar, [1] sbar (accumulated)
    int H;
    int scheme;
    T hl;
    T wmass;
    T chitau;
    T tau;
    T s;
    uint32_t k0, k1, inst, n;
    int gmargin;            // cells the W^- displacement can reach
    const T* zin;           // the step's normals (SoA, 6 x P in the order of x), or null: drawn here
};

// Work item of the particle pass: particles [beg, beg + cnt) of instance inst.
struct WorkItem {
    int64_t beg;
    int32_t cnt;
    int32_t inst;
};

// --- field passes (fft.hip) -------------------------------------------------
// Each launcher runs its pass for `count` instances of grid size H whose
// descriptors are consecutive in the device array `fd`.
// fwd_planes: R2C of ncomp grids (phi + c H^3 -> B1 + c spectrum); consume = clear
//             the input and advance the step counter (the step's deposit).
// xpencils:   mode MODE_STEP / MODE_GRAD / MODE_ADJ_SRC / MODE_ADJ_ACC / MODE_RHO (fft.hip).
// inv_planes: C2R of ncomp spectra (gspec + c spectrum -> G + c H^3).
enum { XP_STEP = 0, XP_GRAD = 1, XP_ADJ_SRC = 2, XP_ADJ_ACC = 3, XP_RHO = 4, XP_ADJ_ACC_SRC = 5 };
template <typename T>
hipError_t launch_fwd_planes(int H, const FieldDesc<T>* fd, int count, int ncomp, bool consume, hipStream_t s);
template <typename T> hipError_t launch_xpencils(int H, const FieldDesc<T>* fd, int count, int mode, hipStream_t s);
template <typename T> hipError_t launch_inv_planes(int H, const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s);
bool fft_size_supported(int H, bool fp64);
// 2-D field passes (field2d.hip): same roles for instances of grid H x H
// (H = 8 .. 4096); xrows takes XP_STEP, XP_GRAD or XP_RHO.
template <typename T>
hipError_t launch_fwd_rows2(int H, const FieldDesc<T>* fd, int count, bool consume, hipStream_t s);
template <typename T> hipError_t launch_xrows2(int H, const FieldDesc<T>* fd, int count, int mode, hipStream_t s);
template <typename T> hipError_t launch_inv_rows2(int H, const FieldDesc<T>* fd, int count, int ncomp, hipStream_t s);
bool fft2d_size_supported(int H);
// digit permutation of the LDS FFT of length N: storage position of frequency k
int fft_perm(int N, int k);

// --- particle pass (particles.hip) -------------------------------------------
// nitems: the item list's header, [0] the count the sort writes and [1] the
// ticket counter of the persistent passes (next_item in pass_common.h).
template <typename T>
// pow2: every instance's H is a power of two (index wraps by mask; else by remainder)
// sorted: the FP32 deposit + push pass keeps each item sorted by cell and
// accumulates runs of equal cells (else the two-phase pass; FP64 and the
// single-phase passes ignore it)
// kcounts: when not null, the deposit + push pass also counts the pushed
// particles' sort tiles into these counts (MAX_KEYS per instance, zero on
// entry), so that the next sort can skip its histogram (launch_sort counted)
hipError_t launch_particles(const PartDesc<T>* pd, const WorkItem* items, int* nitems, int grid, bool deposit,
                            bool push, int scheme, int win_bytes, bool pow2, bool sorted, hipStream_t s,
                            uint32_t* kcounts = nullptr);
// positivity-preserving deposit rounds (positivity.hip): flag nodes below
// -thresh, switch the order-4 particles touching a flagged node to order 2
// (count += switched; sw[i] = tag marks them), clamp negatives to zero; tmp
// and touch are H^3-byte scratch grids for the per-cell dilation of the flags
template <typename T> hipError_t launch_pos_flag(const T* phi, int64_t n, T thresh, uint8_t* flag, hipStream_t s);
template <typename T>
hipError_t launch_pos_switch(const PartDesc<T>* pd, int64_t P, int H, const uint8_t* flag, uint8_t* tmp,
                             uint8_t* touch, uint32_t* sw, uint32_t tag, int* count, hipStream_t s);
template <typename T> hipError_t launch_pos_clamp(T* phi, int64_t n, hipStream_t s);
// 2-D particle pass (particles2d.hip)
template <typename T>
hipError_t launch_particles2(const PartDesc<T>* pd, const WorkItem* items, int* nitems, int grid, bool deposit,
                             bool push, int scheme, int win_bytes, hipStream_t s);
template <typename T> int particle_resident_blocks2(int scheme, int win_bytes);
template <typename T>
// counted: the counts already hold the tiles of src (taken by the previous
// step's particle pass), so the histogram pass is skipped.  The scan checks
// that the counts add up to each instance's P; if not, it lists no work items
// and sets bit 2 of the instance's error flag (the scatter then writes
// nothing past the array).
hipError_t launch_sort(int dim, const PartDesc<T>* src, const PartDesc<T>* dst, const SortChunk* chunks, int nchunks, int ninst,
                       uint32_t* counts, uint32_t* cursor, WorkItem* seg, const int* seg_off, int* seg_n,
                       WorkItem* items, int* nitems, int chunk, hipStream_t s, bool counted = false);
int sort_chunk();
template <typename T>
hipError_t launch_cells(const T* X, int64_t n, int H, T hl, int32_t* cells, hipStream_t s);
template <typename T>
hipError_t launch_philox_dbg(uint64_t seed, int64_t n, const uint32_t* ctr, uint32_t* raw, T* normals, hipStream_t s);
template <typename T>
hipError_t launch_unsort(const PartDesc<T>* pd_host, T* out_xyz, hipStream_t s);
template <typename T>
hipError_t launch_load_positions(const T* xyz, int64_t P, T L, PartDesc<T> pd_host, int* err, hipStream_t s);
template <typename T> hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <typename T> hipError_t launch_adj_seed(const AdjDesc<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_adj_items(const AdjDesc<T>& a, const WorkItem* items, int* nitems, int grid, hipStream_t s);
template <typename T>
hipError_t launch_copy_positions(T* x, T* y, T* z, uint32_t* id, const T* sx, const T* sy, const T* sz,
                                 const uint32_t* sid, int64_t P, hipStream_t s);
// by-id cotangents (P x 3) <-> cotangents in the order of the ids array (SoA)
template <typename T>
hipError_t launch_xbar_order(T* xbar, T* bx, T* by, T* bz, const uint32_t* id, int64_t P, bool to_order,
                             hipStream_t s);
hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t s);
int adj_window_bytes(bool fp64);
// --- direct SIPF (direct.hip) -------------------------------------------------
// One instance of Algorithm 1: particles in original order (SoA), full
// spectra H^3 in natural order.
template <typename T> struct DirDesc {
    T* x;
    T* y;
    T* z;
    int64_t P;
    int H;
    int scheme;
    T L, halfL, invL;
    T bscale;               // M0 / (P L^3)
    T chitau;               // chi tau
    T s;                    // noise scale (as in PartDesc)
    cplx_t<T>* alpha;       // H^3, updated in place
    cplx_t<T>* gc;          // 3 x H^3: i xi_d Phi alpha^(n-1)
    uint32_t* step;         // completed steps, advanced by the step's first kernel
    int* err;
    uint32_t k0, k1, inst;
    FieldDesc<T> fd;        // mode factors, filter, 2 pi / L (the grid pointers are unused)
};
int dir_slices(int H, int64_t P);
int dir_mode_slices(int H, int64_t P);
// part: dir_slices(H, P) x H^3 complex scratch; gpart: ms x 3 x P partial
// gradients, ms = dir_mode_slices(H, P)
template <typename T>
hipError_t launch_direct_step(const DirDesc<T>& d, cplx_t<T>* part, int nslices, T* gpart, int ms, hipStream_t s);

// --- diagnostics (diag.hip) ---------------------------------------------------
// One instance: the regularised density on the grid, the permuted half
// spectrum alpha and the current particle positions.
template <typename T> struct DiagDesc {
    const T* rho;             // H^3
    const cplx_t<T>* alpha;   // H x H x (H/2+1), (kx, ky) in FFT storage order
    const T* x;
    const T* y;
    const T* z;
    int64_t P;
    int H;
    int dim;                  // 3: H x H x (H/2+1) spectrum, (kx, ky) permuted; 2: (H/2+1) x H, kx permuted
    int pm, pt, n1, n2;       // FFT storage order: freq(pos) = pos / pm + pt inner(pos % pm),
                              // inner(r) = r / n2 + n1 (r % n2)
    int nb;                   // workgroups reducing this instance, 1 .. DIAG_MAX_BLOCKS
};
// Sums per instance, in this order: sum rho, max rho, sum_q w|alpha_q|^2,
// the same over |q| >= 4, Re alpha_0, sum sqrt(x^2 + y^2), sum |X|^2, 0.
constexpr int DIAG_NVAL = 8;
constexpr int DIAG_MAX_BLOCKS = 1024;
// workgroups for an instance with P particles on a grid of ng nodes
int diag_blocks(int64_t P, int64_t ng);
// part: n x DIAG_MAX_BLOCKS x DIAG_NVAL doubles of scratch; out: n x DIAG_NVAL
// doubles; nbmax = max over instances of DiagDesc::nb
template <typename T>
hipError_t launch_diag(const DiagDesc<T>* d, int n, int nbmax, double* part, double* out, hipStream_t s);

template <typename T> hipError_t launch_dot(const T* u, const T* v, int64_t n, double* out, hipStream_t s);
template <typename T> hipError_t launch_axpby(T* y, const T* x, T a, T b, int64_t n, hipStream_t s);
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);
hipError_t launch_zero_f64(double* p, int n, hipStream_t s);
int sort_max_keys();
// allocation-free deposit (noalloc.hip): this device's static scratch array
hipError_t noalloc_scratch(void** out, size_t* bytes);
template <typename T>
hipError_t launch_noalloc_setup(const PartDesc<T>& d0, const PartDesc<T>& d1, PartDesc<T>* pd, SortChunk* chunks,
                                int nchunks, int sort_chunk_size, int* seg_off, uint32_t* counts, int nkeys,
                                int* nitems, int* err, uint32_t* step, hipStream_t s);
int particle_threads();
int particle_chunk();
int particle_window_bytes(bool fp64);
template <typename T> int particle_resident_blocks(int scheme, int win_bytes, bool sorted);

}  // namespace sipf
