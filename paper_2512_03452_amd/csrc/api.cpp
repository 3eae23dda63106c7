// Host runtime and C ABI of the SIPF-PIC step (declared in include/sipf.h).
//
// The runtime advances a *group* of independent instances together.  One step
// of a group is one persistent particle launch over the work items of every
// instance, then three field launches (forward planes, x pencils, inverse
// planes) per distinct grid size H, each covering all instances of that size
// (blockIdx.y selects the instance).  Every resort_every steps one sort of all
// instances (four launches) re-bins the particles and rebuilds the work list.
// A simulation context is a group of one; a batch is a group of many.
//
// Stepping replays a captured HIP graph of two sort periods (the sort swaps
// between two particle buffer sets, so two periods return to the starting
// set); steps that do not fill a whole graph run eagerly.  No memset node is
// ever recorded: every buffer the step clears is cleared by a kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "sipf.h"

using namespace sipf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(SIPF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

int dim_of(const sipf_params* p) { return p->dim == 2 ? 2 : 3; }
size_t grid_size(int H, int d) { return d == 2 ? (size_t)H * H : (size_t)H * H * H; }
size_t spec_size(int H, int d) { return d == 2 ? (size_t)H * (H / 2 + 1) : (size_t)H * H * (H / 2 + 1); }

int validate(const sipf_params* p, int64_t P) {
    if (!p) return fail(SIPF_EINVAL, "params is NULL");
    if (p->precision != SIPF_FP32 && p->precision != SIPF_FP64) return fail(SIPF_EINVAL, "precision must be SIPF_FP32 or SIPF_FP64");
    if (p->dim != 0 && p->dim != 2 && p->dim != 3) return fail(SIPF_EINVAL, "dim must be 0, 2 or 3");
    if (dim_of(p) == 3 && !fft_size_supported(p->H, p->precision == SIPF_FP64))
        return fail(SIPF_EINVAL, "H must be 8, 12, 16, 22, 32, 46, 64, 90, 128 or 256 (FP32), or one of those up to 64 (FP64)");
    if (dim_of(p) == 2 && !fft2d_size_supported(p->H))
        return fail(SIPF_EINVAL, "H must be a power of two in [8, 4096] in two dimensions");
    auto fin = [](double v) { return std::isfinite(v); };
    if (!(fin(p->L) && p->L > 0)) return fail(SIPF_EINVAL, "L must be finite and > 0");
    if (!(fin(p->dt) && p->dt > 0)) return fail(SIPF_EINVAL, "dt must be finite and > 0");
    if (!(fin(p->eps) && p->eps >= 0)) return fail(SIPF_EINVAL, "eps must be finite and >= 0");
    if (!(fin(p->mu) && p->mu >= 0)) return fail(SIPF_EINVAL, "mu must be finite and >= 0");
    if (!(fin(p->chi) && p->chi >= 0)) return fail(SIPF_EINVAL, "chi must be finite and >= 0");
    if (!(fin(p->k) && p->k >= 0)) return fail(SIPF_EINVAL, "k must be finite and >= 0");
    if (!(fin(p->M0) && p->M0 >= 0)) return fail(SIPF_EINVAL, "M0 must be finite and >= 0");
    if (!fin(p->H0)) return fail(SIPF_EINVAL, "H0 must be finite");
    if (p->propagator != SIPF_PROP_IMPLICIT && p->propagator != SIPF_PROP_EXP)
        return fail(SIPF_EINVAL, "propagator must be SIPF_PROP_IMPLICIT or SIPF_PROP_EXP");
    if (p->propagator == SIPF_PROP_EXP && p->eps == 0)
        return fail(SIPF_EINVAL, "the exponential propagator needs eps > 0");
    if (p->method != SIPF_METHOD_PIC && p->method != SIPF_METHOD_DIRECT)
        return fail(SIPF_EINVAL, "method must be SIPF_METHOD_PIC or SIPF_METHOD_DIRECT");
    if (p->method == SIPF_METHOD_DIRECT && dim_of(p) != 3)
        return fail(SIPF_EINVAL, "the direct SIPF method is three-dimensional");
    if (p->method == SIPF_METHOD_DIRECT && p->H > 128)
        return fail(SIPF_EINVAL, "the direct SIPF method takes H <= 128");
    if (p->positivity != 0 && p->positivity != 1) return fail(SIPF_EINVAL, "positivity must be 0 or 1");
    if (p->particle_pass < SIPF_PASS_DEFAULT || p->particle_pass > SIPF_PASS_TWO_PHASE)
        return fail(SIPF_EINVAL, "particle_pass must be SIPF_PASS_DEFAULT, SIPF_PASS_SORTED or SIPF_PASS_TWO_PHASE");
    if (p->positivity && (dim_of(p) != 3 || p->method != SIPF_METHOD_PIC))
        return fail(SIPF_EINVAL, "the positivity-preserving deposit is for the 3-D SIPF-PIC step");
    if (p->p2g_order != 4) return fail(SIPF_EINVAL, "p2g_order must be 4");
    if (p->g2p_order != 2) return fail(SIPF_EINVAL, "g2p_order must be 2");
    if (p->scheme != SIPF_STRANG && p->scheme != SIPF_EM) return fail(SIPF_EINVAL, "scheme must be SIPF_STRANG or SIPF_EM");
    const int max_tiles = dim_of(p) == 2 ? 64 : 16;
    if (p->tile != 0 && is_pow2(p->H) && (!is_pow2(p->tile) || p->tile > p->H || (p->H / p->tile) > max_tiles))
        return fail(SIPF_EINVAL, dim_of(p) == 2 ? "tile must be 0 or a power of two with H/64 <= tile <= H"
                                                : "tile must be 0 or a power of two with H/16 <= tile <= H");
    if (p->tile != 0 && !is_pow2(p->H) && (p->tile < 1 || p->tile > p->H || (p->H + p->tile - 1) / p->tile > max_tiles))
        return fail(SIPF_EINVAL, "tile must be 0 or in [1, H] with at most 16 tiles per axis");
    if (p->resort_every < 0) return fail(SIPF_EINVAL, "resort_every must be >= 0");
    if (p->chunk != 0 && (p->chunk < 256 || p->chunk > 4096)) return fail(SIPF_EINVAL, "chunk must be 0 or in [256, 4096]");
    if (P < 1 || P >= (int64_t(1) << 32)) return fail(SIPF_EINVAL, "P must be in [1, 2^32)");
    return SIPF_OK;
}

double filter_h0(const sipf_params* p) {
    if (p->H0 == 0) return std::ceil(8.0 * std::pow((double)p->H, 8.0 / 13.0) * std::pow(p->L, 5.0 / 13.0));
    return p->H0;
}

// Defaults where the parameters leave the tuning open (0): an 8-cell tile at
// H = 128 and H/8 below (3-D), 16-cell tiles up to H = 1024 and H/64 above
// (2-D), a re-sort every 4 steps (items: default_chunk).  A 3-D grid that is not
// a power of two takes the same rule with ceil(H / 8) below H = 128 (the last
// tile of an axis may be partial; the whole axis below H = 16).
int default_tile(const sipf_params* p) {
    if (dim_of(p) == 3 && !is_pow2(p->H)) {
        if (p->tile) return p->tile;
        return p->H < 16 ? p->H : (p->H >= 128 ? 8 : (p->H + 7) / 8);
    }
    if (dim_of(p) == 2) {
        int t = p->tile ? p->tile : std::min(p->H, std::max(16, p->H / 64));
        if (p->H / t > 64) t = p->H / 64;
        return t;
    }
    int t = p->tile ? p->tile : (p->H >= 128 ? 8 : (p->H >= 16 ? p->H / 8 : p->H));
    if (p->H / t > 16) t = p->H / 16;
    return t;
}
// Re-sort period: every 6 steps in 3-D (4 in 2-D), or more often when the
// Brownian spread over the period, sqrt(2 mu tau n), would exceed a quarter of
// a tile (item boxes then outgrow their LDS windows and the pass falls back to
// global atomics).  3-D, FP32 ms per step at periods 4 / 6 / 8: torus P = 1e7
// 0.283 / 0.277 / 0.302 (the collapsing ring's drift outgrows the windows at
// 8); blob P = 2e6 0.138 / 0.124 / 0.115; mixed P = 1e6 0.069 / 0.067 / 0.067.
int default_resort(const sipf_params* p) {
    if (p->resort_every) return p->resort_every;
    const double cap = dim_of(p) == 2 ? 4.0 : 6.0;
    const double q = default_tile(p) * p->L / p->H / 4.0;
    const double spread = 2.0 * p->mu * p->dt;
    if (spread <= 0) return (int)cap;
    const double n = std::floor(q * q / spread);
    return (int)std::max(1.0, std::min(cap, n));
}
// Work-item size: in 3-D, 3072, and 4096 from 2^23 particles per group; 2-D
// keeps 4096.  The particle pass draws items from a ticket queue, so the size
// trades per-item set-up (windows, barriers) against balance.  Measured
// (FP32, ms per step, items of 4096 / 3072 / 2048): torus P = 1e7 0.289 /
// 0.292 / 0.315; torus P = 6.5e6 0.224 / 0.215 / 0.231; blob P = 2e6 0.130 /
// 0.119 / 0.132; mixed P = 1e6 0.087 / 0.070 / 0.072; 64-instance ensemble
// 0.687 / 0.688 / 0.711.  2-D: P = 2^22 disk 0.265 / 0.272 (4096 / 2048).
int default_chunk(const sipf_params* p, int64_t total_P) {
    if (p->chunk) return p->chunk;
    if (dim_of(p) == 2) return 4096;
    return total_P >= (int64_t(1) << 23) ? 4096 : 3072;
}
// Work-item size of the adjoint's per-segment sorts: its reverse item pass
// holds one 512-thread workgroup per CU and prefers smaller items (adjoint
// workload, P = 2e6: reverse sweep ~0.75 ms shorter at 2048 than at 3072).
int default_adj_chunk(const sipf_params* p, int chunk) { return p->chunk ? p->chunk : std::min(chunk, 2048); }
// FP32 3-D deposit + push pass: sorted items or the two-phase pass (the
// choice is shared by a group's instances).
bool sorted_pass(const sipf_params* p, int n) {
    if (p->particle_pass) return p->particle_pass == SIPF_PASS_SORTED;
    return n > 1;
}

}  // namespace

// One instance: its parameters and device buffers.
struct Inst {
    sipf_params prm{};
    int64_t P = 0;
    int H = 0;
    int dim = 3;
    int tile = 8;
    void* xs[2] = {nullptr, nullptr};
    void* ys[2] = {nullptr, nullptr};
    void* zs[2] = {nullptr, nullptr};
    uint32_t* ids[2] = {nullptr, nullptr};
    void* phi = nullptr;    // H^3 deposit
    void* B1 = nullptr;     // half spectrum after the yz pass
    void* alpha = nullptr;  // alpha^(n), permuted (kx, ky)
    void* gspec = nullptr;  // 3 gradient spectra
    void* G = nullptr;      // 3 x H^3 gradient grids
    // direct SIPF (Algorithm 1): alpha is the full H^3 spectrum in natural order
    void* gc = nullptr;     // 3 x H^3 gradient coefficients
    void* part = nullptr;   // nslices x H^3 partial sums of beta
    void* gpart = nullptr;  // mslices x 3 x P partial gradient sums
    int nslices = 0, mslices = 0;
    // positivity-preserving deposit: per-particle switch tags, node flags
    uint32_t* pos_sw = nullptr;
    uint8_t* pos_flag = nullptr;  // node flags, then two H^3-byte scratch grids
};

// Instances of one grid size: FieldDesc slots [first, first + count).
struct HClass {
    int H, first, count;
};

struct Group {
    int prec = SIPF_FP32;
    int dim = 3;  // shared by every instance
    int method = SIPF_METHOD_PIC;
    bool pow2 = true;  // every instance's H is a power of two
    bool positivity = false;  // positivity-preserving deposit (shared by every instance)
    uint32_t pos_tag = 0;     // tag of the last positive deposit
    int* pos_count = nullptr;  // per-instance particles switched in a round
    int64_t pos_switched = 0;  // particles switched by the last positive deposit
    int pos_rounds = 0;        // rounds that switched someone in it
    size_t tsize = 4;
    int scheme = SIPF_STRANG;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    int resort = 4, chunk = 4096, adj_chunk = 2048, win_bytes = 65536, pgrid = 1024;
    bool sorted = false;  // FP32 3-D deposit + push: the sorted pass (else two-phase)
    bool counts_ready = false;  // the last step's particle pass left the tile counts of the next sort
    int since_sort = 0;
    int cur = 0;  // which of the two particle buffer sets holds the current positions
    int64_t n_host = 0;
    std::vector<Inst> in;
    std::vector<HClass> classes;
    std::vector<int> fslot;  // FieldDesc slot of instance i
    uint32_t* steps = nullptr;  // per-instance completed-step counters
    int* errs = nullptr;        // per-instance error flags
    uint32_t* counts = nullptr;  // n x MAX_KEYS tile counts (zero between sorts)
    uint32_t* cursor = nullptr;  // n x MAX_KEYS tile starts / scatter cursors
    void* pdesc = nullptr;       // 2n PartDesc<T>: set s of instance i at s*n + i
    void* fdesc = nullptr;       // n FieldDesc<T>, grouped by H class
    SortChunk* chunks = nullptr;
    int nchunks = 0;
    WorkItem* seg = nullptr;  // per-instance item segments written by the scan
    int* seg_off = nullptr;
    int* seg_n = nullptr;
    WorkItem* items = nullptr;  // concatenated work items of the particle pass
    int* nitems = nullptr;  // [0] item count, [1] ticket counter of the persistent passes (zero between launches)
    int items_cap = 0;
    std::vector<void*> allocs;
    void* diag = nullptr;  // diagnostics scratch, allocated on first use
    // captured graphs of run segments, by (buffer set, steps since the last
    // sort, segment length, whether the tile counts of a due sort are ready):
    // the only host state a step's launches depend on
    bool graphs = true;
    struct GraphSeg {
        int cur, since, len, counted;
        hipGraphExec_t exec;
    };
    std::vector<GraphSeg> gcache;
    // per-phase event timing
    bool prof = false;
    struct Mark {
        int phase;
        hipEvent_t a, b;  // end of the previous phase (or a start marker), end of this phase
    };
    std::vector<hipEvent_t> events;  // every event created for timing, released together
    hipEvent_t last_stop = nullptr;  // end event of the last timed phase
    std::vector<Mark> marks;
    double prof_ms[SIPF_NPHASES] = {0};
    int64_t prof_n[SIPF_NPHASES] = {0};
};

struct sipf_ctx : Group {};
struct sipf_batch : Group {};

namespace {

int dalloc(Group* g, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SIPF_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    g->allocs.push_back(*p);
    return SIPF_OK;
}

// The parameter-derived fields of a particle descriptor (buffers left null).
template <typename T> PartDesc<T> pdesc_params(const sipf_params& p, int64_t P, int H, int dim, int tile) {
    PartDesc<T> d{};
    d.P = P;
    d.H = H;
    d.dim = dim;
    d.scheme = p.scheme;
    d.hl = (T)(H / p.L);
    d.L = (T)p.L;
    d.halfL = (T)(p.L / 2);
    d.invL = (T)(1.0 / p.L);
    d.wmass = (T)(p.M0 / (double)P);
    d.chitau = (T)(p.chi * p.dt);
    d.s = (T)(p.scheme == SIPF_STRANG ? std::sqrt(p.mu * p.dt) : std::sqrt(2.0 * p.mu * p.dt));
    d.k0 = (uint32_t)p.seed;
    d.k1 = (uint32_t)(p.seed >> 32);
    d.inst = p.instance;
    // |W^-| <= s max|z| with max|z| = sqrt(-2 ln 2^-22) = 5.5176 (uniforms are >= 2^-22)
    d.gmargin = p.scheme == SIPF_STRANG ? (int)std::ceil((double)d.s * 5.52 * (double)d.hl) : 0;
    // the Morton key space is a power of two per axis; tiles past H / tile stay empty
    d.tshift = is_pow2(H) && is_pow2(tile) ? ilog2(tile) : -1;
    d.tile = tile;
    const int nt = 1 << ilog2((H + tile - 1) / tile);
    d.nkeys = dim == 2 ? nt * nt : nt * nt * nt;
    return d;
}

template <typename T> PartDesc<T> make_pdesc(const Group* g, int i, int set) {
    const Inst& I = g->in[i];
    PartDesc<T> d = pdesc_params<T>(I.prm, I.P, I.H, I.dim, I.tile);
    d.x = (T*)I.xs[set];
    d.y = (T*)I.ys[set];
    d.z = (T*)I.zs[set];
    d.id = I.ids[set];
    d.phi = (T*)I.phi;
    d.G = (const T*)I.G;
    d.step = g->steps + i;
    d.err = g->errs + i;
    return d;
}

template <typename T> FieldDesc<T> make_fdesc(const Group* g, int i) {
    const Inst& I = g->in[i];
    const sipf_params& p = I.prm;
    FieldDesc<T> f{};
    f.phi = (T*)I.phi;
    f.B1 = (cplx_t<T>*)I.B1;
    f.alpha = (cplx_t<T>*)I.alpha;
    f.gspec = (cplx_t<T>*)I.gspec;
    f.G = (T*)I.G;
    f.step = g->steps + i;
    f.elliptic = p.eps == 0.0 ? 1 : 0;
    f.expo = p.propagator == SIPF_PROP_EXP ? 1 : 0;
    f.dt_over_eps = f.elliptic ? (T)0 : (T)(p.dt / p.eps);
    f.eps_over_dt = (T)(p.eps / p.dt);
    f.k2 = (T)(p.k * p.k);
    f.inv_Ld = (T)(I.dim == 2 ? 1.0 / (p.L * p.L) : 1.0 / (p.L * p.L * p.L));
    f.two_pi_over_L = (T)(2.0 * M_PI / p.L);
    const double h0 = filter_h0(&p);
    f.filt = p.H0 < 0 ? (T)0 : (T)(2.0 * M_PI * M_PI / (h0 * h0));
    return f;
}

template <typename T> int upload_descs(Group* g) {
    const int n = (int)g->in.size();
    std::vector<PartDesc<T>> pd(2 * n);
    std::vector<FieldDesc<T>> fd(n);
    for (int i = 0; i < n; ++i) {
        pd[i] = make_pdesc<T>(g, i, 0);
        pd[n + i] = make_pdesc<T>(g, i, 1);
        fd[g->fslot[i]] = make_fdesc<T>(g, i);
    }
    HIPCHK(hipMemcpy(g->pdesc, pd.data(), pd.size() * sizeof(PartDesc<T>), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->fdesc, fd.data(), fd.size() * sizeof(FieldDesc<T>), hipMemcpyHostToDevice));
    return SIPF_OK;
}

template <typename T> const PartDesc<T>* pdesc_dev(const Group* g, int set) {
    return reinterpret_cast<const PartDesc<T>*>(g->pdesc) + (size_t)set * g->in.size();
}
template <typename T> const FieldDesc<T>* fdesc_dev(const Group* g, int slot) {
    return reinterpret_cast<const FieldDesc<T>*>(g->fdesc) + slot;
}

}  // namespace

thread_local sipf::LaunchTiming* sipf::g_launch_timing = nullptr;

namespace {

// Events of one phase when timing is on.  Each phase's last kernel records
// its end event as part of its dispatch (see launch_kernel); a phase is timed
// from the end of the previous phase to its own end, so the interval holds
// exactly the phase's kernels (kernels of one stream run back to back).  The
// first phase after profiling starts, or after a read-out, begins at a marker.
struct Timed {
    Group* g;
    int phase;
    LaunchTiming lt;
    hipEvent_t a = nullptr;
    Timed(Group* grp, int ph) : g(grp), phase(ph) {
        if (!g->prof) return;
        if (hipEventCreate(&lt.stop) != hipSuccess) {
            lt.stop = nullptr;
            g->prof = false;
            return;
        }
        g->events.push_back(lt.stop);
        a = g->last_stop;
        if (!a) {
            if (hipEventCreate(&a) != hipSuccess) {
                a = nullptr;
                lt.stop = nullptr;
                g->prof = false;
                return;
            }
            g->events.push_back(a);
            if (hipEventRecord(a, g->stream) != hipSuccess) {
                lt.stop = nullptr;
                g->prof = false;
                return;
            }
            g->last_stop = a;
        }
        g_launch_timing = &lt;
    }
    ~Timed() {
        if (!lt.stop) return;
        g_launch_timing = nullptr;
        if (lt.started) {
            g->marks.push_back({phase, a, lt.stop});
            g->last_stop = lt.stop;
        }
    }
};

template <typename T> int do_sort(Group* g) {
    const int dst = 1 - g->cur;
    {
        Timed t(g, SIPF_PHASE_SORT);
        HIPCHK(launch_sort<T>(g->dim, pdesc_dev<T>(g, g->cur), pdesc_dev<T>(g, dst), g->chunks, g->nchunks, (int)g->in.size(),
                              g->counts, g->cursor, g->seg, g->seg_off, g->seg_n, g->items, g->nitems, g->chunk,
                              g->stream, g->counts_ready));
        g->counts_ready = false;
    }
    g->cur = dst;
    g->since_sort = 0;
    return SIPF_OK;
}

// Whether the step's particle pass takes the tile counts of the next sort
// (3-D SIPF-PIC steps without the positivity rounds, whose deposit and push
// run apart).
bool counts_in_pass(const Group* g) {
    return g->dim == 3 && g->method == SIPF_METHOD_PIC && !g->positivity;
}

// The passes of a step in the group's dimension.
template <typename T>
hipError_t particles_any(const Group* g, const PartDesc<T>* pd, bool deposit, bool push, uint32_t* kcounts = nullptr) {
    return g->dim == 2 ? launch_particles2<T>(pd, g->items, g->nitems, g->pgrid, deposit, push, g->scheme,
                                              g->win_bytes, g->stream)
                       : launch_particles<T>(pd, g->items, g->nitems, g->pgrid, deposit, push, g->scheme,
                                             g->win_bytes, g->pow2, g->sorted, g->stream, kcounts);
}
template <typename T> hipError_t field_fwd(const Group* g, int H, const FieldDesc<T>* fd, int count, bool consume) {
    return g->dim == 2 ? launch_fwd_rows2<T>(H, fd, count, consume, g->stream)
                       : launch_fwd_planes<T>(H, fd, count, 1, consume, g->stream);
}
template <typename T> hipError_t field_x(const Group* g, int H, const FieldDesc<T>* fd, int count, int mode) {
    return g->dim == 2 ? launch_xrows2<T>(H, fd, count, mode, g->stream)
                       : launch_xpencils<T>(H, fd, count, mode, g->stream);
}
template <typename T> hipError_t field_inv(const Group* g, int H, const FieldDesc<T>* fd, int count, int ncomp) {
    return g->dim == 2 ? launch_inv_rows2<T>(H, fd, count, ncomp, g->stream)
                       : launch_inv_planes<T>(H, fd, count, ncomp, g->stream);
}

// One step n-1 -> n of every instance: particle pass (deposit X^(n-1), gather
// grad c^(n-1), push), then the field passes that turn the deposit into
// alpha^(n) and grad c^(n).
template <typename T> DirDesc<T> make_ddesc(const Group* g) {
    const Inst& I = g->in[0];
    const sipf_params& p = I.prm;
    DirDesc<T> d{};
    d.x = (T*)I.xs[0];
    d.y = (T*)I.ys[0];
    d.z = (T*)I.zs[0];
    d.P = I.P;
    d.H = I.H;
    d.scheme = p.scheme;
    d.L = (T)p.L;
    d.halfL = (T)(p.L / 2);
    d.invL = (T)(1.0 / p.L);
    d.bscale = (T)(p.M0 / ((double)I.P * p.L * p.L * p.L));
    d.chitau = (T)(p.chi * p.dt);
    d.s = (T)(p.scheme == SIPF_STRANG ? std::sqrt(p.mu * p.dt) : std::sqrt(2.0 * p.mu * p.dt));
    d.alpha = (cplx_t<T>*)I.alpha;
    d.gc = (cplx_t<T>*)I.gc;
    d.step = g->steps;
    d.err = g->errs;
    d.k0 = (uint32_t)p.seed;
    d.k1 = (uint32_t)(p.seed >> 32);
    d.inst = p.instance;
    d.fd = make_fdesc<T>(g, 0);
    return d;
}

// Positivity-preserving deposit (the reading of Remark `smoothness` described
// in positivity.hip): after a deposit-only pass, rounds of flag + switch until
// a round switches nobody, then the clamp.  Each round reads its counts on the
// host, so a group with this option steps without graphs.
template <typename T> int positivity_rounds(Group* g) {
    if (!g->positivity) return SIPF_OK;
    const int n = (int)g->in.size();
    const uint32_t tag = ++g->pos_tag == 0 ? ++g->pos_tag : g->pos_tag;  // 0 marks "never switched"
    const PartDesc<T>* pd = pdesc_dev<T>(g, g->cur);
    // flag threshold: the fixed-point windows round each contribution to
    // 2^-18 (FP32) or 2^-51 (FP64) of a particle's mass or better; a node only
    // that far below zero is rounding left by switched particles (it has no
    // order-4 contributor left), so the threshold sits just under it -- a
    // larger one would miss real negative nodes
    const double rel = g->prec == SIPF_FP32 ? std::ldexp(1.0, -20) : std::ldexp(1.0, -44);
    std::vector<int> cnt(n);
    g->pos_switched = 0;
    g->pos_rounds = 0;
    for (int64_t round = 0; round < (int64_t)1 << 30; ++round) {
        HIPCHK(launch_fill<int>(g->pos_count, n, 0, g->stream));
        for (int i = 0; i < n; ++i) {
            const Inst& I = g->in[i];
            const T thresh = (T)(rel * I.prm.M0 / (double)I.P);
            HIPCHK(launch_pos_flag<T>((const T*)I.phi, (int64_t)grid_size(I.H, I.dim), thresh, I.pos_flag, g->stream));
            const size_t ng = grid_size(I.H, I.dim);
            HIPCHK(launch_pos_switch<T>(pd + i, I.P, I.H, I.pos_flag, I.pos_flag + ng, I.pos_flag + 2 * ng, I.pos_sw,
                                        tag, g->pos_count + i, g->stream));
        }
        HIPCHK(hipMemcpyAsync(cnt.data(), g->pos_count, n * sizeof(int), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        int64_t total = 0;
        for (int c : cnt) total += c;
        if (total == 0) break;
        g->pos_switched += total;
        g->pos_rounds++;
    }
    for (const Inst& I : g->in) HIPCHK(launch_pos_clamp<T>((T*)I.phi, (int64_t)grid_size(I.H, I.dim), g->stream));
    return SIPF_OK;
}

template <typename T> int enqueue_step(Group* g) {
    if (g->method == SIPF_METHOD_DIRECT) {
        Timed t(g, SIPF_PHASE_PARTICLES);
        const Inst& I = g->in[0];
        HIPCHK(launch_direct_step<T>(make_ddesc<T>(g), (cplx_t<T>*)I.part, I.nslices, (T*)I.gpart, I.mslices,
                                     g->stream));
        g->n_host++;
        return SIPF_OK;
    }
    if (g->since_sort >= g->resort) {
        int rc = do_sort<T>(g);
        if (rc) return rc;
    }
    if (g->positivity) {
        // deposit, the positivity rounds on it, then the push (Algorithm 4's two branches apart)
        Timed t(g, SIPF_PHASE_PARTICLES);
        HIPCHK(particles_any<T>(g, pdesc_dev<T>(g, g->cur), true, false));
        int rc = positivity_rounds<T>(g);
        if (rc) return rc;
        HIPCHK(particles_any<T>(g, pdesc_dev<T>(g, g->cur), false, true));
        g->counts_ready = false;
    } else {
        // the step before a due sort also counts the tiles of its output
        Timed t(g, SIPF_PHASE_PARTICLES);
        const bool count = counts_in_pass(g) && g->since_sort + 1 >= g->resort;
        HIPCHK(particles_any<T>(g, pdesc_dev<T>(g, g->cur), true, true, count ? g->counts : nullptr));
        g->counts_ready = count;
    }
    {
        Timed t(g, SIPF_PHASE_FWD);
        for (const HClass& h : g->classes) HIPCHK(field_fwd<T>(g, h.H, fdesc_dev<T>(g, h.first), h.count, true));
    }
    {
        Timed t(g, SIPF_PHASE_XPENCIL);
        for (const HClass& h : g->classes) HIPCHK(field_x<T>(g, h.H, fdesc_dev<T>(g, h.first), h.count, XP_STEP));
    }
    {
        Timed t(g, SIPF_PHASE_INV);
        for (const HClass& h : g->classes)
            HIPCHK(field_inv<T>(g, h.H, fdesc_dev<T>(g, h.first), h.count, g->dim));
    }
    g->since_sort++;
    g->n_host++;
    return SIPF_OK;
}

// Capture `len` steps from the current host stepping state (buffer set
// g->cur, g->since_sort steps since the last sort) on the private stream.
// Nothing runs during capture; the host-side stepping state is put back
// afterwards.
template <typename T> int capture_graph(Group* g, int len, hipGraphExec_t* out) {
    *out = nullptr;
    if (!g->cap) HIPCHK(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    const int since = g->since_sort, cur = g->cur;
    const bool counted = g->counts_ready;
    const int64_t nh = g->n_host;
    hipStream_t user = g->stream;
    g->stream = g->cap;
    HIPCHK(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    int rc = SIPF_OK;
    for (int k = 0; k < len && rc == SIPF_OK; ++k) rc = enqueue_step<T>(g);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    g->stream = user;
    g->since_sort = since;
    g->cur = cur;
    g->counts_ready = counted;
    g->n_host = nh;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(SIPF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(SIPF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    // move the graph's launch resources to the device now (on the library's
    // stream, ahead of any launch of it), so that its first replay costs what
    // every later one does
    e = hipGraphUpload(*out, g->stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(*out);
        *out = nullptr;
        return fail(SIPF_EDEVICE, std::string("hipGraphUpload: ") + hipGetErrorString(e));
    }
    return SIPF_OK;
}

// Length of the next graph segment of a run with `left` steps to go: up to
// the next due sort, or, from a due sort, two sort periods (which end on the
// starting buffer set with a sort due again, so one graph serves a long run).
int segment_len(const Group* g, int64_t left) {
    const int64_t to_sort = g->resort - g->since_sort;
    const int64_t len = to_sort > 0 ? to_sort : 2 * (int64_t)g->resort;
    return (int)std::min(left, len);
}

// Host stepping state after a segment of len steps (the sorts it holds).
void advance_state(Group* g, int len) {
    for (int k = 0; k < len; ++k) {
        if (g->since_sort >= g->resort) {
            g->cur = 1 - g->cur;
            g->since_sort = 0;
            g->counts_ready = false;
        }
        g->counts_ready = counts_in_pass(g) && g->since_sort + 1 >= g->resort;
        g->since_sort++;
    }
    g->n_host += len;
}

constexpr size_t GRAPH_CACHE_MAX = 16;

// The cached graph of a segment of len steps from the current state; captured
// on first use.
template <typename T> int segment_graph(Group* g, int len, hipGraphExec_t* out) {
    for (const auto& gs : g->gcache)
        if (gs.cur == g->cur && gs.since == g->since_sort && gs.len == len && gs.counted == (int)g->counts_ready) {
            *out = gs.exec;
            return SIPF_OK;
        }
    if (g->gcache.size() >= GRAPH_CACHE_MAX) {
        (void)hipGraphExecDestroy(g->gcache.front().exec);
        g->gcache.erase(g->gcache.begin());
    }
    int rc = capture_graph<T>(g, len, out);
    if (rc) return rc;
    g->gcache.push_back({g->cur, g->since_sort, len, (int)g->counts_ready, *out});
    return SIPF_OK;
}

template <typename T> int run_typed(Group* g, int64_t nsteps) {
    int64_t left = nsteps;
    while (left > 0) {
        if (g->graphs && !g->prof) {
            const int len = segment_len(g, left);
            hipGraphExec_t ge = nullptr;
            int rc = segment_graph<T>(g, len, &ge);
            if (rc) return rc;
            HIPCHK(hipGraphLaunch(ge, g->stream));
            advance_state(g, len);
            left -= len;
            continue;
        }
        int rc = enqueue_step<T>(g);
        if (rc) return rc;
        --left;
    }
    return SIPF_OK;
}

// Capture (without running) every graph that a run of nsteps from the
// current state will replay.
template <typename T> int prepare_typed(Group* g, int64_t nsteps) {
    if (!g->graphs) return SIPF_OK;
    const int since = g->since_sort, cur = g->cur;
    const bool counted = g->counts_ready;
    const int64_t nh = g->n_host;
    int rc = SIPF_OK;
    for (int64_t left = nsteps; left > 0 && rc == SIPF_OK;) {
        const int len = segment_len(g, left);
        hipGraphExec_t ge = nullptr;
        rc = segment_graph<T>(g, len, &ge);
        advance_state(g, len);
        left -= len;
    }
    g->since_sort = since;
    g->cur = cur;
    g->counts_ready = counted;
    g->n_host = nh;
    return rc;
}

int prepare_group(Group* g, int64_t nsteps) {
    return g->prec == SIPF_FP32 ? prepare_typed<float>(g, nsteps) : prepare_typed<double>(g, nsteps);
}

int run_group(Group* g, int64_t nsteps) {
    return g->prec == SIPF_FP32 ? run_typed<float>(g, nsteps) : run_typed<double>(g, nsteps);
}

void release_marks(Group* g) {
    for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
    g->events.clear();
    g->last_stop = nullptr;
    g->marks.clear();
}

int drain_marks(Group* g) {
    if (g->events.empty()) return SIPF_OK;
    HIPCHK(hipStreamSynchronize(g->stream));
    for (auto& m : g->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            g->prof_ms[m.phase] += ms;
            g->prof_n[m.phase] += 1;
        }
    }
    release_marks(g);
    return SIPF_OK;
}

int check_err(Group* g) {
    const int n = (int)g->in.size();
    std::vector<int> e(n, 0);
    HIPCHK(hipMemcpyAsync(e.data(), g->errs, n * sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    for (int i = 0; i < n; ++i) {
        const std::string who = n > 1 ? " (instance " + std::to_string(i) + ")" : std::string();
        if (e[i] & 2) return fail(SIPF_ENUMERIC, "non-finite initial position" + who);
        if (e[i] & 1) return fail(SIPF_ENUMERIC, "a step produced a non-finite position" + who);
        if (e[i] & 4) return fail(SIPF_EDEVICE, "the sort's tile counts did not match the particle count" + who);
    }
    return SIPF_OK;
}

// 2-D: natural (kx, ky) half spectrum H x (H/2+1) <-> the device layout
// (H/2+1) x H, ky-major with kx in the FFT storage order
void permute_spectrum2(const void* src, void* dst, int H, size_t tsize, bool to_perm) {
    const int HH = H / 2 + 1;
    const size_t e = 2 * tsize;
    for (int kx = 0; kx < H; ++kx) {
        const int p = fft_perm(H, kx);
        for (int ky = 0; ky < HH; ++ky) {
            const size_t nat = (size_t)kx * HH + ky;
            const size_t per = (size_t)ky * H + p;
            if (to_perm) std::memcpy((char*)dst + per * e, (const char*)src + nat * e, e);
            else std::memcpy((char*)dst + nat * e, (const char*)src + per * e, e);
        }
    }
}

// natural <-> permuted (kx, ky) layout of a half spectrum (host arrays of 2*T per entry)
void permute_spectrum(const void* src, void* dst, int H, size_t tsize, bool to_perm) {
    const int HH = H / 2 + 1;
    const size_t e = 2 * tsize;
    for (int kx = 0; kx < H; ++kx)
        for (int ky = 0; ky < H; ++ky) {
            const size_t nat = ((size_t)kx * H + ky) * HH;
            const size_t per = ((size_t)fft_perm(H, kx) * H + fft_perm(H, ky)) * HH;
            if (to_perm) std::memcpy((char*)dst + per * e, (const char*)src + nat * e, HH * e);
            else std::memcpy((char*)dst + nat * e, (const char*)src + per * e, HH * e);
        }
}

// Set up the group's instances (parameters already in g->in): tuning, H
// classes, device buffers and descriptors.
template <typename T> int alloc_direct(Group* g) {
    Inst& I = g->in[0];
    int rc;
    const size_t H3 = (size_t)I.H * I.H * I.H;
    const size_t V = 2 * sizeof(T);
    I.nslices = dir_slices(I.H, I.P);
    I.mslices = dir_mode_slices(I.H, I.P);
    if ((rc = dalloc(g, &I.xs[0], I.P * sizeof(T)))) return rc;
    if ((rc = dalloc(g, &I.ys[0], I.P * sizeof(T)))) return rc;
    if ((rc = dalloc(g, &I.zs[0], I.P * sizeof(T)))) return rc;
    if ((rc = dalloc(g, (void**)&I.ids[0], I.P * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(g, &I.alpha, H3 * V))) return rc;
    if ((rc = dalloc(g, &I.gc, 3 * H3 * V))) return rc;
    if ((rc = dalloc(g, &I.part, (size_t)I.nslices * H3 * V))) return rc;
    if ((rc = dalloc(g, &I.gpart, (size_t)I.mslices * 3 * I.P * sizeof(T)))) return rc;
    if ((rc = dalloc(g, (void**)&g->steps, sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(g, (void**)&g->errs, sizeof(int)))) return rc;
    HIPCHK(hipMemset(g->steps, 0, sizeof(uint32_t)));
    HIPCHK(hipMemset(g->errs, 0, sizeof(int)));
    g->classes.push_back(HClass{I.H, 0, 1});
    g->fslot.assign(1, 0);
    return SIPF_OK;
}

template <typename T> int alloc_group(Group* g) {
    if (g->method == SIPF_METHOD_DIRECT) return alloc_direct<T>(g);
    const int n = (int)g->in.size();
    const int mk = sort_max_keys();
    int rc;
    // H classes in ascending H; FieldDesc slots grouped by class
    std::vector<int> hs;
    for (const Inst& I : g->in) hs.push_back(I.H);
    std::sort(hs.begin(), hs.end());
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    g->fslot.assign(n, 0);
    int slot = 0;
    for (int H : hs) {
        HClass c{H, slot, 0};
        for (int i = 0; i < n; ++i)
            if (g->in[i].H == H) {
                g->fslot[i] = slot++;
                c.count++;
            }
        g->classes.push_back(c);
    }
    std::vector<SortChunk> chunks;
    std::vector<int> seg_off(n);
    int64_t cap = 0;
    const int sc = sort_chunk();
    for (int i = 0; i < n; ++i) {
        Inst& I = g->in[i];
        const int64_t P = I.P;
        const int d = I.dim;
        const size_t ng = grid_size(I.H, d);
        const size_t nspec = spec_size(I.H, d);
        for (int s = 0; s < 2; ++s) {
            if ((rc = dalloc(g, &I.xs[s], P * sizeof(T)))) return rc;
            if ((rc = dalloc(g, &I.ys[s], P * sizeof(T)))) return rc;
            if (d == 3 && (rc = dalloc(g, &I.zs[s], P * sizeof(T)))) return rc;
            if ((rc = dalloc(g, (void**)&I.ids[s], P * sizeof(uint32_t)))) return rc;
        }
        if ((rc = dalloc(g, &I.phi, ng * sizeof(T)))) return rc;
        if ((rc = dalloc(g, &I.B1, nspec * 2 * sizeof(T)))) return rc;
        if ((rc = dalloc(g, &I.alpha, nspec * 2 * sizeof(T)))) return rc;
        if ((rc = dalloc(g, &I.gspec, d * nspec * 2 * sizeof(T)))) return rc;
        if ((rc = dalloc(g, &I.G, d * ng * sizeof(T)))) return rc;
        for (int64_t b = 0; b < P; b += sc) chunks.push_back(SortChunk{b, i, 0});
        const int nt = (I.H + I.tile - 1) / I.tile;  // tiles per axis, the last may be partial
        seg_off[i] = (int)cap;
        const int64_t ch = std::min(g->chunk, g->adj_chunk);  // the smaller item size gives more items
        cap += (P + ch - 1) / ch + (d == 2 ? (int64_t)nt * nt : (int64_t)nt * nt * nt);
    }
    if (cap >= (int64_t(1) << 31) || chunks.size() >= (size_t(1) << 31))
        return fail(SIPF_EINVAL, "too many particles in one group");
    g->items_cap = (int)cap;
    g->nchunks = (int)chunks.size();
    if ((rc = dalloc(g, (void**)&g->counts, (size_t)n * mk * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(g, (void**)&g->cursor, (size_t)n * mk * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(g, (void**)&g->steps, n * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(g, (void**)&g->errs, n * sizeof(int)))) return rc;
    if ((rc = dalloc(g, &g->pdesc, 2 * n * sizeof(PartDesc<T>)))) return rc;
    if ((rc = dalloc(g, &g->fdesc, n * sizeof(FieldDesc<T>)))) return rc;
    if ((rc = dalloc(g, (void**)&g->chunks, chunks.size() * sizeof(SortChunk)))) return rc;
    if ((rc = dalloc(g, (void**)&g->seg, cap * sizeof(WorkItem)))) return rc;
    if ((rc = dalloc(g, (void**)&g->seg_off, n * sizeof(int)))) return rc;
    if ((rc = dalloc(g, (void**)&g->seg_n, n * sizeof(int)))) return rc;
    if ((rc = dalloc(g, (void**)&g->items, cap * sizeof(WorkItem)))) return rc;
    if ((rc = dalloc(g, (void**)&g->nitems, 16))) return rc;
    HIPCHK(hipMemcpy(g->chunks, chunks.data(), chunks.size() * sizeof(SortChunk), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->seg_off, seg_off.data(), n * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(g->nitems, 0, 16));
    HIPCHK(hipMemset(g->counts, 0, (size_t)n * mk * sizeof(uint32_t)));
    HIPCHK(hipMemset(g->steps, 0, n * sizeof(uint32_t)));
    HIPCHK(hipMemset(g->errs, 0, n * sizeof(int)));
    if (g->positivity) {
        if ((rc = dalloc(g, (void**)&g->pos_count, n * sizeof(int)))) return rc;
        for (Inst& I : g->in) {
            if ((rc = dalloc(g, (void**)&I.pos_sw, I.P * sizeof(uint32_t)))) return rc;
            if ((rc = dalloc(g, (void**)&I.pos_flag, 3 * grid_size(I.H, I.dim)))) return rc;  // flags, 2 scratch
            HIPCHK(hipMemset(I.pos_sw, 0, I.P * sizeof(uint32_t)));
        }
    }
    g->pgrid = std::max(1, std::min(g->items_cap, g->dim == 2 ? particle_resident_blocks2<T>(g->scheme, g->win_bytes)
                                                                : particle_resident_blocks<T>(g->scheme, g->win_bytes,
                                                                                              g->sorted)));
    return upload_descs<T>(g);
}

// Positions of instance i (AoS, host or device) -> SoA set 0, wrapped, ids 0..P-1.
template <typename T> int load_positions(Group* g, int i, const void* X0, int on_device) {
    const int64_t P = g->in[i].P;
    const PartDesc<T> d0 = make_pdesc<T>(g, i, 0);
    const T L = (T)g->in[i].prm.L;
    if (on_device) {
        HIPCHK(launch_load_positions<T>((const T*)X0, P, L, d0, g->errs + i, g->stream));
        return SIPF_OK;
    }
    // host positions go through a temporary device buffer freed before return
    void* tmp = nullptr;
    const int64_t nv = (int64_t)g->in[i].dim * P;
    if (hipMalloc(&tmp, nv * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SIPF_ENOMEM, "hipMalloc failed for the staging buffer");
    }
    hipError_t e = hipMemcpyAsync(tmp, X0, nv * sizeof(T), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = launch_load_positions<T>((const T*)tmp, P, L, d0, g->errs + i, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(SIPF_EDEVICE, std::string("loading X0: ") + hipGetErrorString(e));
    return SIPF_OK;
}

// alpha0 (natural half spectrum) -> the full spectrum of a direct context,
// extended by Hermitian symmetry alpha_{-q} = conj(alpha_q)
template <typename T> int init_direct_fields(Group* g, const void* alpha0, int alpha0_on_device) {
    const Inst& I = g->in[0];
    const int H = I.H, HH = H / 2 + 1;
    const size_t H3 = (size_t)H * H * H;
    if (alpha0 == nullptr) {
        HIPCHK(launch_fill<T>((T*)I.alpha, 2 * H3, (T)0, g->stream));
        return SIPF_OK;
    }
    std::vector<T> half(2 * (size_t)H * H * HH), full(2 * H3);
    if (alpha0_on_device) HIPCHK(hipMemcpy(half.data(), alpha0, half.size() * sizeof(T), hipMemcpyDeviceToHost));
    else std::memcpy(half.data(), alpha0, half.size() * sizeof(T));
    for (T v : half)
        if (!std::isfinite((double)v)) return fail(SIPF_ENUMERIC, "non-finite alpha0");
    for (int kx = 0; kx < H; ++kx)
        for (int ky = 0; ky < H; ++ky)
            for (int kz = 0; kz < H; ++kz) {
                const bool direct = kz <= H / 2;
                const int sx = direct ? kx : (H - kx) % H, sy = direct ? ky : (H - ky) % H;
                const int sz = direct ? kz : H - kz;
                const size_t src = ((size_t)sx * H + sy) * HH + sz, dst = ((size_t)kx * H + ky) * H + kz;
                full[2 * dst] = half[2 * src];
                full[2 * dst + 1] = direct ? half[2 * src + 1] : -half[2 * src + 1];
            }
    HIPCHK(hipMemcpy(I.alpha, full.data(), full.size() * sizeof(T), hipMemcpyHostToDevice));
    return SIPF_OK;
}

template <typename T> int init_fields(Group* g, int i, const void* alpha0, int alpha0_on_device) {
    if (g->method == SIPF_METHOD_DIRECT) return init_direct_fields<T>(g, alpha0, alpha0_on_device);
    const Inst& I = g->in[i];
    const int H = I.H;
    const size_t nspec = spec_size(H, I.dim);
    const size_t ng = grid_size(H, I.dim);
    HIPCHK(launch_fill<T>((T*)I.phi, ng, (T)0, g->stream));
    HIPCHK(launch_fill<T>((T*)I.G, I.dim * ng, (T)0, g->stream));
    if (alpha0 == nullptr) {
        HIPCHK(launch_fill<T>((T*)I.alpha, 2 * nspec, (T)0, g->stream));
        return SIPF_OK;
    }
    std::vector<T> nat(2 * nspec), per(2 * nspec);
    if (alpha0_on_device) HIPCHK(hipMemcpy(nat.data(), alpha0, nat.size() * sizeof(T), hipMemcpyDeviceToHost));
    else std::memcpy(nat.data(), alpha0, nat.size() * sizeof(T));
    for (T v : nat)
        if (!std::isfinite((double)v)) return fail(SIPF_ENUMERIC, "non-finite alpha0");
    if (I.dim == 2) permute_spectrum2(nat.data(), per.data(), H, sizeof(T), true);
    else permute_spectrum(nat.data(), per.data(), H, sizeof(T), true);
    HIPCHK(hipMemcpyAsync(I.alpha, per.data(), per.size() * sizeof(T), hipMemcpyHostToDevice, g->stream));
    HIPCHK(field_x<T>(g, H, fdesc_dev<T>(g, g->fslot[i]), 1, XP_GRAD));
    HIPCHK(field_inv<T>(g, H, fdesc_dev<T>(g, g->fslot[i]), 1, I.dim));
    HIPCHK(hipStreamSynchronize(g->stream));
    return SIPF_OK;
}

// Full initialisation of a group whose g->in holds validated parameters.
template <typename T>
int init_group(Group* g, const void* const* X0, int x0_on_device, const void* alpha0, int alpha0_on_device) {
    int rc;
    if ((rc = alloc_group<T>(g))) return rc;
    for (int i = 0; i < (int)g->in.size(); ++i) {
        if ((rc = load_positions<T>(g, i, X0[i], x0_on_device))) return rc;
        if ((rc = init_fields<T>(g, i, i == 0 ? alpha0 : nullptr, alpha0_on_device))) return rc;
    }
    g->cur = 0;
    if (g->method != SIPF_METHOD_DIRECT && (rc = do_sort<T>(g))) return rc;
    HIPCHK(hipStreamSynchronize(g->stream));
    return check_err(g);
}

void free_group(Group* g) {
    if (!g) return;
    release_marks(g);
    for (auto& gs : g->gcache)
        if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
    g->gcache.clear();
    if (g->cap) (void)hipStreamDestroy(g->cap);
    for (void* p : g->allocs) (void)hipFree(p);
}

// Shared set-up of contexts and batches: validation, host checks, tuning.
int setup_group(Group* g, int32_t n, const sipf_params* prm, const int64_t* P, const void* const* X0,
                int x0_on_device, void* hip_stream) {
    if (n < 1 || n > 1024) return fail(SIPF_EINVAL, "instance count must be in [1, 1024]");
    if (!prm || !P || !X0) return fail(SIPF_EINVAL, "NULL argument");
    for (int i = 0; i < n; ++i) {
        int rc = validate(&prm[i], P[i]);
        if (rc) return n > 1 ? fail(rc, "instance " + std::to_string(i) + ": " + g_err) : rc;
        if (!X0[i]) return fail(SIPF_EINVAL, "X0 is NULL");
        if (prm[i].precision != prm[0].precision) return fail(SIPF_EINVAL, "all instances must share the precision");
        if (prm[i].scheme != prm[0].scheme) return fail(SIPF_EINVAL, "all instances must share the scheme");
        if (dim_of(&prm[i]) != dim_of(&prm[0])) return fail(SIPF_EINVAL, "all instances must share the dimension");
        if (prm[i].positivity != prm[0].positivity)
            return fail(SIPF_EINVAL, "all instances must share the positivity option");
        if (prm[i].particle_pass != prm[0].particle_pass)
            return fail(SIPF_EINVAL, "all instances must share the particle pass");
    }
    if (prm[0].method == SIPF_METHOD_DIRECT && n != 1)
        return fail(SIPF_EINVAL, "the direct SIPF method runs single contexts, not batches");
    const size_t ts = prm[0].precision == SIPF_FP32 ? 4 : 8;
    if (!x0_on_device) {
        // reject non-finite host input before touching the device
        for (int i = 0; i < n; ++i)
            for (int64_t j = 0; j < dim_of(&prm[i]) * P[i]; ++j) {
                const double v = ts == 4 ? (double)((const float*)X0[i])[j] : ((const double*)X0[i])[j];
                if (!std::isfinite(v)) return fail(SIPF_ENUMERIC, "non-finite value in X0");
            }
    }
    g->prec = prm[0].precision;
    g->dim = dim_of(&prm[0]);
    g->method = prm[0].method;
    if (g->method == SIPF_METHOD_DIRECT) g->graphs = false;
    g->positivity = prm[0].positivity != 0;
    if (g->positivity) g->graphs = false;  // the rounds read their counts on the host
    g->tsize = ts;
    g->scheme = prm[0].scheme;
    g->stream = (hipStream_t)hip_stream;
    g->resort = default_resort(&prm[0]);
    for (int i = 1; i < n; ++i) g->resort = std::min(g->resort, default_resort(&prm[i]));
    int64_t total_P = 0;
    for (int i = 0; i < n; ++i) total_P += P[i];
    g->chunk = default_chunk(&prm[0], total_P);
    g->adj_chunk = default_adj_chunk(&prm[0], g->chunk);
    g->win_bytes = particle_window_bytes(g->prec == SIPF_FP64);
    g->sorted = sorted_pass(&prm[0], n);
    g->in.resize(n);
    for (int i = 0; i < n; ++i) {
        Inst& I = g->in[i];
        I.prm = prm[i];
        I.P = P[i];
        I.H = prm[i].H;
        I.dim = dim_of(&prm[i]);
        I.tile = default_tile(&prm[i]);
        if (!is_pow2(I.H)) g->pow2 = false;
    }
    return SIPF_OK;
}

int init_any(Group* g, const void* const* X0, int x0_on_device, const void* alpha0, int alpha0_on_device) {
    return g->prec == SIPF_FP32 ? init_group<float>(g, X0, x0_on_device, alpha0, alpha0_on_device)
                                : init_group<double>(g, X0, x0_on_device, alpha0, alpha0_on_device);
}

template <typename T> int get_field_typed(Group* g, int i, int which, void* out, int on_device) {
    const Inst& I = g->in[i];
    if (g->method == SIPF_METHOD_DIRECT) {
        if (which != SIPF_FIELD_ALPHA) return fail(SIPF_EINVAL, "a direct SIPF context has no grids");
        const int H = I.H, HH = H / 2 + 1;
        std::vector<T> full(2 * (size_t)H * H * H), half(2 * (size_t)H * H * HH);
        HIPCHK(hipMemcpyAsync(full.data(), I.alpha, full.size() * sizeof(T), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        for (size_t r = 0; r < (size_t)H * H; ++r)
            std::memcpy(half.data() + 2 * r * HH, full.data() + 2 * r * H, 2 * HH * sizeof(T));
        if (on_device) HIPCHK(hipMemcpy(out, half.data(), half.size() * sizeof(T), hipMemcpyHostToDevice));
        else std::memcpy(out, half.data(), half.size() * sizeof(T));
        return check_err(g);
    }
    const int H = I.H;
    const size_t ng = grid_size(H, I.dim);
    const size_t nspec = spec_size(H, I.dim);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (which == SIPF_FIELD_RHO) {
        // deposit-only pass over every instance, then clear every deposit again
        HIPCHK(particles_any<T>(g, pdesc_dev<T>(g, g->cur), true, false));
        int rc = positivity_rounds<T>(g);
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(out, I.phi, ng * sizeof(T), kind, g->stream));
        for (const Inst& J : g->in) HIPCHK(launch_fill<T>((T*)J.phi, (int64_t)grid_size(J.H, J.dim), (T)0, g->stream));
    } else if (which == SIPF_FIELD_GRAD) {
        HIPCHK(hipMemcpyAsync(out, I.G, I.dim * ng * sizeof(T), kind, g->stream));
    } else if (which == SIPF_FIELD_ALPHA) {
        std::vector<T> per(2 * nspec), nat(2 * nspec);
        HIPCHK(hipMemcpyAsync(per.data(), I.alpha, per.size() * sizeof(T), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        if (I.dim == 2) permute_spectrum2(per.data(), nat.data(), H, sizeof(T), false);
        else permute_spectrum(per.data(), nat.data(), H, sizeof(T), false);
        if (on_device) HIPCHK(hipMemcpy(out, nat.data(), nat.size() * sizeof(T), hipMemcpyHostToDevice));
        else std::memcpy(out, nat.data(), nat.size() * sizeof(T));
    } else {
        return fail(SIPF_EINVAL, "unknown field");
    }
    HIPCHK(hipStreamSynchronize(g->stream));
    return check_err(g);
}

template <typename T> int get_positions_typed(Group* g, int i, void* out, int on_device) {
    const PartDesc<T> d = make_pdesc<T>(g, i, g->cur);
    if (on_device) {
        HIPCHK(launch_unsort<T>(&d, (T*)out, g->stream));
    } else {
        void* tmp = nullptr;
        const size_t bytes = (size_t)d.dim * d.P * sizeof(T);
        HIPCHK(hipMalloc(&tmp, bytes));
        hipError_t e = launch_unsort<T>(&d, (T*)tmp, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(SIPF_EDEVICE, std::string("get_positions: ") + hipGetErrorString(e));
    }
    HIPCHK(hipStreamSynchronize(g->stream));
    return check_err(g);
}

// Diagnostics of every instance: deposit of the current positions, forward
// plane pass (consuming the deposit, step counters untouched), x pencils with
// the Gaussian factor, inverse plane pass of one component into the deposit
// grid (rho_num), then the reductions; the deposit grids are cleared again.
template <typename T> int diagnostics_typed(Group* g, sipf_diag* out) {
    const int n = (int)g->in.size();
    const size_t part_b = (size_t)n * DIAG_MAX_BLOCKS * DIAG_NVAL * sizeof(double);
    const size_t res_b = (size_t)n * DIAG_NVAL * sizeof(double);
    const size_t dd_b = ((size_t)n * sizeof(DiagDesc<T>) + 255) / 256 * 256;
    const size_t fd_b = (size_t)n * sizeof(FieldDesc<T>);
    int rc;
    if (!g->diag && (rc = dalloc(g, &g->diag, part_b + res_b + dd_b + fd_b))) return rc;
    char* base = (char*)g->diag;
    double* part = (double*)base;
    double* res = (double*)(base + part_b);
    DiagDesc<T>* ddev = (DiagDesc<T>*)(base + part_b + res_b);
    FieldDesc<T>* fdev = (FieldDesc<T>*)(base + part_b + res_b + dd_b);
    std::vector<DiagDesc<T>> dd(n);
    std::vector<FieldDesc<T>> fd(n);
    int nbmax = 1;
    for (int i = 0; i < n; ++i) {
        const Inst& I = g->in[i];
        FieldDesc<T> f = make_fdesc<T>(g, i);
        f.G = (T*)I.phi;
        f.step = nullptr;
        fd[g->fslot[i]] = f;
        DiagDesc<T> d{};
        d.rho = (const T*)I.phi;
        d.alpha = (const cplx_t<T>*)I.alpha;
        d.x = (const T*)I.xs[g->cur];
        d.y = (const T*)I.ys[g->cur];
        d.z = (const T*)I.zs[g->cur];
        d.P = I.P;
        d.H = I.H;
        d.dim = I.dim;
        d.pm = I.H > 256 ? I.H / 16 : I.H;
        d.pt = I.H > 256 ? 16 : 1;
        d.n2 = fft_perm(d.pm, 1);
        d.n1 = d.pm / d.n2;
        d.nb = diag_blocks(I.P, (int64_t)grid_size(I.H, I.dim));
        nbmax = std::max(nbmax, d.nb);
        dd[i] = d;
    }
    HIPCHK(hipMemcpyAsync(ddev, dd.data(), n * sizeof(DiagDesc<T>), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(fdev, fd.data(), fd_b, hipMemcpyHostToDevice, g->stream));
    HIPCHK(particles_any<T>(g, pdesc_dev<T>(g, g->cur), true, false));
    if (int rc = positivity_rounds<T>(g)) return rc;
    for (const HClass& h : g->classes) {
        HIPCHK(field_fwd<T>(g, h.H, fdev + h.first, h.count, true));
        HIPCHK(field_x<T>(g, h.H, fdev + h.first, h.count, XP_RHO));
        HIPCHK(field_inv<T>(g, h.H, fdev + h.first, h.count, 1));
    }
    HIPCHK(launch_diag<T>(ddev, n, nbmax, part, res, g->stream));
    std::vector<double> host((size_t)n * DIAG_NVAL);
    std::vector<uint32_t> steps(n);
    HIPCHK(hipMemcpyAsync(host.data(), res, res_b, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipMemcpyAsync(steps.data(), g->steps, n * sizeof(uint32_t), hipMemcpyDeviceToHost, g->stream));
    for (const Inst& J : g->in) HIPCHK(launch_fill<T>((T*)J.phi, (int64_t)grid_size(J.H, J.dim), (T)0, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    for (int i = 0; i < n; ++i) {
        const Inst& I = g->in[i];
        const double* v = host.data() + (size_t)i * DIAG_NVAL;
        const double L = I.prm.L, h = L / I.H;
        const double hd = I.dim == 2 ? h * h : h * h * h, Ld = I.dim == 2 ? L * L : L * L * L;
        sipf_diag& o = out[i];
        o.step = steps[i];
        o.mass = v[0] * hd;
        o.rho_max = v[1];
        o.hf_share = v[2] > 0 ? v[3] / v[2] : 0.0;
        o.c_integral = Ld * v[4];
        o.r_num = v[5] / (double)I.P;
        o.m2 = v[6] / (double)I.P;
    }
    return check_err(g);
}

int diagnostics_any(Group* g, sipf_diag* out) {
    return g->prec == SIPF_FP32 ? diagnostics_typed<float>(g, out) : diagnostics_typed<double>(g, out);
}

int get_field_any(Group* g, int i, int which, void* out, int on_device) {
    return g->prec == SIPF_FP32 ? get_field_typed<float>(g, i, which, out, on_device)
                                : get_field_typed<double>(g, i, which, out, on_device);
}
int get_positions_any(Group* g, int i, void* out, int on_device) {
    return g->prec == SIPF_FP32 ? get_positions_typed<float>(g, i, out, on_device)
                                : get_positions_typed<double>(g, i, out, on_device);
}

int get_step_any(Group* g, int i, int64_t* n) {
    uint32_t s = 0;
    HIPCHK(hipMemcpyAsync(&s, g->steps + i, sizeof(s), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *n = s;
    return SIPF_OK;
}

int profile_any(Group* g, int enable) {
    int rc = drain_marks(g);
    if (rc) return rc;
    for (int i = 0; i < SIPF_NPHASES; ++i) {
        g->prof_ms[i] = 0;
        g->prof_n[i] = 0;
    }
    g->prof = enable != 0;
    return SIPF_OK;
}

int profile_read_any(Group* g, double* ms, int64_t* launches) {
    int rc = drain_marks(g);
    if (rc) return rc;
    for (int i = 0; i < SIPF_NPHASES; ++i) {
        ms[i] = g->prof_ms[i];
        launches[i] = g->prof_n[i];
    }
    return SIPF_OK;
}

int destroy_any(Group* g) {
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    else (void)hipDeviceSynchronize();
    free_group(g);
    return SIPF_OK;
}

// ---------------------------------------------------------------------------
// pathwise adjoint of a single-instance context
// ---------------------------------------------------------------------------

// Device buffer freed when it goes out of scope (adjoint temporaries).
// Device work buffers of the adjoint are kept for later calls instead of
// freed: an FP64 adjoint of 2e6 particles holds about 2 GB of tape, segment
// and noise buffers, and hipMalloc + hipFree of those cost milliseconds per
// call (hipFree also waits for the device).  Cached blocks are reused by any
// later adjoint on the same device whose request fits (best fit, at most
// twice the request) and returned by sipf_release_cached_memory.
struct BufCache {
    struct Blk {
        int dev;
        size_t n;
        void* p;
    };
    std::mutex mu;
    std::vector<Blk> free_blocks;
    hipError_t get(size_t n, void** out) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lock(mu);
            int best = -1;
            for (int i = 0; i < (int)free_blocks.size(); ++i) {
                const Blk& b = free_blocks[i];
                if (b.dev == dev && b.n >= n && b.n <= 2 * n && (best < 0 || b.n < free_blocks[best].n)) best = i;
            }
            if (best >= 0) {
                *out = free_blocks[best].p;
                free_blocks.erase(free_blocks.begin() + best);
                return hipSuccess;
            }
        }
        return hipMalloc(out, n);
    }
    void put(void* p, size_t n) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(p);
            return;
        }
        std::lock_guard<std::mutex> lock(mu);
        free_blocks.push_back({dev, n, p});
    }
    void release() {
        std::lock_guard<std::mutex> lock(mu);
        for (const Blk& b : free_blocks) {
            int cur = 0;
            if (hipGetDevice(&cur) == hipSuccess && cur != b.dev) (void)hipSetDevice(b.dev);
            (void)hipFree(b.p);
            if (cur != b.dev) (void)hipSetDevice(cur);
        }
        free_blocks.clear();
    }
};
BufCache g_buf_cache;

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    ~DevBuf() {
        if (p) g_buf_cache.put(p, n);
    }
    hipError_t alloc(size_t bytes) {
        n = bytes ? bytes : 16;
        return g_buf_cache.get(n, &p);
    }
};

// Waits for a stream when it goes out of scope (declared after a function's
// DevBufs, it runs before they return to the cache, on every exit path).
struct StreamSync {
    hipStream_t s;
    ~StreamSync() { (void)hipStreamSynchronize(s); }
};

template <typename T> PartDesc<T> pdesc_on(const Group* g, T* x, T* y, T* z, uint32_t* id) {
    PartDesc<T> d = make_pdesc<T>(g, 0, 0);
    d.x = x;
    d.y = y;
    d.z = z;
    d.id = id;
    return d;
}

// Gradient grids of alpha (the instance's alpha buffer) into its G.
template <typename T> int recompute_grad(Group* g) {
    const FieldDesc<T>* fd = fdesc_dev<T>(g, 0);
    HIPCHK(launch_xpencils<T>(g->in[0].H, fd, 1, XP_GRAD, g->stream));
    HIPCHK(launch_inv_planes<T>(g->in[0].H, fd, 1, 3, g->stream));
    return SIPF_OK;
}

// Reverse mode of N steps of a single-instance context along its noise path.
//   forward:  the usual steps, taping alpha^(n-1) every step and X^(n-1) every
//             K steps;
//   per segment [base, base + len), last segment first:
//     sort X^(base) into tile order (this rebuilds the work items; later
//     positions of the segment keep that order), recompute X^(base+m) and the
//     gradient grids G^(base+m) of the segment, then for n = base+len .. base+1
//       phibar^(n-1) = L^-3 C2R(B abar^(n))              (n < N)
//       reverse particle pass at X^(n-1) with G^(n-1): Xbar, Gbar, chibar, sbar
//       abar^(n-1)   = A abar^(n) + sum_d (-i xi_d Phi) R2C(Gbar_d).
// Position cotangents live in segment order during a segment and by particle
// id between segments.
template <typename T>
int adjoint_typed(Group* c, int64_t N, int K, const T* phibar_in, double* loss_out, double* dchi_out,
                  double* dmu_out, T* dX0) {
    using V = cplx_t<T>;
    Inst& I = c->in[0];
    int64_t n0 = 0;
    int rc;
    if ((rc = get_step_any(c, 0, &n0))) return rc;
    if (n0 != 0 || c->n_host != 0) return fail(SIPF_ESTATE, "sipf_adjoint needs a context at step 0");
    if (K > N) K = (int)N;
    const int H = I.H;
    const int64_t P = I.P;
    const size_t H3 = (size_t)H * H * H;
    const size_t nspec = (size_t)H * H * (H / 2 + 1);
    const int64_t nseg = (N + K - 1) / K;
    const size_t pos_bytes = (size_t)P * (3 * sizeof(T) + sizeof(uint32_t));
    auto need = [&](DevBuf& b, size_t n) -> int {
        if (b.alloc(n) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SIPF_ENOMEM, "adjoint: device allocation failed");
        }
        return SIPF_OK;
    };
    DevBuf tape, ckpt, seg, Gseg, xbar, xbs, Gbar, phibar, abar, aN, scr, gs1, fdS, fdA, fdR, pdR, pdS, consts, acc,
        zseg;
    const StreamSync drain{c->stream};  // no work on these buffers is pending when they go back to the cache
    // FP64: the segment's forward recompute keeps each step's normals for the
    // reverse pass, whose double-precision Box-Muller would otherwise redraw
    // them (about 0.1 ms per step on the adjoint workload; the normals cost
    // 48 bytes per particle written and read once).  FP32 redraws them: there
    // the draw hides under the pass's other work.
    const bool keep_noise = sizeof(T) == 8 && K > 1;
    // The gradient grids of a segment's taped alpha states do not depend on
    // its recomputed positions: they are made GB steps at a time in one
    // batched launch per field pass (each step with its own spectra), instead
    // of one small launch pair per step.
    const int GB = std::min(K, 16);
    if ((rc = need(tape, (size_t)N * nspec * sizeof(V)))) return rc;
    if ((rc = need(ckpt, (size_t)nseg * pos_bytes))) return rc;
    if ((rc = need(seg, (size_t)K * pos_bytes))) return rc;
    if ((rc = need(Gseg, (size_t)K * 3 * H3 * sizeof(T)))) return rc;
    if ((rc = need(xbar, (size_t)P * 3 * sizeof(T)))) return rc;
    if ((rc = need(xbs, (size_t)P * 3 * sizeof(T)))) return rc;
    if ((rc = need(Gbar, 3 * H3 * sizeof(T)))) return rc;
    if ((rc = need(phibar, H3 * sizeof(T)))) return rc;
    if ((rc = need(abar, nspec * sizeof(V)))) return rc;
    if ((rc = need(aN, nspec * sizeof(V)))) return rc;
    if ((rc = need(scr, (size_t)GB * 3 * nspec * sizeof(V)))) return rc;
    if ((rc = need(gs1, nspec * sizeof(V)))) return rc;
    if ((rc = need(fdS, sizeof(FieldDesc<T>)))) return rc;
    if ((rc = need(fdA, sizeof(FieldDesc<T>)))) return rc;
    if ((rc = need(fdR, (size_t)N * sizeof(FieldDesc<T>)))) return rc;
    if ((rc = need(pdR, (size_t)N * sizeof(PartDesc<T>)))) return rc;
    if ((rc = need(pdS, (size_t)(nseg + 1) * sizeof(PartDesc<T>)))) return rc;
    if ((rc = need(consts, (size_t)N * sizeof(uint32_t)))) return rc;
    if ((rc = need(acc, 4 * sizeof(double)))) return rc;
    if (keep_noise && (rc = need(zseg, (size_t)(K - 1) * 6 * P * sizeof(T)))) return rc;
    // position slot j of a buffer: x, y, z, id
    auto slot = [&](void* base, int64_t j, T*& x, T*& y, T*& z, uint32_t*& id) {
        char* b = (char*)base + (size_t)j * pos_bytes;
        x = (T*)b;
        y = x + P;
        z = y + P;
        id = (uint32_t*)(z + P);
    };
    T* gseg = (T*)Gseg.p;
    {
        // adjoint field descriptors: source (abar -> phibar) and accumulation (Gbar -> abar)
        FieldDesc<T> f = make_fdesc<T>(c, 0);
        f.alpha = (V*)abar.p;
        f.gspec = (V*)gs1.p;
        f.G = (T*)phibar.p;
        f.step = nullptr;
        HIPCHK(hipMemcpy(fdS.p, &f, sizeof(f), hipMemcpyHostToDevice));
        f = make_fdesc<T>(c, 0);
        f.phi = (T*)Gbar.p;
        f.B1 = (V*)scr.p;
        f.alpha = (V*)abar.p;
        f.gspec = (V*)gs1.p;  // the fused accumulation + source pass writes the source spectrum here
        f.step = nullptr;
        HIPCHK(hipMemcpy(fdA.p, &f, sizeof(f), hipMemcpyHostToDevice));
        // per step t: gradient grids of the taped alpha^(t) into the segment store,
        // and the push of step t + 1 in place on segment slot (t mod K) + 1
        std::vector<FieldDesc<T>> fr(N);
        std::vector<PartDesc<T>> pr(N);
        for (int64_t t = 0; t < N; ++t) {
            fr[t] = make_fdesc<T>(c, 0);
            fr[t].alpha = (V*)tape.p + (size_t)t * nspec;
            fr[t].gspec = (V*)scr.p + (size_t)((t % K) % GB) * 3 * nspec;
            fr[t].G = gseg + (size_t)(t % K) * 3 * H3;
            fr[t].step = nullptr;
            // reads segment slot t mod K, writes slot t mod K + 1 (used while that is < K)
            const int sl = (int)(t % K) + 1 < K ? (int)(t % K) + 1 : 0;
            T *x, *y, *z, *x1, *y1, *z1;
            uint32_t *id, *id1;
            slot(seg.p, (int)(t % K), x, y, z, id);
            slot(seg.p, sl, x1, y1, z1, id1);
            pr[t] = pdesc_on<T>(c, x, y, z, id);
            pr[t].ox = x1;
            pr[t].oy = y1;
            pr[t].oz = z1;
            pr[t].oid = id1;
            pr[t].G = gseg + (size_t)(t % K) * 3 * H3;
            pr[t].step = (const uint32_t*)consts.p + t;
            // the normals of step t + 1, read back by the reverse pass of that step
            pr[t].zout = keep_noise && (int)(t % K) + 1 < K ? (T*)zseg.p + (size_t)(t % K) * 6 * P : nullptr;
        }
        HIPCHK(hipMemcpy(fdR.p, fr.data(), fr.size() * sizeof(FieldDesc<T>), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(pdR.p, pr.data(), pr.size() * sizeof(PartDesc<T>), hipMemcpyHostToDevice));
        // sort descriptors: checkpoint j (source) and segment slot 0 (destination)
        std::vector<PartDesc<T>> ps(nseg + 1);
        for (int64_t j = 0; j <= nseg; ++j) {
            T *x, *y, *z;
            uint32_t* id;
            slot(j < nseg ? ckpt.p : seg.p, j < nseg ? j : 0, x, y, z, id);
            ps[j] = pdesc_on<T>(c, x, y, z, id);
        }
        HIPCHK(hipMemcpy(pdS.p, ps.data(), ps.size() * sizeof(PartDesc<T>), hipMemcpyHostToDevice));
        HIPCHK(launch_iota_u32((uint32_t*)consts.p, N, c->stream));
    }
    const FieldDesc<T>* fr_dev = (const FieldDesc<T>*)fdR.p;
    // gradient grids of the taped alpha^(t), t = t0 .. t0 + len - 1 (within one
    // segment), into the segment store
    auto grad_of_tape = [&](int64_t t0, int len) -> int {
        for (int b = 0; b < len; b += GB) {
            const int cnt = std::min(GB, len - b);
            HIPCHK(launch_xpencils<T>(H, fr_dev + t0 + b, cnt, XP_GRAD, c->stream));
            HIPCHK(launch_inv_planes<T>(H, fr_dev + t0 + b, cnt, 3, c->stream));
        }
        return SIPF_OK;
    };

    // ---- forward with tape: alpha^(n-1) every step, X^(n-1) every K steps
    for (int64_t n = 1; n <= N; ++n) {
        if ((n - 1) % K == 0) {
            T *x, *y, *z;
            uint32_t* id;
            slot(ckpt.p, (n - 1) / K, x, y, z, id);
            HIPCHK(launch_copy_positions<T>(x, y, z, id, (const T*)I.xs[c->cur], (const T*)I.ys[c->cur],
                                            (const T*)I.zs[c->cur], I.ids[c->cur], P, c->stream));
        }
        HIPCHK(hipMemcpyAsync((V*)tape.p + (size_t)(n - 1) * nspec, I.alpha, nspec * sizeof(V),
                              hipMemcpyDeviceToDevice, c->stream));
        if ((rc = enqueue_step<T>(c))) return rc;
    }
    HIPCHK(hipMemcpyAsync(aN.p, I.alpha, nspec * sizeof(V), hipMemcpyDeviceToDevice, c->stream));
    if (c->counts_ready) {
        // the last forward step took the tile counts of a sort that the
        // segment sorts below do not consume: clear them
        HIPCHK(launch_fill<float>((float*)c->counts, (int64_t)sort_max_keys(), 0.0f, c->stream));
        c->counts_ready = false;
    }

    // ---- loss and its cotangent phibar^(N)
    HIPCHK(launch_zero_f64((double*)acc.p, 4, c->stream));
    HIPCHK(launch_particles<T>(pdesc_dev<T>(c, c->cur), c->items, c->nitems, c->pgrid, true, false, c->scheme,
                               c->win_bytes, c->pow2, c->sorted, c->stream));
    if (phibar_in) {
        HIPCHK(launch_dot<T>(phibar_in, (const T*)I.phi, (int64_t)H3, (double*)acc.p + 2, c->stream));
        HIPCHK(hipMemcpyAsync(phibar.p, phibar_in, H3 * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    } else {
        HIPCHK(launch_dot<T>((const T*)I.phi, (const T*)I.phi, (int64_t)H3, (double*)acc.p + 2, c->stream));
        HIPCHK(launch_fill<T>((T*)phibar.p, (int64_t)H3, (T)0, c->stream));
        HIPCHK(launch_axpby<T>((T*)phibar.p, (const T*)I.phi, (T)2, (T)0, (int64_t)H3, c->stream));
    }
    HIPCHK(launch_fill<T>((T*)I.phi, (int64_t)H3, (T)0, c->stream));

    AdjDesc<T> ad{};
    ad.P = P;
    ad.H = H;
    ad.scheme = c->scheme;
    const PartDesc<T> ref = make_pdesc<T>(c, 0, c->cur);
    ad.hl = ref.hl;
    ad.wmass = ref.wmass;
    ad.chitau = ref.chitau;
    ad.tau = (T)I.prm.dt;
    ad.s = ref.s;
    ad.k0 = ref.k0;
    ad.k1 = ref.k1;
    ad.inst = ref.inst;
    ad.gmargin = ref.gmargin;
    ad.xbar = (T*)xbar.p;
    ad.xbx = (T*)xbs.p;
    ad.xby = ad.xbx + P;
    ad.xbz = ad.xby + P;
    ad.Gbar = (T*)Gbar.p;
    ad.acc = (double*)acc.p;
    // seed: Xbar^(N) (by id) from phibar^(N) at X^(N)
    ad.x = (const T*)I.xs[c->cur];
    ad.y = (const T*)I.ys[c->cur];
    ad.z = (const T*)I.zs[c->cur];
    ad.id = I.ids[c->cur];
    ad.G = (const T*)I.G;
    ad.phibar = (const T*)phibar.p;
    HIPCHK(launch_adj_seed<T>(ad, c->stream));
    HIPCHK(launch_fill<T>((T*)abar.p, (int64_t)(2 * nspec), (T)0, c->stream));

    // ---- reverse sweep, one checkpoint segment at a time
    HIPCHK(launch_fill<T>((T*)Gbar.p, (int64_t)(3 * H3), (T)0, c->stream));
    const PartDesc<T>* ps_dev = (const PartDesc<T>*)pdS.p;
    bool src_ready = false;  // phibar^(n-1) already made by the fused pass of step n + 1
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
        const int64_t base = sgi * K;
        const int len = (int)std::min<int64_t>(K, N - base);
        HIPCHK(launch_sort<T>(3, ps_dev + sgi, ps_dev + nseg, c->chunks, c->nchunks, 1, c->counts, c->cursor, c->seg,
                              c->seg_off, c->seg_n, c->items, c->nitems, c->adj_chunk, c->stream));
        if ((rc = grad_of_tape(base, len))) return rc;
        for (int m = 1; m < len; ++m) {
            // X^(base+m) = push of X^(base+m-1) (slot m-1 -> slot m) with G^(base+m-1)
            // (step base+m)
            HIPCHK(launch_particles<T>((const PartDesc<T>*)pdR.p + (base + m - 1), c->items, c->nitems, c->pgrid,
                                       false, true, c->scheme, c->win_bytes, c->pow2, c->sorted, c->stream));
        }
        {
            T *x, *y, *z;
            uint32_t* id;
            slot(seg.p, 0, x, y, z, id);
            HIPCHK(launch_xbar_order<T>((T*)xbar.p, ad.xbx, ad.xby, ad.xbz, id, P, true, c->stream));
        }
        for (int64_t n = base + len; n > base; --n) {
            // (a) phibar^(n-1) = L^-3 C2R(B abar^(n)); zero at n = N (abar^(N) = 0)
            const bool src = n < N;
            if (src && !src_ready) {
                HIPCHK(launch_xpencils<T>(H, (const FieldDesc<T>*)fdS.p, 1, XP_ADJ_SRC, c->stream));
                HIPCHK(launch_inv_planes<T>(H, (const FieldDesc<T>*)fdS.p, 1, 1, c->stream));
            }
            src_ready = false;
            // (b) particles of X^(n-1) with G^(n-1) (Gbar is zero: cleared once before the
            // sweep, then by the forward plane pass that consumes it)
            T *x, *y, *z;
            uint32_t* id;
            slot(seg.p, n - 1 - base, x, y, z, id);
            ad.x = x;
            ad.y = y;
            ad.z = z;
            ad.id = id;
            ad.G = gseg + (size_t)(n - 1 - base) * 3 * H3;
            ad.phibar = src ? (const T*)phibar.p : nullptr;
            ad.n = (uint32_t)n;
            // steps base+1 .. base+len-1 were pushed by the recompute, which kept their normals
            ad.zin = keep_noise && n < base + len ? (const T*)zseg.p + (size_t)(n - base - 1) * 6 * P : nullptr;
            HIPCHK(launch_adj_items<T>(ad, c->items, c->nitems, c->pgrid, c->stream));
            // (c) abar^(n-1) = A abar^(n) + sum_d (-i xi_d Phi) R2C(Gbar_d); for n > 1 the
            // same pass also makes the source term of abar^(n-1), i.e. phibar^(n-2) of step n - 1
            HIPCHK(launch_fwd_planes<T>(H, (const FieldDesc<T>*)fdA.p, 1, 3, true, c->stream));
            if (n > 1) {
                HIPCHK(launch_xpencils<T>(H, (const FieldDesc<T>*)fdA.p, 1, XP_ADJ_ACC_SRC, c->stream));
                HIPCHK(launch_inv_planes<T>(H, (const FieldDesc<T>*)fdS.p, 1, 1, c->stream));
                src_ready = true;
            } else {
                HIPCHK(launch_xpencils<T>(H, (const FieldDesc<T>*)fdA.p, 1, XP_ADJ_ACC, c->stream));
            }
        }
        {
            T *x, *y, *z;
            uint32_t* id;
            slot(seg.p, 0, x, y, z, id);
            HIPCHK(launch_xbar_order<T>((T*)xbar.p, ad.xbx, ad.xby, ad.xbz, id, P, false, c->stream));
        }
    }
    // ---- results and restoration of the context state (X^(N), alpha^(N), G^(N), n = N,
    // work items of the current positions)
    double hacc[4];
    HIPCHK(hipMemcpyAsync(hacc, acc.p, sizeof(hacc), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(dX0, xbar.p, (size_t)P * 3 * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(I.alpha, aN.p, nspec * sizeof(V), hipMemcpyDeviceToDevice, c->stream));
    if ((rc = recompute_grad<T>(c))) return rc;
    HIPCHK(launch_set_u32(c->steps, (uint32_t)N, c->stream));
    if ((rc = do_sort<T>(c))) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    const double tau = I.prm.dt, mu = I.prm.mu;
    const double dsdmu = c->scheme == SIPF_STRANG ? tau / (2.0 * std::sqrt(mu * tau)) : tau / std::sqrt(2.0 * mu * tau);
    *loss_out = hacc[2];
    *dchi_out = hacc[0];
    *dmu_out = mu > 0 ? hacc[1] * dsdmu : 0.0;
    return check_err(c);
}

// ---------------------------------------------------------------------------
// snapshots: header, positions in original order, alpha in natural order
// ---------------------------------------------------------------------------
const char kMagic[8] = {'S', 'I', 'P', 'F', 'S', 'N', 'A', 'P'};
constexpr uint32_t kVersion = 4;

struct SnapHeader {
    char magic[8];
    uint32_t version;
    uint32_t tsize;
    sipf_params prm;
    int64_t P;
    int64_t n;
};

int save_ctx(sipf_ctx* c, const char* path) {
    const Inst& I = c->in[0];
    const size_t nspec = spec_size(I.H, I.dim);
    SnapHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.tsize = (uint32_t)c->tsize;
    h.prm = I.prm;
    h.P = I.P;
    int rc;
    if ((rc = get_step_any(c, 0, &h.n))) return rc;
    std::vector<char> X((size_t)I.P * I.dim * c->tsize), A(2 * nspec * c->tsize);
    if ((rc = get_positions_any(c, 0, X.data(), 0))) return rc;
    if ((rc = get_field_any(c, 0, SIPF_FIELD_ALPHA, A.data(), 0))) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SIPF_EIO, std::string("cannot open ") + path + " for writing");
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(X.data(), 1, X.size(), f) == X.size() &&
              std::fwrite(A.data(), 1, A.size(), f) == A.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(SIPF_EIO, std::string("writing ") + path + " failed");
    return SIPF_OK;
}

int load_ctx(const char* path, void* hip_stream, sipf_ctx** out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SIPF_EIO, std::string("cannot open ") + path);
    SnapHeader h{};
    std::vector<char> X, A;
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && std::memcmp(h.magic, kMagic, 8) == 0 &&
              h.version == kVersion && (h.tsize == 4 || h.tsize == 8) &&
              h.tsize == (h.prm.precision == SIPF_FP32 ? 4u : 8u) && h.P >= 1 && h.P < (int64_t(1) << 32) &&
              h.n >= 0 && h.n < (int64_t(1) << 32);
    if (ok) ok = h.prm.dim == 0 || h.prm.dim == 2 || h.prm.dim == 3;
    if (ok) ok = dim_of(&h.prm) == 2 ? fft2d_size_supported(h.prm.H) : fft_size_supported(h.prm.H, h.prm.precision == SIPF_FP64);
    if (ok) {
        const int d = dim_of(&h.prm);
        const size_t nspec = spec_size(h.prm.H, d);
        X.resize((size_t)h.P * d * h.tsize);
        A.resize(2 * nspec * h.tsize);
        ok = std::fread(X.data(), 1, X.size(), f) == X.size() && std::fread(A.data(), 1, A.size(), f) == A.size();
        char extra;
        ok = ok && std::fread(&extra, 1, 1, f) == 0;
    }
    std::fclose(f);
    if (!ok) return fail(SIPF_EIO, std::string(path) + ": not a complete snapshot");
    sipf_ctx* c = nullptr;
    int rc = sipf_init(&h.prm, h.P, X.data(), 0, A.data(), 0, hip_stream, &c);
    if (rc) return rc;
    if (h.n > 0) {
        hipError_t e = launch_set_u32(c->steps, (uint32_t)h.n, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            sipf_destroy(c);
            return fail(SIPF_EDEVICE, std::string("restoring the step counter: ") + hipGetErrorString(e));
        }
    }
    *out = c;
    return SIPF_OK;
}

// ---------------------------------------------------------------------------
// autotuner: coordinate search over (tile, chunk, resort period)
// ---------------------------------------------------------------------------
// The deposit of Algorithm 2 (load, tile sort, deposit-only particle pass)
// on caller buffers, with every intermediate in the device's static scratch
// array (noalloc.hip) instead of allocated memory.
constexpr int64_t NOALLOC_MAX_P = int64_t(1) << 19;

template <typename T> int deposit_noalloc_typed(const sipf_params* p, int64_t P, const void* X, void* phi, hipStream_t s) {
    void* base = nullptr;
    size_t bytes = 0;
    HIPCHK(noalloc_scratch(&base, &bytes));
    const int H = p->H, tile = default_tile(p), chunk = default_chunk(p, P);
    const int mk = sort_max_keys(), sc = sort_chunk();
    const int nchunks = (int)((P + sc - 1) / sc);
    const int nt = (H + tile - 1) / tile;
    const int cap = (int)((P + chunk - 1) / chunk) + nt * nt * nt;
    size_t off = 0;
    auto take = [&](size_t n) {
        unsigned char* q = (unsigned char*)base + off;
        off += (n + 255) / 256 * 256;
        return q;
    };
    PartDesc<T> d[2];
    for (int set = 0; set < 2; ++set) {
        d[set] = pdesc_params<T>(*p, P, H, 3, tile);
        d[set].x = (T*)take(P * sizeof(T));
        d[set].y = (T*)take(P * sizeof(T));
        d[set].z = (T*)take(P * sizeof(T));
        d[set].id = (uint32_t*)take(P * sizeof(uint32_t));
        d[set].phi = (T*)phi;
    }
    uint32_t* counts = (uint32_t*)take(mk * sizeof(uint32_t));
    uint32_t* cursor = (uint32_t*)take(mk * sizeof(uint32_t));
    PartDesc<T>* pd = (PartDesc<T>*)take(2 * sizeof(PartDesc<T>));
    SortChunk* chunks = (SortChunk*)take(nchunks * sizeof(SortChunk));
    WorkItem* seg = (WorkItem*)take(cap * sizeof(WorkItem));
    int* seg_off = (int*)take(sizeof(int));
    int* seg_n = (int*)take(sizeof(int));
    WorkItem* items = (WorkItem*)take(cap * sizeof(WorkItem));
    int* nitems = (int*)take(16);
    int* err = (int*)take(sizeof(int));
    uint32_t* step = (uint32_t*)take(sizeof(uint32_t));
    if (off > bytes) return fail(SIPF_EINVAL, "the allocation-free scratch is too small for this call");
    for (int set = 0; set < 2; ++set) {
        d[set].step = step;
        d[set].err = err;
    }
    HIPCHK(launch_noalloc_setup<T>(d[0], d[1], pd, chunks, nchunks, sc, seg_off, counts, mk, nitems, err, step, s));
    HIPCHK(launch_fill<T>((T*)phi, (int64_t)H * H * H, (T)0, s));
    HIPCHK(launch_load_positions<T>((const T*)X, P, (T)p->L, d[0], err, s));
    HIPCHK(launch_sort<T>(3, pd, pd + 1, chunks, nchunks, 1, counts, cursor, seg, seg_off, seg_n, items, nitems, chunk, s));
    const int win = particle_window_bytes(sizeof(T) == 8);
    const int grid = std::max(1, std::min(cap, particle_resident_blocks<T>(p->scheme, win, false)));
    HIPCHK(launch_particles<T>(pd + 1, items, nitems, grid, true, false, p->scheme, win, is_pow2(H), false, s));
    return SIPF_OK;
}

int time_config(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device, int nsteps, void* hip_stream,
                double* ms) {
    sipf_ctx* c = nullptr;
    int rc = sipf_init(prm, P, X0, x0_on_device, nullptr, 0, hip_stream, &c);
    if (rc) return rc;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        // Timed window: whole multiples of two sort periods starting at a due
        // sort, so that every candidate period pays its sorts in proportion;
        // one untimed window first captures the graphs the timed one replays.
        const int64_t period = 2 * (int64_t)c->resort;
        const int64_t T = (nsteps + period - 1) / period * period;
        rc = run_group(c, c->resort);  // to the first due sort
        if (!rc) rc = run_group(c, T);
        if (!rc) e = hipEventRecord(a, c->stream);
        if (!rc && e == hipSuccess) rc = run_group(c, T);
        if (!rc && e == hipSuccess) e = hipEventRecord(b, c->stream);
        if (!rc && e == hipSuccess) e = hipEventSynchronize(b);
        float f = 0.f;
        if (!rc && e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
        *ms = f / (double)T;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (!rc) rc = check_err(c);
    std::string keep = g_err;
    sipf_destroy(c);
    g_err = keep;
    if (!rc && e != hipSuccess) return fail(SIPF_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sipf_last_error(void) { return g_err.c_str(); }

int sipf_params_default(sipf_params* p) {
    if (!p) return fail(SIPF_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->L = 2.0;
    p->chi = 1.0;
    p->mu = 1.0;
    p->eps = 1.0;
    p->k = 1.0;
    p->M0 = 1.0;
    p->dt = 1e-4;
    p->H0 = 0.0;
    p->H = 64;
    p->p2g_order = 4;
    p->g2p_order = 2;
    p->scheme = SIPF_STRANG;
    p->precision = SIPF_FP32;
    p->dim = 3;
    return SIPF_OK;
}

int sipf_init(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device, const void* alpha0,
              int alpha0_on_device, void* hip_stream, sipf_ctx** out) {
    if (!out) return fail(SIPF_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(prm, P);
    if (rc) return rc;
    if (!X0) return fail(SIPF_EINVAL, "X0 is NULL");
    sipf_ctx* c = new (std::nothrow) sipf_ctx();
    if (!c) return fail(SIPF_ENOMEM, "host allocation failed");
    const void* xs[1] = {X0};
    rc = setup_group(c, 1, prm, &P, xs, x0_on_device, hip_stream);
    if (!rc) rc = init_any(c, xs, x0_on_device, alpha0, alpha0_on_device);
    if (rc) {
        std::string keep = g_err;
        free_group(c);
        delete c;
        g_err = keep;
        return rc;
    }
    *out = c;
    return SIPF_OK;
}

int sipf_prepare_run(sipf_ctx* c, int64_t nsteps) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
    return prepare_group(c, nsteps);
}

int sipf_step(sipf_ctx* c) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return c->prec == SIPF_FP32 ? enqueue_step<float>(c) : enqueue_step<double>(c);
}

int sipf_run(sipf_ctx* c, int64_t nsteps) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
    return run_group(c, nsteps);
}

int sipf_use_graphs(sipf_ctx* c, int enable) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    c->graphs = enable != 0 && c->method != SIPF_METHOD_DIRECT && !c->positivity;
    return SIPF_OK;
}

int sipf_get_params(sipf_ctx* c, sipf_params* prm, int64_t* P) {
    if (!c || !prm || !P) return fail(SIPF_EINVAL, "NULL argument");
    *prm = c->in[0].prm;
    *P = c->in[0].P;
    return SIPF_OK;
}

int sipf_sync(sipf_ctx* c) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return check_err(c);
}

int sipf_get_step(sipf_ctx* c, int64_t* n) {
    if (!c || !n) return fail(SIPF_EINVAL, "NULL argument");
    return get_step_any(c, 0, n);
}

int sipf_diagnostics(sipf_ctx* c, sipf_diag* out) {
    if (!c || !out) return fail(SIPF_EINVAL, "NULL argument");
    if (c->method == SIPF_METHOD_DIRECT) return fail(SIPF_EINVAL, "a direct SIPF context has no grids");
    return diagnostics_any(c, out);
}

int sipf_get_positions(sipf_ctx* c, void* out, int on_device) {
    if (!c || !out) return fail(SIPF_EINVAL, "NULL argument");
    return get_positions_any(c, 0, out, on_device);
}

int sipf_get_field(sipf_ctx* c, int which, void* out, int on_device) {
    if (!c || !out) return fail(SIPF_EINVAL, "NULL argument");
    return get_field_any(c, 0, which, out, on_device);
}

int sipf_profile(sipf_ctx* c, int enable) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return profile_any(c, enable);
}

int sipf_profile_read(sipf_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(SIPF_EINVAL, "NULL argument");
    return profile_read_any(c, ms, launches);
}

int sipf_adjoint(sipf_ctx* c, int64_t nsteps, int32_t ckpt_every, const void* phi_bar, double* loss, double* dchi,
                 double* dmu, void* dX0) {
    if (!c || !loss || !dchi || !dmu || !dX0) return fail(SIPF_EINVAL, "NULL argument");
    if (nsteps < 1 || nsteps > (int64_t)1 << 30) return fail(SIPF_EINVAL, "nsteps must be >= 1");
    if (ckpt_every < 1) return fail(SIPF_EINVAL, "ckpt_every must be >= 1");
    if (c->dim != 3) return fail(SIPF_EINVAL, "sipf_adjoint is available in three dimensions only");
    if (c->method == SIPF_METHOD_DIRECT) return fail(SIPF_EINVAL, "sipf_adjoint runs SIPF-PIC contexts only");
    if (!c->pow2) return fail(SIPF_EINVAL, "sipf_adjoint needs H a power of two");
    for (const Inst& I : c->in)
        if (I.H > 128) return fail(SIPF_EINVAL, "sipf_adjoint takes H <= 128");
    if (c->positivity) return fail(SIPF_EINVAL, "sipf_adjoint does not differentiate the positivity rounds");
    return c->prec == SIPF_FP32
               ? adjoint_typed<float>(c, nsteps, ckpt_every, (const float*)phi_bar, loss, dchi, dmu, (float*)dX0)
               : adjoint_typed<double>(c, nsteps, ckpt_every, (const double*)phi_bar, loss, dchi, dmu, (double*)dX0);
}

int sipf_save(sipf_ctx* c, const char* path) {
    if (!c || !path) return fail(SIPF_EINVAL, "NULL argument");
    if (c->method == SIPF_METHOD_DIRECT)
        return fail(SIPF_EINVAL, "snapshots hold half spectra; a direct SIPF context keeps the full one");
    return save_ctx(c, path);
}

int sipf_load(const char* path, void* hip_stream, sipf_ctx** out) {
    if (!out || !path) return fail(SIPF_EINVAL, "NULL argument");
    *out = nullptr;
    return load_ctx(path, hip_stream, out);
}

int sipf_destroy(sipf_ctx* c) {
    if (!c) return SIPF_OK;
    destroy_any(c);
    delete c;
    return SIPF_OK;
}

int sipf_autotune(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device, int32_t nsteps,
                  void* hip_stream, sipf_params* best, double* ms_per_step) {
    if (!best || !ms_per_step) return fail(SIPF_EINVAL, "NULL argument");
    int rc = validate(prm, P);
    if (rc) return rc;
    if (!X0) return fail(SIPF_EINVAL, "X0 is NULL");
    if (nsteps < 1) return fail(SIPF_EINVAL, "nsteps must be >= 1");
    if (prm->method == SIPF_METHOD_DIRECT) return fail(SIPF_EINVAL, "the direct SIPF method has nothing to tune");
    sipf_params cur = *prm;
    cur.tile = default_tile(prm);
    cur.chunk = default_chunk(prm, P);
    cur.resort_every = default_resort(prm);
    double t_best = 0;
    if ((rc = time_config(&cur, P, X0, x0_on_device, nsteps, hip_stream, &t_best))) return rc;
    auto try_axis = [&](int32_t sipf_params::*field, const std::vector<int>& cands) -> int {
        for (int v : cands) {
            if (v == cur.*field) continue;
            sipf_params p = cur;
            p.*field = v;
            if (validate(&p, P) != SIPF_OK) continue;
            double t = 0;
            int r = time_config(&p, P, X0, x0_on_device, nsteps, hip_stream, &t);
            if (r) return r;
            if (t < t_best) {
                t_best = t;
                cur = p;
            }
        }
        return SIPF_OK;
    };
    std::vector<int> tiles;
    if (dim_of(prm) == 2) {
        for (int t = 8; t <= 128; t *= 2)
            if (t <= prm->H && prm->H / t <= 64) tiles.push_back(t);
    } else if (is_pow2(prm->H)) {
        for (int t = 4; t <= 32; t *= 2)
            if (t <= prm->H && prm->H / t <= 16) tiles.push_back(t);
    } else {
        for (int t : {4, 6, 8, 12, 16, 24, 32})
            if (t <= prm->H && (prm->H + t - 1) / t <= 16) tiles.push_back(t);
    }
    if ((rc = try_axis(&sipf_params::tile, tiles))) return rc;
    if ((rc = try_axis(&sipf_params::chunk, {1024, 2048, 3072, 4096}))) return rc;
    if ((rc = try_axis(&sipf_params::resort_every, {2, 4, 6, 8, 16}))) return rc;
    if (prm->precision == SIPF_FP32 && dim_of(prm) == 3) {
        cur.particle_pass = sorted_pass(&cur, 1) ? SIPF_PASS_SORTED : SIPF_PASS_TWO_PHASE;
        if ((rc = try_axis(&sipf_params::particle_pass, {SIPF_PASS_SORTED, SIPF_PASS_TWO_PHASE}))) return rc;
    }
    *best = cur;
    *ms_per_step = t_best;
    return SIPF_OK;
}

int sipf_batch_init(int32_t n, const sipf_params* prm, const int64_t* P, const void* const* X0, int x0_on_device,
                    void* hip_stream, sipf_batch** out) {
    if (!out) return fail(SIPF_EINVAL, "out is NULL");
    *out = nullptr;
    sipf_batch* b = new (std::nothrow) sipf_batch();
    if (!b) return fail(SIPF_ENOMEM, "host allocation failed");
    int rc = setup_group(b, n, prm, P, X0, x0_on_device, hip_stream);
    if (!rc) rc = init_any(b, X0, x0_on_device, nullptr, 0);
    if (rc) {
        std::string keep = g_err;
        free_group(b);
        delete b;
        g_err = keep;
        return rc;
    }
    *out = b;
    return SIPF_OK;
}

int sipf_batch_prepare_run(sipf_batch* b, int64_t nsteps) {
    if (!b) return fail(SIPF_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
    return prepare_group(b, nsteps);
}

int sipf_batch_run(sipf_batch* b, int64_t nsteps) {
    if (!b) return fail(SIPF_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
    return run_group(b, nsteps);
}

int sipf_batch_sync(sipf_batch* b) {
    if (!b) return fail(SIPF_EINVAL, "batch is NULL");
    return check_err(b);
}

int sipf_batch_get_step(sipf_batch* b, int32_t i, int64_t* n) {
    if (!b || !n) return fail(SIPF_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)b->in.size()) return fail(SIPF_EINVAL, "instance index out of range");
    return get_step_any(b, i, n);
}

int sipf_batch_diagnostics(sipf_batch* b, sipf_diag* out) {
    if (!b || !out) return fail(SIPF_EINVAL, "NULL argument");
    return diagnostics_any(b, out);
}

int sipf_batch_get_positions(sipf_batch* b, int32_t i, void* out, int on_device) {
    if (!b || !out) return fail(SIPF_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)b->in.size()) return fail(SIPF_EINVAL, "instance index out of range");
    return get_positions_any(b, i, out, on_device);
}

int sipf_batch_get_field(sipf_batch* b, int32_t i, int which, void* out, int on_device) {
    if (!b || !out) return fail(SIPF_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)b->in.size()) return fail(SIPF_EINVAL, "instance index out of range");
    return get_field_any(b, i, which, out, on_device);
}

int sipf_batch_profile(sipf_batch* b, int enable) {
    if (!b) return fail(SIPF_EINVAL, "batch is NULL");
    return profile_any(b, enable);
}

int sipf_batch_profile_read(sipf_batch* b, double* ms, int64_t* launches) {
    if (!b || !ms || !launches) return fail(SIPF_EINVAL, "NULL argument");
    return profile_read_any(b, ms, launches);
}

int sipf_positivity_stats(sipf_ctx* c, int64_t* switched, int32_t* rounds) {
    if (!c || !switched || !rounds) return fail(SIPF_EINVAL, "NULL argument");
    *switched = c->pos_switched;
    *rounds = c->pos_rounds;
    return SIPF_OK;
}

int sipf_batch_use_graphs(sipf_batch* b, int enable) {
    if (!b) return fail(SIPF_EINVAL, "batch is NULL");
    b->graphs = enable != 0 && !b->positivity;
    return SIPF_OK;
}

int sipf_batch_destroy(sipf_batch* b) {
    if (!b) return SIPF_OK;
    destroy_any(b);
    delete b;
    return SIPF_OK;
}

int sipf_dbg_philox(uint64_t seed, int64_t count, const uint32_t* ctr, uint32_t* raw, void* normals, int precision,
                    void* hip_stream) {
    if (count < 0 || (count > 0 && !ctr)) return fail(SIPF_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (precision == SIPF_FP32) HIPCHK(launch_philox_dbg<float>(seed, count, ctr, raw, (float*)normals, s));
    else if (precision == SIPF_FP64) HIPCHK(launch_philox_dbg<double>(seed, count, ctr, raw, (double*)normals, s));
    else return fail(SIPF_EINVAL, "bad precision");
    HIPCHK(hipStreamSynchronize(s));
    return SIPF_OK;
}

int sipf_dbg_cells(const sipf_params* prm, int64_t count, const void* X, int32_t* cells, void* hip_stream) {
    int rc = validate(prm, count > 0 ? count : 1);
    if (rc) return rc;
    if (dim_of(prm) != 3) return fail(SIPF_EINVAL, "test entry points are three-dimensional");
    if (count < 0 || (count > 0 && (!X || !cells))) return fail(SIPF_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (prm->precision == SIPF_FP32)
        HIPCHK(launch_cells<float>((const float*)X, count, prm->H, (float)(prm->H / prm->L), cells, s));
    else
        HIPCHK(launch_cells<double>((const double*)X, count, prm->H, (double)(prm->H / prm->L), cells, s));
    HIPCHK(hipStreamSynchronize(s));
    return SIPF_OK;
}

int sipf_release_cached_memory(void) {
    g_buf_cache.release();
    return SIPF_OK;
}

int sipf_deposit_noalloc(const sipf_params* prm, int64_t count, const void* X, void* phi, void* hip_stream) {
    if (!prm || !X || !phi) return fail(SIPF_EINVAL, "NULL argument");
    int rc = validate(prm, count);
    if (rc) return rc;
    if (dim_of(prm) != 3) return fail(SIPF_EINVAL, "the allocation-free deposit is three-dimensional");
    if (prm->method == SIPF_METHOD_DIRECT) return fail(SIPF_EINVAL, "the direct SIPF method has no grid deposit");
    if (prm->positivity) return fail(SIPF_EINVAL, "the allocation-free deposit has no positivity option");
    if (count < 1 || count > NOALLOC_MAX_P)
        return fail(SIPF_EINVAL, "count must be in [1, " + std::to_string(NOALLOC_MAX_P) +
                                     "] for the allocation-free deposit (its scratch is a fixed-size device array)");
    hipStream_t s = (hipStream_t)hip_stream;
    return prm->precision == SIPF_FP32 ? deposit_noalloc_typed<float>(prm, count, X, phi, s)
                                       : deposit_noalloc_typed<double>(prm, count, X, phi, s);
}

int sipf_dbg_deposit(const sipf_params* prm, int64_t count, const void* X, void* phi, void* hip_stream) {
    if (!phi) return fail(SIPF_EINVAL, "phi is NULL");
    if (prm && dim_of(prm) != 3) return fail(SIPF_EINVAL, "test entry points are three-dimensional");
    sipf_ctx* c = nullptr;
    int rc = sipf_init(prm, count, X, 1, nullptr, 0, hip_stream, &c);
    if (rc) return rc;
    rc = sipf_get_field(c, SIPF_FIELD_RHO, phi, 1);
    sipf_destroy(c);
    return rc;
}

}  // extern "C"
