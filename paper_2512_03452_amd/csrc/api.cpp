// Host runtime and C ABI of the SIPF-PIC step (declared in include/sipf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
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

int validate(const sipf_params* p, int64_t P) {
    if (!p) return fail(SIPF_EINVAL, "params is NULL");
    if (p->precision != SIPF_FP32 && p->precision != SIPF_FP64) return fail(SIPF_EINVAL, "precision must be SIPF_FP32 or SIPF_FP64");
    if (!fft_size_supported(p->H, p->precision == SIPF_FP64))
        return fail(SIPF_EINVAL, "H must be a power of two in [8, 128] (FP32) or [8, 64] (FP64)");
    auto fin = [](double v) { return std::isfinite(v); };
    if (!(fin(p->L) && p->L > 0)) return fail(SIPF_EINVAL, "L must be finite and > 0");
    if (!(fin(p->dt) && p->dt > 0)) return fail(SIPF_EINVAL, "dt must be finite and > 0");
    if (!(fin(p->eps) && p->eps > 0)) return fail(SIPF_EINVAL, "eps must be finite and > 0");
    if (!(fin(p->mu) && p->mu >= 0)) return fail(SIPF_EINVAL, "mu must be finite and >= 0");
    if (!(fin(p->chi) && p->chi >= 0)) return fail(SIPF_EINVAL, "chi must be finite and >= 0");
    if (!(fin(p->k) && p->k >= 0)) return fail(SIPF_EINVAL, "k must be finite and >= 0");
    if (!(fin(p->M0) && p->M0 >= 0)) return fail(SIPF_EINVAL, "M0 must be finite and >= 0");
    if (!fin(p->H0)) return fail(SIPF_EINVAL, "H0 must be finite");
    if (p->p2g_order != 4) return fail(SIPF_EINVAL, "p2g_order must be 4");
    if (p->g2p_order != 2) return fail(SIPF_EINVAL, "g2p_order must be 2");
    if (p->scheme != SIPF_STRANG && p->scheme != SIPF_EM) return fail(SIPF_EINVAL, "scheme must be SIPF_STRANG or SIPF_EM");
    if (p->tile != 0 && (!is_pow2(p->tile) || p->tile > p->H || (p->H / p->tile) > 16))
        return fail(SIPF_EINVAL, "tile must be 0 or a power of two with H/16 <= tile <= H");
    if (p->resort_every < 0) return fail(SIPF_EINVAL, "resort_every must be >= 0");
    if (p->chunk != 0 && (p->chunk < 256 || p->chunk > 4096)) return fail(SIPF_EINVAL, "chunk must be 0 or in [256, 4096]");
    if (p->reserved != 0) return fail(SIPF_EINVAL, "reserved must be 0");
    if (P < 1 || P >= (int64_t(1) << 32)) return fail(SIPF_EINVAL, "P must be in [1, 2^32)");
    return SIPF_OK;
}

double filter_h0(const sipf_params* p) {
    if (p->H0 == 0) return std::ceil(8.0 * std::pow((double)p->H, 8.0 / 13.0) * std::pow(p->L, 5.0 / 13.0));
    return p->H0;
}

// default tuning (overridden by explicit parameters)
void tuning(const sipf_params* p, int64_t P, int& tile, int& resort, int& chunk) {
    tile = p->tile ? p->tile : (p->H >= 128 ? 8 : (p->H >= 16 ? p->H / 8 : p->H));
    if (p->H / tile > 16) tile = p->H / 16;
    resort = p->resort_every ? p->resort_every : 4;
    chunk = p->chunk ? p->chunk : 4096;
    (void)P;
}

}  // namespace

struct sipf_ctx {
    sipf_params prm{};
    int64_t P = 0;
    int H = 0;
    int prec = SIPF_FP32;
    size_t tsize = 4;
    hipStream_t stream = nullptr;
    int tile = 8, resort = 4, chunk = 4096, win_bytes = 65536, pgrid = 1024;
    int since_sort = 0;
    int cur = 0;  // which of the two particle buffer sets holds the current positions
    int64_t n_host = 0;
    void* xs[2] = {nullptr, nullptr};
    void* ys[2] = {nullptr, nullptr};
    void* zs[2] = {nullptr, nullptr};
    uint32_t* ids[2] = {nullptr, nullptr};
    void* phi = nullptr;
    void* B1 = nullptr;
    void* alpha = nullptr;
    void* gspec = nullptr;
    void* G = nullptr;
    uint32_t* counts = nullptr;
    uint32_t* cursor = nullptr;
    uint32_t* step = nullptr;
    int* err = nullptr;
    void* pdesc = nullptr;  // two PartDesc<T> (one per buffer set)
    void* fdesc = nullptr;  // one FieldDesc<T>
    WorkItem* items = nullptr;  // work items of the particle pass, rebuilt by every sort
    int* nitems = nullptr;      // device count of items
    int items_cap = 0;
    std::vector<void*> allocs;
    // captured graph of a whole number of sort periods
    hipGraphExec_t gexec = nullptr;
    int64_t graph_steps = 0;
    // per-phase event timing (sipf_profile)
    bool prof = false;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    double prof_ms[SIPF_NPHASES] = {0};
    int64_t prof_n[SIPF_NPHASES] = {0};
};

namespace {

int dalloc(sipf_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SIPF_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    return SIPF_OK;
}

template <typename T> PartDesc<T> make_pdesc(const sipf_ctx* c, int set) {
    PartDesc<T> d{};
    d.x = (T*)c->xs[set];
    d.y = (T*)c->ys[set];
    d.z = (T*)c->zs[set];
    d.id = c->ids[set];
    d.P = c->P;
    d.phi = (T*)c->phi;
    d.G = (const T*)c->G;
    d.step = c->step;
    d.err = c->err;
    d.H = c->H;
    d.scheme = c->prm.scheme;
    d.hl = (T)(c->H / c->prm.L);
    d.L = (T)c->prm.L;
    d.halfL = (T)(c->prm.L / 2);
    d.invL = (T)(1.0 / c->prm.L);
    d.wmass = (T)(c->prm.M0 / (double)c->P);
    d.chitau = (T)(c->prm.chi * c->prm.dt);
    d.s = (T)(c->prm.scheme == SIPF_STRANG ? std::sqrt(c->prm.mu * c->prm.dt) : std::sqrt(2.0 * c->prm.mu * c->prm.dt));
    d.k0 = (uint32_t)c->prm.seed;
    d.k1 = (uint32_t)(c->prm.seed >> 32);
    d.inst = c->prm.instance;
    // |W^-| <= s max|z| with max|z| = sqrt(-2 ln 2^-24) (uniforms are >= 2^-24)
    d.gmargin = c->prm.scheme == SIPF_STRANG ? (int)std::ceil((double)d.s * 5.7677 * (double)d.hl) : 0;
    return d;
}

template <typename T> FieldDesc<T> make_fdesc(const sipf_ctx* c) {
    FieldDesc<T> f{};
    const sipf_params& p = c->prm;
    f.phi = (T*)c->phi;
    f.B1 = (cplx_t<T>*)c->B1;
    f.alpha = (cplx_t<T>*)c->alpha;
    f.gspec = (cplx_t<T>*)c->gspec;
    f.G = (T*)c->G;
    f.step = c->step;
    f.dt_over_eps = (T)(p.dt / p.eps);
    f.eps_over_dt = (T)(p.eps / p.dt);
    f.k2 = (T)(p.k * p.k);
    f.inv_L3 = (T)(1.0 / (p.L * p.L * p.L));
    f.two_pi_over_L = (T)(2.0 * M_PI / p.L);
    const double h0 = filter_h0(&p);
    f.filt = p.H0 < 0 ? (T)0 : (T)(2.0 * M_PI * M_PI / (h0 * h0));
    return f;
}

template <typename T> int upload_descs(sipf_ctx* c) {
    PartDesc<T> pd[2] = {make_pdesc<T>(c, 0), make_pdesc<T>(c, 1)};
    FieldDesc<T> fd = make_fdesc<T>(c);
    HIPCHK(hipMemcpy(c->pdesc, pd, sizeof(pd), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->fdesc, &fd, sizeof(fd), hipMemcpyHostToDevice));
    return SIPF_OK;
}

template <typename T> const PartDesc<T>* pdesc_dev(const sipf_ctx* c, int set) {
    return reinterpret_cast<const PartDesc<T>*>(c->pdesc) + set;
}

// Event bracket around one launch when timing is on.
struct Timed {
    sipf_ctx* c;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(sipf_ctx* ctx, int ph) : c(ctx), phase(ph) {
        if (!c->prof) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            c->prof = false;
            return;
        }
        (void)hipEventRecord(a, c->stream);
    }
    ~Timed() {
        if (!c->prof || !a) return;
        (void)hipEventRecord(b, c->stream);
        c->marks.push_back({phase, a, b});
    }
};

template <typename T> int do_sort(sipf_ctx* c) {
    const PartDesc<T> src = make_pdesc<T>(c, c->cur);
    const int dst = 1 - c->cur;
    {
        Timed t(c, SIPF_PHASE_SORT);
        HIPCHK(launch_sort<T>(&src, reinterpret_cast<PartDesc<T>*>(c->pdesc) + c->cur, (T*)c->xs[dst],
                              (T*)c->ys[dst], (T*)c->zs[dst], c->ids[dst], c->counts, c->cursor, c->tile, c->chunk,
                              c->items, c->nitems, 0, c->stream));
    }
    c->cur = dst;
    c->since_sort = 0;
    return SIPF_OK;
}

// One step n-1 -> n: particle pass (deposit X^(n-1), gather grad c^(n-1), push),
// then the field passes that turn the deposit into alpha^(n) and grad c^(n).
template <typename T> int enqueue_step(sipf_ctx* c) {
    if (c->since_sort >= c->resort) {
        int rc = do_sort<T>(c);
        if (rc) return rc;
    }
    {
        Timed t(c, SIPF_PHASE_PARTICLES);
        HIPCHK(launch_particles<T>(pdesc_dev<T>(c, c->cur), c->items, c->nitems, c->pgrid, true, true,
                                   c->prm.scheme, c->win_bytes, c->stream));
    }
    const FieldDesc<T>* fd = reinterpret_cast<const FieldDesc<T>*>(c->fdesc);
    {
        Timed t(c, SIPF_PHASE_FWD);
        HIPCHK(launch_fwd_planes<T>(c->H, fd, 1, 1, true, c->stream));
    }
    {
        Timed t(c, SIPF_PHASE_XPENCIL);
        HIPCHK(launch_xpencils<T>(c->H, fd, 1, XP_STEP, c->stream));
    }
    {
        Timed t(c, SIPF_PHASE_INV);
        HIPCHK(launch_inv_planes<T>(c->H, fd, 1, 3, c->stream));
    }
    c->since_sort++;
    c->n_host++;
    return SIPF_OK;
}

int drain_marks(sipf_ctx* c) {
    if (c->marks.empty()) return SIPF_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    for (auto& m : c->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            c->prof_ms[m.phase] += ms;
            c->prof_n[m.phase] += 1;
        }
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    c->marks.clear();
    return SIPF_OK;
}

int step_dispatch(sipf_ctx* c) { return c->prec == SIPF_FP32 ? enqueue_step<float>(c) : enqueue_step<double>(c); }

int check_err(sipf_ctx* c) {
    int e = 0;
    HIPCHK(hipMemcpyAsync(&e, c->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (e & 2) return fail(SIPF_ENUMERIC, "non-finite initial position");
    if (e & 1) return fail(SIPF_ENUMERIC, "a step produced a non-finite position");
    return SIPF_OK;
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

template <typename T> int init_fields(sipf_ctx* c, const void* alpha0, int alpha0_on_device) {
    const int H = c->H;
    const size_t HH = H / 2 + 1;
    const size_t nspec = (size_t)H * H * HH;
    const size_t H3 = (size_t)H * H * H;
    HIPCHK(launch_fill<T>((T*)c->phi, H3, (T)0, c->stream));
    HIPCHK(launch_fill<T>((T*)c->G, 3 * H3, (T)0, c->stream));
    if (alpha0 == nullptr) {
        HIPCHK(launch_fill<T>((T*)c->alpha, 2 * nspec, (T)0, c->stream));
        return SIPF_OK;
    }
    std::vector<T> nat(2 * nspec), per(2 * nspec);
    if (alpha0_on_device) HIPCHK(hipMemcpy(nat.data(), alpha0, nat.size() * sizeof(T), hipMemcpyDeviceToHost));
    else std::memcpy(nat.data(), alpha0, nat.size() * sizeof(T));
    for (T v : nat)
        if (!std::isfinite((double)v)) return fail(SIPF_ENUMERIC, "non-finite alpha0");
    permute_spectrum(nat.data(), per.data(), H, sizeof(T), true);
    HIPCHK(hipMemcpy(c->alpha, per.data(), per.size() * sizeof(T), hipMemcpyHostToDevice));
    const FieldDesc<T>* fd = reinterpret_cast<const FieldDesc<T>*>(c->fdesc);
    HIPCHK(launch_xpencils<T>(H, fd, 1, XP_GRAD, c->stream));
    HIPCHK(launch_inv_planes<T>(H, fd, 1, 3, c->stream));
    return SIPF_OK;
}

template <typename T>
int init_typed(sipf_ctx* c, const void* X0, int x0_on_device, const void* alpha0, int alpha0_on_device) {
    const int64_t P = c->P;
    const int H = c->H;
    const size_t H3 = (size_t)H * H * H;
    const size_t nspec = (size_t)H * H * (H / 2 + 1);
    int rc;
    for (int s = 0; s < 2; ++s) {
        if ((rc = dalloc(c, &c->xs[s], P * sizeof(T)))) return rc;
        if ((rc = dalloc(c, &c->ys[s], P * sizeof(T)))) return rc;
        if ((rc = dalloc(c, &c->zs[s], P * sizeof(T)))) return rc;
        if ((rc = dalloc(c, (void**)&c->ids[s], P * sizeof(uint32_t)))) return rc;
    }
    if ((rc = dalloc(c, &c->phi, H3 * sizeof(T)))) return rc;
    if ((rc = dalloc(c, &c->B1, nspec * 2 * sizeof(T)))) return rc;
    if ((rc = dalloc(c, &c->alpha, nspec * 2 * sizeof(T)))) return rc;
    if ((rc = dalloc(c, &c->gspec, 3 * nspec * 2 * sizeof(T)))) return rc;
    if ((rc = dalloc(c, &c->G, 3 * H3 * sizeof(T)))) return rc;
    if ((rc = dalloc(c, (void**)&c->counts, sort_max_keys() * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(c, (void**)&c->cursor, sort_max_keys() * sizeof(uint32_t)))) return rc;
    if ((rc = dalloc(c, (void**)&c->step, 16))) return rc;
    if ((rc = dalloc(c, (void**)&c->err, 16))) return rc;
    if ((rc = dalloc(c, &c->pdesc, 2 * sizeof(PartDesc<T>)))) return rc;
    if ((rc = dalloc(c, &c->fdesc, sizeof(FieldDesc<T>)))) return rc;
    c->items_cap = (int)((P + particle_chunk() - 1) / particle_chunk()) + sort_max_keys();
    if ((rc = dalloc(c, (void**)&c->items, c->items_cap * sizeof(WorkItem)))) return rc;
    if ((rc = dalloc(c, (void**)&c->nitems, 16))) return rc;
    HIPCHK(hipMemset(c->nitems, 0, 16));
    c->pgrid = std::min(c->items_cap, 1024);
    HIPCHK(hipMemset(c->counts, 0, sort_max_keys() * sizeof(uint32_t)));
    HIPCHK(hipMemset(c->step, 0, 16));
    HIPCHK(hipMemset(c->err, 0, 16));
    if ((rc = upload_descs<T>(c))) return rc;
    // positions: AoS (host or device) -> SoA set 0, wrapped, ids 0..P-1
    const T* xyz = (const T*)X0;
    if (!x0_on_device) {
        // host positions go through a temporary device buffer freed before return
        void* tmp = nullptr;
        if (hipMalloc(&tmp, 3 * P * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SIPF_ENOMEM, "hipMalloc failed for the staging buffer");
        }
        hipError_t e = hipMemcpy(tmp, X0, 3 * P * sizeof(T), hipMemcpyHostToDevice);
        PartDesc<T> d0 = make_pdesc<T>(c, 0);
        if (e == hipSuccess) e = launch_load_positions<T>((const T*)tmp, P, (T)c->prm.L, d0, c->err, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(SIPF_EDEVICE, std::string("loading X0: ") + hipGetErrorString(e));
    } else {
        PartDesc<T> d0 = make_pdesc<T>(c, 0);
        HIPCHK(launch_load_positions<T>(xyz, P, (T)c->prm.L, d0, c->err, c->stream));
    }
    if ((rc = init_fields<T>(c, alpha0, alpha0_on_device))) return rc;
    c->cur = 0;
    if ((rc = do_sort<T>(c))) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    return check_err(c);
}

void free_ctx(sipf_ctx* c) {
    if (!c) return;
    for (auto& m : c->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

template <typename T> int get_field_typed(sipf_ctx* c, int which, void* out, int on_device) {
    const int H = c->H;
    const size_t H3 = (size_t)H * H * H;
    const size_t nspec = (size_t)H * H * (H / 2 + 1);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (which == SIPF_FIELD_RHO) {
        HIPCHK(launch_particles<T>(pdesc_dev<T>(c, c->cur), c->items, c->nitems, c->pgrid, true, false,
                                   c->prm.scheme, c->win_bytes, c->stream));
        HIPCHK(hipMemcpyAsync(out, c->phi, H3 * sizeof(T), kind, c->stream));
        HIPCHK(launch_fill<T>((T*)c->phi, H3, (T)0, c->stream));
    } else if (which == SIPF_FIELD_GRAD) {
        HIPCHK(hipMemcpyAsync(out, c->G, 3 * H3 * sizeof(T), kind, c->stream));
    } else if (which == SIPF_FIELD_ALPHA) {
        std::vector<T> per(2 * nspec), nat(2 * nspec);
        HIPCHK(hipMemcpyAsync(per.data(), c->alpha, per.size() * sizeof(T), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        permute_spectrum(per.data(), nat.data(), H, sizeof(T), false);
        if (on_device) HIPCHK(hipMemcpy(out, nat.data(), nat.size() * sizeof(T), hipMemcpyHostToDevice));
        else std::memcpy(out, nat.data(), nat.size() * sizeof(T));
    } else {
        return fail(SIPF_EINVAL, "unknown field");
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return check_err(c);
}

template <typename T> int get_positions_typed(sipf_ctx* c, void* out, int on_device) {
    const PartDesc<T> d = make_pdesc<T>(c, c->cur);
    if (on_device) {
        HIPCHK(launch_unsort<T>(&d, (T*)out, c->stream));
    } else {
        void* tmp = nullptr;
        HIPCHK(hipMalloc(&tmp, 3 * c->P * sizeof(T)));
        hipError_t e = launch_unsort<T>(&d, (T*)tmp, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, 3 * c->P * sizeof(T), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(SIPF_EDEVICE, std::string("get_positions: ") + hipGetErrorString(e));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return check_err(c);
}

// Device buffer freed when it goes out of scope (adjoint temporaries).
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc(&p, n ? n : 16); }
};

template <typename T> PartDesc<T> pdesc_on(const sipf_ctx* c, T* x, T* y, T* z, uint32_t* id) {
    PartDesc<T> d = make_pdesc<T>(c, 0);
    d.x = x;
    d.y = y;
    d.z = z;
    d.id = id;
    return d;
}

// Gradient grids of alpha (the context's alpha buffer) into the context's G.
template <typename T> int recompute_grad(sipf_ctx* c) {
    const FieldDesc<T>* fd = reinterpret_cast<const FieldDesc<T>*>(c->fdesc);
    HIPCHK(launch_xpencils<T>(c->H, fd, 1, XP_GRAD, c->stream));
    HIPCHK(launch_inv_planes<T>(c->H, fd, 1, 3, c->stream));
    return SIPF_OK;
}

template <typename T>
int adjoint_typed(sipf_ctx* c, int64_t N, int K, const T* phibar_in, double* loss_out, double* dchi_out,
                  double* dmu_out, T* dX0) {
    using V = cplx_t<T>;
    int64_t n0 = 0;
    {
        uint32_t s = 0;
        HIPCHK(hipMemcpyAsync(&s, c->step, sizeof(s), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        n0 = s;
    }
    if (n0 != 0 || c->n_host != 0) return fail(SIPF_ESTATE, "sipf_adjoint needs a context at step 0");
    if (K > N) K = (int)N;
    const int H = c->H;
    const int64_t P = c->P;
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
    DevBuf tape, ckpt, seg, xbar, Gbar, phibar, abar, aN, scr, gs1, fdS, fdA, acc, pds, items, nit;
    int rc;
    if ((rc = need(tape, (size_t)N * nspec * sizeof(V)))) return rc;
    if ((rc = need(ckpt, (size_t)nseg * pos_bytes))) return rc;
    if ((rc = need(seg, (size_t)K * pos_bytes))) return rc;
    if ((rc = need(xbar, (size_t)P * 3 * sizeof(T)))) return rc;
    if ((rc = need(Gbar, 3 * H3 * sizeof(T)))) return rc;
    if ((rc = need(phibar, H3 * sizeof(T)))) return rc;
    if ((rc = need(abar, nspec * sizeof(V)))) return rc;
    if ((rc = need(aN, nspec * sizeof(V)))) return rc;
    if ((rc = need(scr, 3 * nspec * sizeof(V)))) return rc;
    if ((rc = need(gs1, nspec * sizeof(V)))) return rc;
    if ((rc = need(fdS, sizeof(FieldDesc<T>)))) return rc;
    if ((rc = need(fdA, sizeof(FieldDesc<T>)))) return rc;
    if ((rc = need(acc, 4 * sizeof(double)))) return rc;
    if ((rc = need(pds, (size_t)K * sizeof(PartDesc<T>)))) return rc;
    const int nu = (int)((P + particle_chunk() - 1) / particle_chunk());
    if ((rc = need(items, (size_t)nu * sizeof(WorkItem)))) return rc;
    if ((rc = need(nit, 16))) return rc;
    // position slot j of a buffer: x, y, z, id
    auto slot = [&](void* base, int64_t j, T*& x, T*& y, T*& z, uint32_t*& id) {
        char* b = (char*)base + (size_t)j * pos_bytes;
        x = (T*)b;
        y = x + P;
        z = y + P;
        id = (uint32_t*)(z + P);
    };
    {
        // adjoint field descriptors: source (abar -> phibar) and accumulation (Gbar -> abar)
        FieldDesc<T> f = make_fdesc<T>(c);
        f.alpha = (V*)abar.p;
        f.gspec = (V*)gs1.p;
        f.G = (T*)phibar.p;
        f.step = nullptr;
        HIPCHK(hipMemcpy(fdS.p, &f, sizeof(f), hipMemcpyHostToDevice));
        f = make_fdesc<T>(c);
        f.phi = (T*)Gbar.p;
        f.B1 = (V*)scr.p;
        f.alpha = (V*)abar.p;
        f.step = nullptr;
        HIPCHK(hipMemcpy(fdA.p, &f, sizeof(f), hipMemcpyHostToDevice));
        std::vector<PartDesc<T>> pd(K);
        for (int j = 0; j < K; ++j) {
            T *x, *y, *z;
            uint32_t* id;
            slot(seg.p, j, x, y, z, id);
            pd[j] = pdesc_on<T>(c, x, y, z, id);
        }
        HIPCHK(hipMemcpy(pds.p, pd.data(), pd.size() * sizeof(PartDesc<T>), hipMemcpyHostToDevice));
        std::vector<WorkItem> it(nu);
        for (int i = 0; i < nu; ++i) {
            it[i].beg = (int64_t)i * particle_chunk();
            it[i].cnt = (int32_t)std::min<int64_t>(particle_chunk(), P - it[i].beg);
            it[i].inst = 0;
        }
        HIPCHK(hipMemcpy(items.p, it.data(), it.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(nit.p, &nu, sizeof(int), hipMemcpyHostToDevice));
    }
    const FieldDesc<T>* fdc = reinterpret_cast<const FieldDesc<T>*>(c->fdesc);
    auto copy_positions = [&](T* x, T* y, T* z, uint32_t* id, const T* sx, const T* sy, const T* sz,
                              const uint32_t* sid) -> int {
        HIPCHK(hipMemcpyAsync(x, sx, P * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(y, sy, P * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(z, sz, P * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(id, sid, P * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream));
        return SIPF_OK;
    };

    // ---- forward with tape: alpha^(n-1) every step, X^(n-1) every K steps
    for (int64_t n = 1; n <= N; ++n) {
        if ((n - 1) % K == 0) {
            T *x, *y, *z;
            uint32_t* id;
            slot(ckpt.p, (n - 1) / K, x, y, z, id);
            if ((rc = copy_positions(x, y, z, id, (const T*)c->xs[c->cur], (const T*)c->ys[c->cur],
                                     (const T*)c->zs[c->cur], c->ids[c->cur])))
                return rc;
        }
        HIPCHK(hipMemcpyAsync((V*)tape.p + (size_t)(n - 1) * nspec, c->alpha, nspec * sizeof(V),
                              hipMemcpyDeviceToDevice, c->stream));
        if ((rc = enqueue_step<T>(c))) return rc;
    }
    HIPCHK(hipMemcpyAsync(aN.p, c->alpha, nspec * sizeof(V), hipMemcpyDeviceToDevice, c->stream));

    // ---- loss and its cotangent phibar^(N)
    HIPCHK(launch_zero_f64((double*)acc.p, 4, c->stream));
    HIPCHK(launch_particles<T>(pdesc_dev<T>(c, c->cur), c->items, c->nitems, c->pgrid, true, false, c->prm.scheme,
                               c->win_bytes, c->stream));
    if (phibar_in) {
        HIPCHK(launch_dot<T>(phibar_in, (const T*)c->phi, (int64_t)H3, (double*)acc.p + 2, c->stream));
        HIPCHK(hipMemcpyAsync(phibar.p, phibar_in, H3 * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    } else {
        HIPCHK(launch_dot<T>((const T*)c->phi, (const T*)c->phi, (int64_t)H3, (double*)acc.p + 2, c->stream));
        HIPCHK(launch_fill<T>((T*)phibar.p, (int64_t)H3, (T)0, c->stream));
        HIPCHK(launch_axpby<T>((T*)phibar.p, (const T*)c->phi, (T)2, (T)0, (int64_t)H3, c->stream));
    }
    HIPCHK(launch_fill<T>((T*)c->phi, (int64_t)H3, (T)0, c->stream));

    AdjDesc<T> ad{};
    ad.P = P;
    ad.H = H;
    ad.scheme = c->prm.scheme;
    const PartDesc<T> ref = make_pdesc<T>(c, c->cur);
    ad.hl = ref.hl;
    ad.wmass = ref.wmass;
    ad.chitau = ref.chitau;
    ad.tau = (T)c->prm.dt;
    ad.s = ref.s;
    ad.k0 = ref.k0;
    ad.k1 = ref.k1;
    ad.inst = ref.inst;
    ad.xbar = (T*)xbar.p;
    ad.Gbar = (T*)Gbar.p;
    ad.acc = (double*)acc.p;
    ad.G = (const T*)c->G;
    // seed: Xbar^(N) from phibar^(N) at X^(N)
    ad.x = (const T*)c->xs[c->cur];
    ad.y = (const T*)c->ys[c->cur];
    ad.z = (const T*)c->zs[c->cur];
    ad.id = c->ids[c->cur];
    ad.phibar = (const T*)phibar.p;
    HIPCHK(launch_adj_seed<T>(ad, c->stream));
    HIPCHK(launch_fill<T>((T*)abar.p, (int64_t)(2 * nspec), (T)0, c->stream));

    // ---- reverse sweep, one checkpoint segment at a time
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
        const int64_t base = sgi * K;
        const int len = (int)std::min<int64_t>(K, N - base);
        {
            T *x, *y, *z, *cx, *cy, *cz;
            uint32_t *id, *cid;
            slot(seg.p, 0, x, y, z, id);
            slot(ckpt.p, sgi, cx, cy, cz, cid);
            if ((rc = copy_positions(x, y, z, id, cx, cy, cz, cid))) return rc;
        }
        for (int m = 1; m < len; ++m) {
            // X^(base+m) = push of X^(base+m-1) with the gradient of alpha^(base+m-1), step base+m
            HIPCHK(hipMemcpyAsync(c->alpha, (V*)tape.p + (size_t)(base + m - 1) * nspec, nspec * sizeof(V),
                                  hipMemcpyDeviceToDevice, c->stream));
            if ((rc = recompute_grad<T>(c))) return rc;
            T *x, *y, *z, *px, *py, *pz;
            uint32_t *id, *pid;
            slot(seg.p, m, x, y, z, id);
            slot(seg.p, m - 1, px, py, pz, pid);
            if ((rc = copy_positions(x, y, z, id, px, py, pz, pid))) return rc;
            HIPCHK(launch_set_u32(c->step, (uint32_t)(base + m - 1), c->stream));
            HIPCHK(launch_particles<T>(reinterpret_cast<const PartDesc<T>*>(pds.p) + m, (const WorkItem*)items.p,
                                       (const int*)nit.p, std::min(nu, 1024), false, true, c->prm.scheme,
                                       c->win_bytes, c->stream));
        }
        for (int64_t n = base + len; n > base; --n) {
            // (a) phibar^(n-1) = L^-3 C2R(B abar^(n)); zero at n = N (abar^(N) = 0)
            const bool src = n < N;
            if (src) {
                HIPCHK(launch_xpencils<T>(H, (const FieldDesc<T>*)fdS.p, 1, XP_ADJ_SRC, c->stream));
                HIPCHK(launch_inv_planes<T>(H, (const FieldDesc<T>*)fdS.p, 1, 1, c->stream));
            }
            // (b) G^(n-1)
            HIPCHK(hipMemcpyAsync(c->alpha, (V*)tape.p + (size_t)(n - 1) * nspec, nspec * sizeof(V),
                                  hipMemcpyDeviceToDevice, c->stream));
            if ((rc = recompute_grad<T>(c))) return rc;
            // (c) particles of X^(n-1)
            HIPCHK(launch_fill<T>((T*)Gbar.p, (int64_t)(3 * H3), (T)0, c->stream));
            T *x, *y, *z;
            uint32_t* id;
            slot(seg.p, n - 1 - base, x, y, z, id);
            ad.x = x;
            ad.y = y;
            ad.z = z;
            ad.id = id;
            ad.phibar = src ? (const T*)phibar.p : nullptr;
            ad.n = (uint32_t)n;
            HIPCHK(launch_adj_step<T>(ad, c->stream));
            // (d) abar^(n-1) = A abar^(n) + sum_d (-i xi_d Phi) R2C(Gbar_d)
            HIPCHK(launch_fwd_planes<T>(H, (const FieldDesc<T>*)fdA.p, 1, 3, false, c->stream));
            HIPCHK(launch_xpencils<T>(H, (const FieldDesc<T>*)fdA.p, 1, XP_ADJ_ACC, c->stream));
        }
    }
    // ---- results and restoration of the context state (X^(N), alpha^(N), G^(N), n = N)
    double hacc[4];
    HIPCHK(hipMemcpyAsync(hacc, acc.p, sizeof(hacc), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(dX0, xbar.p, (size_t)P * 3 * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->alpha, aN.p, nspec * sizeof(V), hipMemcpyDeviceToDevice, c->stream));
    if ((rc = recompute_grad<T>(c))) return rc;
    HIPCHK(launch_set_u32(c->step, (uint32_t)N, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    (void)fdc;
    const double tau = c->prm.dt, mu = c->prm.mu;
    const double dsdmu = c->prm.scheme == SIPF_STRANG ? tau / (2.0 * std::sqrt(mu * tau)) : tau / std::sqrt(2.0 * mu * tau);
    *loss_out = hacc[2];
    *dchi_out = hacc[0];
    *dmu_out = mu > 0 ? hacc[1] * dsdmu : 0.0;
    return check_err(c);
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
    return SIPF_OK;
}

int sipf_init(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device, const void* alpha0,
              int alpha0_on_device, void* hip_stream, sipf_ctx** out) {
    if (!out) return fail(SIPF_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(prm, P);
    if (rc) return rc;
    if (!X0) return fail(SIPF_EINVAL, "X0 is NULL");
    const size_t ts = prm->precision == SIPF_FP32 ? 4 : 8;
    if (!x0_on_device) {
        // reject non-finite host input before touching the device
        for (int64_t i = 0; i < 3 * P; ++i) {
            const double v = ts == 4 ? (double)((const float*)X0)[i] : ((const double*)X0)[i];
            if (!std::isfinite(v)) return fail(SIPF_ENUMERIC, "non-finite value in X0");
        }
    }
    sipf_ctx* c = new (std::nothrow) sipf_ctx();
    if (!c) return fail(SIPF_ENOMEM, "host allocation failed");
    c->prm = *prm;
    c->P = P;
    c->H = prm->H;
    c->prec = prm->precision;
    c->tsize = ts;
    c->stream = (hipStream_t)hip_stream;
    tuning(prm, P, c->tile, c->resort, c->chunk);
    // LDS per particle-pass workgroup: the larger of the two fast windows
    c->win_bytes = particle_window_bytes(c->prec == SIPF_FP64);
    rc = c->prec == SIPF_FP32 ? init_typed<float>(c, X0, x0_on_device, alpha0, alpha0_on_device)
                              : init_typed<double>(c, X0, x0_on_device, alpha0, alpha0_on_device);
    if (rc) {
        std::string keep = g_err;
        free_ctx(c);
        g_err = keep;
        return rc;
    }
    *out = c;
    return SIPF_OK;
}

int sipf_step(sipf_ctx* c) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return step_dispatch(c);
}

int sipf_run(sipf_ctx* c, int64_t nsteps) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(SIPF_EINVAL, "nsteps must be >= 0");
    for (int64_t i = 0; i < nsteps; ++i) {
        int rc = step_dispatch(c);
        if (rc) return rc;
    }
    return SIPF_OK;
}

int sipf_sync(sipf_ctx* c) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return check_err(c);
}

int sipf_get_step(sipf_ctx* c, int64_t* n) {
    if (!c || !n) return fail(SIPF_EINVAL, "NULL argument");
    uint32_t s = 0;
    HIPCHK(hipMemcpyAsync(&s, c->step, sizeof(s), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *n = s;
    return SIPF_OK;
}

int sipf_get_positions(sipf_ctx* c, void* out, int on_device) {
    if (!c || !out) return fail(SIPF_EINVAL, "NULL argument");
    return c->prec == SIPF_FP32 ? get_positions_typed<float>(c, out, on_device)
                                : get_positions_typed<double>(c, out, on_device);
}

int sipf_get_field(sipf_ctx* c, int which, void* out, int on_device) {
    if (!c || !out) return fail(SIPF_EINVAL, "NULL argument");
    return c->prec == SIPF_FP32 ? get_field_typed<float>(c, which, out, on_device)
                                : get_field_typed<double>(c, which, out, on_device);
}

int sipf_profile(sipf_ctx* c, int enable) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    int rc = drain_marks(c);
    if (rc) return rc;
    for (int i = 0; i < SIPF_NPHASES; ++i) {
        c->prof_ms[i] = 0;
        c->prof_n[i] = 0;
    }
    c->prof = enable != 0;
    return SIPF_OK;
}

int sipf_profile_read(sipf_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(SIPF_EINVAL, "NULL argument");
    int rc = drain_marks(c);
    if (rc) return rc;
    for (int i = 0; i < SIPF_NPHASES; ++i) {
        ms[i] = c->prof_ms[i];
        launches[i] = c->prof_n[i];
    }
    return SIPF_OK;
}

int sipf_adjoint(sipf_ctx* c, int64_t nsteps, int32_t ckpt_every, const void* phi_bar, double* loss, double* dchi,
                 double* dmu, void* dX0) {
    if (!c || !loss || !dchi || !dmu || !dX0) return fail(SIPF_EINVAL, "NULL argument");
    if (nsteps < 1 || nsteps > (int64_t)1 << 30) return fail(SIPF_EINVAL, "nsteps must be >= 1");
    if (ckpt_every < 1) return fail(SIPF_EINVAL, "ckpt_every must be >= 1");
    return c->prec == SIPF_FP32
               ? adjoint_typed<float>(c, nsteps, ckpt_every, (const float*)phi_bar, loss, dchi, dmu, (float*)dX0)
               : adjoint_typed<double>(c, nsteps, ckpt_every, (const double*)phi_bar, loss, dchi, dmu, (double*)dX0);
}

int sipf_save(sipf_ctx* c, const char*) {
    if (!c) return fail(SIPF_EINVAL, "ctx is NULL");
    return fail(SIPF_EIO, "save not available in this build");
}

int sipf_load(const char*, void*, sipf_ctx** out) {
    if (out) *out = nullptr;
    return fail(SIPF_EIO, "load not available in this build");
}

int sipf_destroy(sipf_ctx* c) {
    if (!c) return SIPF_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_ctx(c);
    return SIPF_OK;
}

int sipf_batch_init(int32_t, const sipf_params*, const int64_t*, const void* const*, void*, sipf_batch** out) {
    if (out) *out = nullptr;
    return fail(SIPF_EINVAL, "batched mode not available in this build");
}
int sipf_batch_run(sipf_batch*, int64_t) { return fail(SIPF_EINVAL, "batched mode not available in this build"); }
int sipf_batch_get_positions(sipf_batch*, int32_t, void*, int) {
    return fail(SIPF_EINVAL, "batched mode not available in this build");
}
int sipf_batch_get_field(sipf_batch*, int32_t, int, void*, int) {
    return fail(SIPF_EINVAL, "batched mode not available in this build");
}
int sipf_batch_destroy(sipf_batch*) { return SIPF_OK; }

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
    if (count < 0 || (count > 0 && (!X || !cells))) return fail(SIPF_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    if (prm->precision == SIPF_FP32)
        HIPCHK(launch_cells<float>((const float*)X, count, prm->H, (float)(prm->H / prm->L), cells, s));
    else
        HIPCHK(launch_cells<double>((const double*)X, count, prm->H, (double)(prm->H / prm->L), cells, s));
    HIPCHK(hipStreamSynchronize(s));
    return SIPF_OK;
}

int sipf_dbg_deposit(const sipf_params* prm, int64_t count, const void* X, void* phi, void* hip_stream) {
    if (!phi) return fail(SIPF_EINVAL, "phi is NULL");
    sipf_ctx* c = nullptr;
    int rc = sipf_init(prm, count, X, 1, nullptr, 0, hip_stream, &c);
    if (rc) return rc;
    rc = sipf_get_field(c, SIPF_FIELD_RHO, phi, 1);
    sipf_destroy(c);
    return rc;
}

}  // extern "C"
