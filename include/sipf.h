/*
 * sipf.h -- C ABI of the SIPF-PIC time step on AMD Instinct MI355X (gfx950).
 *
 * The method is the stochastic interacting particle-field method with
 * particle-in-cell acceleration of Hu, Wang, Xin and Zhang (arXiv:2512.03452)
 * for the 3-D parabolic-parabolic Keller-Segel system
 *     rho_t = div(mu grad rho - chi rho grad c),
 *     eps c_t = lap c - k^2 c + rho                       (eq. para_system)
 * on the periodic box [-L/2, L/2)^3 (Sec. 2.2).  One step (Algorithm 4):
 *   1. deposit the P equal-mass particles onto the H^3 grid with the
 *      fourth-order stencil (Definition particle2grid, Algorithm 2);
 *   2. forward FFT, beta_q = L^-3 sum_j phi_j exp(-2 pi i q.j/H) (Sec. 3.1);
 *   3. implicit mode update alpha_q <- A_q alpha_q + B_q beta_q
 *      (eq. alpha_hat_update);
 *   4. spectral gradient of the previous field with the Gaussian filter
 *      Phi_q = exp(-2 pi^2 |q|^2 / H0^2), inverse FFT to the grid (Algorithm 4);
 *   5. trilinear interpolation back to the particles (Definition
 *      grid2particle, Algorithm 3) and the stochastic push: split
 *      (W^- , drift, W^+; Algorithm 4) or Euler-Maruyama (eq. rho_hat_update).
 * Both branches of step n read the state after step n-1 (Algorithm 4), so the
 * gradient gathered in step n is that of alpha^(n-1).
 *
 * Noise (the paper fixes no generator): particle id (its index in X0) at
 * step n draws one Philox4x32-10 block with key (low, high 32 bits of seed)
 * and counter (id, n, 0, instance).  Its 128 bits give six 21-bit fields
 * f_i = r_i >> 11 (i < 4), f_4 = (r0 & 0x7FF) << 10 | (r1 & 0x3FF),
 * f_5 = (r2 & 0x7FF) << 10 | (r3 & 0x3FF), uniforms u = (f + 1/2) 2^-21 and
 * three Box-Muller pairs z = sqrt(-2 ln u_2j) (cos, sin)(2 pi u_2j+1).
 * Split step: W^- = sqrt(mu tau) (z0, z1, z2), W^+ = sqrt(mu tau) (z3, z4, z5);
 * Euler-Maruyama: W = sqrt(2 mu tau) (z0, z1, z2).
 *
 * Conventions for every function below:
 *   - Return value: SIPF_OK (0) or a negative SIPF_E* code.  The message of the
 *     last failure on the calling thread is returned by sipf_last_error().
 *     No C++ exception crosses this interface.
 *   - Positions are P x 3, row-major (x, y, z per particle), in the context's
 *     precision (float for SIPF_FP32, double for SIPF_FP64), in original
 *     particle order.  "on_device" arguments say whether a pointer is device
 *     memory (1) or host memory (0); device pointers must be on the current
 *     HIP device.
 *   - Spectral arrays are the Hermitian half spectrum of a real field:
 *     H x H x (H/2+1) interleaved complex (re, im) values, index
 *     (kx, ky, kz) at (kx*H + ky)*(H/2+1) + kz; array index k stands for the
 *     frequency q = k for k < H/2 and q = k - H otherwise (kz = 0..H/2).
 *   - Grids are H x H x H real arrays, index (ix, iy, iz) at (ix*H + iy)*H + iz;
 *     node g (integer vector, position g*L/H) is stored at g mod H.
 *   - All work is enqueued on the context's HIP stream and is asynchronous
 *     unless stated otherwise.  A context is not thread-safe; distinct
 *     contexts are independent.  After SIPF_EDEVICE the context must be
 *     destroyed.
 *   - H must be a power of two with 8 <= H <= 256 (FP32) or 8 <= H <= 64
 *     (FP64).  Up to H = 128 one yz-plane of the half spectrum is transformed
 *     in the 160 KB of LDS of a gfx950 compute unit; at H = 256 the plane
 *     passes split into row and column passes; sipf_adjoint and the direct
 *     method take H <= 128.  The mixed-radix grids H = 12, 22, 46 (both
 *     precisions) and 90 (FP32) of the SIPF against SIPF-PIC comparison
 *     (Sec. 5.1) are also accepted; on them the tile side is any integer
 *     with at most 16 tiles per axis (the last may be partial), and
 *     sipf_adjoint returns SIPF_EINVAL.  Other sizes return SIPF_EINVAL.
 *
 * Variants (Sec. 5.2):
 *   - eps = 0 makes the c-equation elliptic, -lap c + k^2 c = rho: the mode
 *     update becomes alpha_q = B_q beta_q with B_q = 1/(|xi_q|^2 + k^2), and
 *     alpha_0 = 0 when k = 0 (the periodic problem only sees rho minus its
 *     mean and fixes c up to a constant).  tau still sets the push.
 *   - sipf_params.dim = 2 runs the same algorithm in two dimensions on
 *     [-L/2, L/2)^2: the 12-node fourth-order deposit (the construction of
 *     eq. 4ord with d = 2), bilinear gather, beta_q = L^-2 sum_j phi_j
 *     exp(-2 pi i q.j/H).  Positions are P x 2; grids H x H (index ix*H + iy);
 *     spectra H x (H/2+1) (index kx*(H/2+1) + ky, ky = 0..H/2); gradients
 *     2 x H^2.  Split-step noise W^- = sqrt(mu tau) (z0, z1),
 *     W^+ = sqrt(mu tau) (z2, z3); Euler-Maruyama W = sqrt(2 mu tau) (z0, z1).
 *     H is a power of two with 8 <= H <= 4096 in both precisions (one row of
 *     the spectrum and its twiddles fit in LDS).  sipf_adjoint and the test
 *     entry points are 3-D only (SIPF_EINVAL); every other call works in 2-D
 *     with the sizes above.
 */
#ifndef SIPF_H
#define SIPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SIPF_OK        0
#define SIPF_EINVAL   (-1)  /* invalid argument or parameter; nothing was touched */
#define SIPF_ENOMEM   (-2)  /* device or host allocation failed */
#define SIPF_EDEVICE  (-3)  /* HIP runtime error; destroy the context */
#define SIPF_ENUMERIC (-4)  /* NaN/Inf in inputs or produced by a step */
#define SIPF_ESTATE   (-5)  /* call not valid in the context's current state */
#define SIPF_EIO      (-6)  /* snapshot file missing, truncated or corrupt */

/* particle push (Algorithm 4 split step, or eq. rho_hat_update) */
#define SIPF_STRANG 0       /* X' = wrap(Y + chi tau I*grad c(Y) + W+), Y = X + W-, W+- ~ N(0, mu tau) */
#define SIPF_EM     1       /* X' = wrap(X + chi tau I*grad c(X) + W),  W ~ N(0, 2 mu tau) */

/* propagator of the c-equation over one step (eps > 0) */
#define SIPF_PROP_IMPLICIT 0  /* eq. alpha_hat_update: alpha' = A (alpha + (tau/eps) beta), A = 1/(1 + tau s/eps) */
#define SIPF_PROP_EXP      1  /* Sec. 3.4: the same with kappa = exp(-tau s/eps) in place of A; s = |xi|^2 + k^2 */

/* method of a context: SIPF-PIC (Algorithm 4), or the direct SIPF method of
 * Algorithm 1 (every particle meets every mode of U, O(P H^3) per step, no
 * grid), the baseline the particle-in-cell step is measured against.  A
 * direct context is three-dimensional and single-instance; it supports
 * sipf_step/run/sync/get_step/get_positions/get_params/destroy and
 * sipf_get_field(SIPF_FIELD_ALPHA) (the kz = 0..H/2 half of its full
 * spectrum); the other calls return SIPF_EINVAL.  Its push follows
 * sipf_params.scheme (Algorithm 1 prints Euler-Maruyama) and its gradient
 * sum is Re sum_{q in U} i xi_q Phi_q alpha_q exp(i xi_q . X) (eq. gradc; set
 * H0 < 0 for Algorithm 1's unfiltered sum).  An alpha0 given to sipf_init is
 * extended to U by Hermitian symmetry. */
#define SIPF_METHOD_PIC    0
#define SIPF_METHOD_DIRECT 1

/* sipf_params.positivity = 1: positivity-preserving deposit, the smoothing near
 * the edge of the particle cloud that Remark `smoothness` (Sec. 3.1) asks for
 * so that the operator-splitting update of Sec. 3.4 keeps c non-negative (the
 * paper cites the procedure without giving it; this is the reading built
 * here).  After the order-4 deposit, rounds repeat until one switches nobody:
 * every particle still on the order-4 weights whose 32 stencil nodes include a
 * node where the deposit is below -2^-20 (FP32) or -2^-44 (FP64) of a
 * particle's mass M0/P switches to the order-2 weights of eq. 2ord; then
 * negative values left by rounding are set to zero.  The mass is unchanged up
 * to that rounding; in the bulk of the cloud the deposit stays order 4.  Each
 * round reads a count on the host, so such a context steps without graphs
 * (sipf_use_graphs keeps them off).  3-D SIPF-PIC only; all instances of a
 * batch share it; sipf_adjoint returns SIPF_EINVAL.  It applies to the step's
 * deposit, sipf_get_field(SIPF_FIELD_RHO) and sipf_diagnostics. */

/* sipf_params.particle_pass: how the FP32 3-D step runs its particle pass
 * (deposit of Algorithm 2, then gather and push of Algorithm 3).  Both give
 * the same deposit up to the rounding of the weights' fixed-point sums, and
 * the same positions; they differ in speed, which depends on the workload.
 *   SIPF_PASS_TWO_PHASE  each work item (particles of one tile) deposits all
 *                        its particles, then gathers and pushes them;
 *   SIPF_PASS_SORTED     each work item keeps its particles sorted by cell,
 *                        deposits runs of equal cells as one sum, and pushes
 *                        particles while it deposits (both LDS windows live);
 *   SIPF_PASS_DEFAULT    the two-phase pass for a single instance, the sorted
 *                        pass for a batch of several.
 * FP64 and 2-D steps always take the two-phase pass. */
#define SIPF_PASS_DEFAULT   0
#define SIPF_PASS_SORTED    1
#define SIPF_PASS_TWO_PHASE 2

/* arithmetic precision of particles, grids and spectra */
#define SIPF_FP32 0
#define SIPF_FP64 1

/* fields for sipf_get_field */
#define SIPF_FIELD_RHO   0  /* deposit of the current positions, mass units, H^3 real */
#define SIPF_FIELD_ALPHA 1  /* current alpha^(n), half spectrum */
#define SIPF_FIELD_GRAD  2  /* grad c of alpha^(n) on the grid (filtered), 3 x H^3 real, d-major */

/*
 * Problem and discretisation parameters.  Physical constants follow
 * eq. para_system; H, H0 and tau follow Algorithm 4; the default H0 rule is
 * the one of Sec. 5.1.  Fill with sipf_params_default() and override.
 */
typedef struct sipf_params {
    double   L;            /* box side; Omega = [-L/2, L/2)^3, periodic            */
    double   chi;          /* chemotactic sensitivity (>= 0)                      */
    double   mu;           /* particle diffusivity (>= 0)                         */
    double   eps;          /* relaxation constant of c (>= 0; 0: elliptic)        */
    double   k;            /* degradation constant of c (>= 0)                    */
    double   M0;           /* total mass of the particles (>= 0)                  */
    double   dt;           /* time step tau (> 0)                                 */
    double   H0;           /* filter scale; 0: ceil(8 H^(8/13) L^(5/13)); <0: off */
    int32_t  H;            /* grid points per axis (see above)                    */
    int32_t  p2g_order;    /* must be 4 (Remark after Definition grid2particle)  */
    int32_t  g2p_order;    /* must be 2 (same remark)                             */
    int32_t  scheme;       /* SIPF_STRANG (default) or SIPF_EM                    */
    int32_t  precision;    /* SIPF_FP32 (default) or SIPF_FP64                    */
    int32_t  tile;         /* binning tile side in cells; 0 = tuned default; at most
                              16 (3-D) or 64 (2-D) tiles per axis; a power of two,
                              or any side when H is not one                      */
    int32_t  resort_every; /* re-sort period in steps; 0 = default: 6 in 3-D, 4 in 2-D,
                              or fewer when sqrt(2 mu tau n) exceeds a quarter of a tile */
    int32_t  chunk;        /* max particles per work item of the particle pass (256..4096); 0 = default:
                              4096 in 2-D and from 2^23 particles per 3-D group, else 3072;
                              the adjoint's reverse pass then uses items of at most 2048 */
    uint64_t seed;         /* Philox key                                          */
    uint32_t instance;     /* fourth Philox counter word                          */
    uint32_t dim;          /* space dimension: 3 (0 means 3) or 2                 */
    int32_t  propagator;   /* SIPF_PROP_IMPLICIT (default) or SIPF_PROP_EXP (needs eps > 0) */
    int32_t  method;       /* SIPF_METHOD_PIC (default, Algorithm 4) or SIPF_METHOD_DIRECT */
    int32_t  positivity;   /* 1: positivity-preserving deposit (see below), 0: plain order 4 */
    int32_t  particle_pass; /* FP32 3-D deposit + push pass: SIPF_PASS_DEFAULT, SIPF_PASS_SORTED
                               or SIPF_PASS_TWO_PHASE (see below); ignored elsewhere          */
} sipf_params;

typedef struct sipf_ctx sipf_ctx;
typedef struct sipf_batch sipf_batch;

/* Fill *p with the defaults (L = 2, chi = mu = eps = k = 1, M0 = 1,
 * dt = 1e-4, H = 64, H0 = 0, orders 4/2, Strang, FP32, seed 0). */
int sipf_params_default(sipf_params* p);

/*
 * Create a simulation context (Algorithm 4 initialisation).
 *   P          number of particles (1 <= P < 2^32); each carries mass M0/P
 *              (eq. def_rho_hat).
 *   X0         initial positions, P x 3 in the context precision (host or
 *              device per x0_on_device); wrapped into [-L/2, L/2) on entry.
 *   alpha0     initial coefficients of c (half spectrum, context precision,
 *              host or device per alpha0_on_device), or NULL for c(x,0) = 0.
 *   hip_stream hipStream_t the context enqueues on (NULL = default stream).
 * The inputs are copied into library-owned device memory and the stream is
 * synchronised before return, so the caller may free X0/alpha0 afterwards.
 * Errors: SIPF_EINVAL (bad parameter), SIPF_ENUMERIC (NaN/Inf in X0),
 * SIPF_ENOMEM, SIPF_EDEVICE.  On error *out is NULL.
 */
int sipf_init(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device,
              const void* alpha0, int alpha0_on_device, void* hip_stream, sipf_ctx** out);

/* Advance one step n-1 -> n (Algorithm 4).  Asynchronous. */
int sipf_step(sipf_ctx* ctx);

/* Advance nsteps >= 0 steps.  Asynchronous.  The run is cut into segments
 * (up to the next due re-sort; from a due re-sort, two re-sort periods) and
 * each segment replays a HIP graph captured on its first use (kernels only,
 * no memset or copy nodes), cached by (particle buffer set, steps since the
 * last re-sort, length).  Graph replay and eager stepping enqueue the same
 * kernels with the same arguments.  With graphs off, or while phase
 * profiling is on, every step is enqueued eagerly. */
int sipf_run(sipf_ctx* ctx, int64_t nsteps);

/* Capture, without running any step, every graph that sipf_run(ctx, nsteps)
 * issued next would replay, and upload each to the device on the context's
 * stream, so that the run itself only replays (graphs captured during a run
 * are uploaded the same way before their first launch).  The context's state
 * is unchanged.  Errors: SIPF_EINVAL (nsteps < 0), SIPF_EDEVICE (capture,
 * instantiation or upload failed). */
int sipf_prepare_run(sipf_ctx* ctx, int64_t nsteps);

/* Switch graph replay in sipf_run on (1, the default) or off (0). */
int sipf_use_graphs(sipf_ctx* ctx, int enable);

/* Wait for the context's stream and report any device-side error flag
 * (SIPF_ENUMERIC for a non-finite position). */
int sipf_sync(sipf_ctx* ctx);

/* The parameters the context was created with (tuning fields as given,
 * 0 where left to the defaults) and its particle count. */
int sipf_get_params(sipf_ctx* ctx, sipf_params* prm, int64_t* P);

/* Number of completed steps n (synchronises). */
int sipf_get_step(sipf_ctx* ctx, int64_t* n);

/* Current positions X^(n) in original particle order into a caller-owned
 * P x 3 buffer (host or device).  Synchronises. */
int sipf_get_positions(sipf_ctx* ctx, void* out, int on_device);

/* A field of the current state into a caller-owned buffer (see SIPF_FIELD_*;
 * sizes H^3, H*H*(H/2+1) complex, 3*H^3 in the context precision).
 * Synchronises. */
int sipf_get_field(sipf_ctx* ctx, int which, void* out, int on_device);

/*
 * Run-time diagnostics of the current state (Sec. 5.2 and 5.5), computed on
 * the device:
 *   step        completed steps n;
 *   mass        sum_j rho_num(x_j) h^3 over the grid nodes, h = L/H (equals
 *               M0 up to rounding);
 *   rho_max     max_j rho_num(x_j), the blow-up indicator of Sec. 5.2;
 *   hf_share    share of the energy of c_hat in the modes |q| >= 4:
 *               sum_{|q|>=4} |alpha_q|^2 / sum_q |alpha_q|^2 over the full
 *               spectrum of alpha^(n) (0 when alpha^(n) = 0);
 *   c_integral  integral of c_hat over the box, L^3 Re alpha_0^(n);
 *   r_num       (1/P) sum_p sqrt(X_p1^2 + X_p2^2) (Sec. 5.5);
 *   m2          (1/P) sum_p |X_p|^2, coordinates in [-L/2, L/2).
 * rho_num = rho_hat_P * G0 with G0 the isotropic Gaussian of standard
 * deviation L/H0 per axis, reconstructed on the grid as the step does it: the
 * order-4 deposit of X^(n), F_H, the factor exp(-2 pi^2 |q|^2 / H0^2) and the
 * inverse transform (no filter when H0 < 0).  The sums are FP64 and
 * deterministic for a given particle order.  The state is left unchanged.
 * The first call allocates a scratch buffer (about 64 KB per instance) that
 * the context keeps.  Synchronises.  Errors: SIPF_EINVAL for NULL
 * arguments, SIPF_EDEVICE, SIPF_ENUMERIC as for sipf_sync.
 */
typedef struct sipf_diag {
    int64_t step;
    double mass;
    double rho_max;
    double hf_share;
    double c_integral;
    double r_num;
    double m2;
} sipf_diag;
int sipf_diagnostics(sipf_ctx* ctx, sipf_diag* out);

/*
 * Pathwise adjoint (reverse mode along the fixed Philox noise path).
 * Runs nsteps forward steps from the current state (which must be the
 * initial state, n = 0, with alpha0 = 0; otherwise SIPF_ESTATE), storing the
 * positions every ckpt_every steps and alpha every step, then the reverse
 * sweep, recomputing positions inside each checkpoint segment.
 *   phi_bar  device pointer to dL/dphi^(N) (H^3, context precision) for a
 *            loss linear in the final deposit, or NULL for L = sum_j phi_j^2,
 *            phi the order-4 deposit of X^(N) in mass units (Algorithm 2).
 *   loss     out: L (host double).
 *   dchi,dmu out: dL/dchi, dL/dmu (host doubles).
 *   dX0      out: dL/dX^(0), device buffer P x 3 in original particle order.
 * floor() is treated as locally constant and the periodic wrap as the
 * identity (both hold almost everywhere).  After return the context holds
 * X^(N), alpha^(N) (n = nsteps).  Synchronises.  SIPF_EINVAL in two
 * dimensions, for the direct method and for H that is not a power of two.
 */
int sipf_adjoint(sipf_ctx* ctx, int64_t nsteps, int32_t ckpt_every, const void* phi_bar,
                 double* loss, double* dchi, double* dmu, void* dX0);

/*
 * Counts of the last positivity-preserving deposit of a context (see
 * sipf_params.positivity): *switched = particles that moved to the order-2
 * weights, *rounds = rounds that switched at least one.  Both 0 when the
 * option is off or nothing was negative.  Errors: SIPF_EINVAL for NULL
 * arguments.
 */
int sipf_positivity_stats(sipf_ctx* ctx, int64_t* switched, int32_t* rounds);

/* Per-phase timing with HIP events recorded on the context's stream around
 * every launch of the step's kernels (enable = 1 starts it, 0 stops it; the
 * accumulators are cleared on enable).  sipf_profile_read synchronises and
 * writes, for each of the SIPF_NPHASES phases (SIPF_PHASE_*), the summed
 * duration in milliseconds and the number of launches timed.  Used by the
 * benchmark to measure the dominant kernel live on the library's stream. */
#define SIPF_PHASE_SORT      0  /* tile sort (histogram, scan, scatter)           */
#define SIPF_PHASE_PARTICLES 1  /* fused deposit + gather + push                  */
#define SIPF_PHASE_FWD       2  /* forward yz-plane pass                          */
#define SIPF_PHASE_XPENCIL   3  /* x pencils + mode update + gradient spectra     */
#define SIPF_PHASE_INV       4  /* inverse yz-plane pass                          */
#define SIPF_NPHASES         5
int sipf_profile(sipf_ctx* ctx, int enable);
int sipf_profile_read(sipf_ctx* ctx, double* ms, int64_t* launches);

/* Snapshot (parameters, n, positions in original order, alpha^(n) in
 * natural order) to a file and back.  The noise is a function of
 * (seed, instance, particle id, n), so a loaded context draws the same
 * increments as the saved one would; its results agree with an uninterrupted
 * run up to the rounding of summation order (the deposit accumulates in an
 * order that depends on scheduling and on the particle sort).  The file is
 * native-endian; sipf_save: SIPF_EIO if the file cannot be written;
 * sipf_load: SIPF_EIO on a missing, truncated, oversized or corrupt file,
 * otherwise the errors of sipf_init. */
int sipf_save(sipf_ctx* ctx, const char* path);
int sipf_load(const char* path, void* hip_stream, sipf_ctx** out);

/* Release all device memory of the context (NULL is a no-op). */
int sipf_destroy(sipf_ctx* ctx);

/* Message of the last failure on this thread ("" if none). */
const char* sipf_last_error(void);

/*
 * Tile / chunk / re-sort autotuner.  Times nsteps steps (after a warm-up that
 * includes graph capture) of fresh contexts built from prm, P and X0 (same
 * meaning as in sipf_init), searching one axis at a time: the binning tile
 * (powers of two from 4 to 32, or 4, 6, 8, 12, 16, 24, 32 when H is not a
 * power of two, within the limits of sipf_params.tile), the
 * work-item size (1024, 2048, 3072, 4096), the re-sort period (2, 4, 6, 8, 16)
 * and, for FP32 3-D steps, the particle pass (sorted, two-phase), starting
 * from the defaults.  *best receives prm with tile, chunk, resort_every and
 * particle_pass set to the fastest combination found, *ms_per_step its time.
 * Every trial context is destroyed before return; each needs the memory of
 * one sipf_init.  Synchronises.  Errors: those of sipf_init.
 */
int sipf_autotune(const sipf_params* prm, int64_t P, const void* X0, int x0_on_device, int32_t nsteps,
                  void* hip_stream, sipf_params* best, double* ms_per_step);

/*
 * Batched ensembles: n (1..1024) independent instances advanced together.
 * Each has its own parameters (H, chi, mu, M0, dt, seed, instance word, tile
 * ...); all must share the precision and the scheme (SIPF_EINVAL otherwise).
 * The group's chunk is that of prm[0] and its re-sort period the smallest
 * of the instances' periods.  Per step the
 * batch issues one persistent particle launch over the work items of every
 * instance and one launch per FFT phase and distinct grid size H; every
 * re-sort period one sort of every instance (four launches).
 *   prm[i], P[i]  parameters and particle count of instance i;
 *   X0[i]         its P[i] x 3 positions (host or device per x0_on_device).
 * Inputs are copied; the caller keeps ownership.  Instance i of a batch
 * computes what a context created by sipf_init with prm[i], P[i], X0[i]
 * computes (same noise, same arithmetic), up to summation order.
 * sipf_batch_run advances every instance by nsteps (asynchronous, graph
 * replay as in sipf_run); the get functions address instance i and
 * synchronise; sipf_batch_profile/_read time the batch's phases as
 * sipf_profile does.  Errors as for the single-instance calls, plus
 * SIPF_EINVAL for an instance index out of range.
 */
int sipf_batch_init(int32_t n, const sipf_params* prm, const int64_t* P, const void* const* X0,
                    int x0_on_device, void* hip_stream, sipf_batch** out);
int sipf_batch_run(sipf_batch* b, int64_t nsteps);
int sipf_batch_prepare_run(sipf_batch* b, int64_t nsteps);  /* as sipf_prepare_run */
int sipf_batch_use_graphs(sipf_batch* b, int enable);
int sipf_batch_sync(sipf_batch* b);
int sipf_batch_get_step(sipf_batch* b, int32_t i, int64_t* n);
int sipf_batch_get_positions(sipf_batch* b, int32_t i, void* out, int on_device);
int sipf_batch_get_field(sipf_batch* b, int32_t i, int which, void* out, int on_device);
/* Diagnostics of every instance (out: n entries, see sipf_diagnostics). */
int sipf_batch_diagnostics(sipf_batch* b, sipf_diag* out);
int sipf_batch_profile(sipf_batch* b, int enable);
int sipf_batch_profile_read(sipf_batch* b, double* ms, int64_t* launches);
int sipf_batch_destroy(sipf_batch* b);

/*
 * Test entry points: each exposes one piece of the step on caller data.
 * All pointers are device pointers; each call synchronises the given stream.
 *
 * sipf_dbg_philox: for count counters ctr (count x 4 uint32: id, n, 0,
 *   instance in the step's stream; any words are accepted) under key seed,
 *   writes the raw Philox4x32-10 outputs (count x 4 uint32) and the six
 *   normals of the stream contract (count x 6 in the given precision).
 * sipf_dbg_cells: the integer cell g = floor(X H / L) (count x 3 int32) that
 *   the particle pass uses for positions X (count x 3, precision of prm).
 * sipf_dbg_deposit: phi = I(sum_p w delta_{X_p}) with w = M0/count on the
 *   H^3 grid (the deposit of Algorithm 2 through the binning + LDS path).
 */
int sipf_dbg_philox(uint64_t seed, int64_t count, const uint32_t* ctr, uint32_t* raw,
                    void* normals, int precision, void* hip_stream);
int sipf_dbg_cells(const sipf_params* prm, int64_t count, const void* X, int32_t* cells,
                   void* hip_stream);
int sipf_dbg_deposit(const sipf_params* prm, int64_t count, const void* X, void* phi,
                     void* hip_stream);

/* Return to the device the work buffers that sipf_adjoint keeps between
 * calls (on every device).  Call with no adjoint running. */
int sipf_release_cached_memory(void);

/*
 * Allocation-free deposit, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation and kernels as sipf_dbg_deposit, i.e.
 * phi = I(sum_p w delta_{X_p}) with w = M0/count on the H^3 grid, but every
 * intermediate (particle copies in two sort buffer sets, tile counts and
 * cursors, work items, descriptors) lives in a fixed-size static device
 * array of 32 MiB that each GPU the library runs on holds until the process
 * ends.  The call allocates nothing and does not synchronise: it only
 * enqueues kernels on hip_stream.  prm: three-dimensional, any precision,
 * no positivity option; count in [1, 524288]; X: count x 3 positions on the
 * device (precision of prm), read only; phi: H^3 device grid (precision of
 * prm), overwritten.  Non-finite positions are not reported.  All calls on
 * one GPU share that GPU's array, so calls that overlap in time on one GPU
 * (different streams or threads) race; serialise them.  Errors: SIPF_EINVAL
 * (NULL pointer, invalid parameters, count out of range), SIPF_EDEVICE (a HIP
 * launch failed or the scratch array's address could not be obtained).
 */
int sipf_deposit_noalloc(const sipf_params* prm, int64_t count, const void* X, void* phi,
                         void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SIPF_H */
