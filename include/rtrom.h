/*
 * rtrom.h -- C ABI of librtrom.so: on-the-fly ROM-accelerated source
 * iteration with diffusion synthetic acceleration (SI-DSA) for backward-Euler,
 * discrete-ordinates radiative transfer with isotropic scattering, on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Liu & Peng, "On-the-Fly ROM-Based Acceleration of SI-DSA for
 * Implicit Time Marching of the Radiative Transfer Equation" (arXiv 2603.19647).
 *
 * Conventions
 *  - Every call returns rtrom_status (or nothing for destroy); nothing throws
 *    across the ABI.  On an error, rtrom_last_error() returns a message
 *    (thread-local, valid until the next call on the same thread).
 *  - All array arguments are HOST pointers.  create / submit copy every input
 *    array; the caller may free them as soon as the call returns.  Output
 *    buffers are caller owned and carry an explicit element count; a count
 *    that is too small gives RTROM_EINVAL and writes nothing.
 *  - A problem handle owns all of its device state (angular flux, density,
 *    right-hand side, ROM bases, state machine).  A handle is not thread safe;
 *    distinct handles may be used from different threads.
 *  - Arguments are validated on the host before any device call, so every
 *    RTROM_EINVAL path runs without a GPU.
 *  - Layout of per-cell arrays: [ny][nx], x fastest.  1D: ny = 1.
 *  - "rho" is the paper's density: the angular average with quadrature
 *    weights summing to one (Sec. 2, eq. governing and Sec. 2.1).  The
 *    conventional scalar flux is 2 rho (slab) or 4 pi rho (sphere).
 */
#ifndef RTROM_H
#define RTROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTROM_OK = 0,
  RTROM_EINVAL = -1,  /* invalid argument; nothing was changed */
  RTROM_ENOMEM = -2,  /* device or host allocation failed / budget exceeded */
  RTROM_ENOCONV = -3, /* a step hit max_iter: the state DID advance with the
                         last iterate and the step is counted in
                         rtrom_stats.nonconverged_steps */
  RTROM_EDEVICE = -4, /* HIP runtime error or no usable gfx950 device */
  RTROM_EBUSY = -5    /* server: result not ready yet */
} rtrom_status;

/* Inner solver (Sec. 2.3 Alg. 1; Sec. 3.2 Alg. 2). */
typedef enum {
  RTROM_SI_DSA = 0,     /* memory-efficient SI with DSA (Alg. 1) */
  RTROM_ROM_SI_DSA = 1, /* on-the-fly DMD initial guess + hybrid ROM/DSA
                           preconditioner with error-indicator updates (Alg. 2) */
  RTROM_SI_PLAIN = 2    /* unaccelerated source iteration (reference only) */
} rtrom_method;

typedef enum {
  RTROM_FP64 = 0,  /* every sweep in FP64 */
  RTROM_MIXED = 1  /* SI increments swept in FP32, accumulated in FP64; the
                      stop test runs at tol / 16 and is re-checked on an FP64
                      sweep before a step is accepted (DG-P1: also on the
                      step to the next DSA-corrected iterate).  f, b~, rho
                      and all ROM work stay FP64. */
} rtrom_precision;

/* Correction applied where Alg. 1 uses DSA. */
typedef enum {
  RTROM_PC_DSA = 0, /* diffusion synthetic acceleration (Sec. 2.3, eq. rho_residual) */
  RTROM_PC_MH = 1   /* McClarren-Haut (Sec. 3.3): a DMD model of the sweep
                       operator T Sigma_s built from the pairs of the current
                       step's iterates, rho^{(l-1)} - rho^{(l-2)} and their
                       images, gives d = Q (I - A~)^{-1} A~ Q^T (y - rho^{(l-1)})
                       (eq. ideal_correct restricted to the pairs' span).  With
                       RTROM_ROM_SI_DSA this is the hybrid of Sec. 4.5: the ROM
                       initial guess and first correction, McClarren-Haut for
                       the later iterations.  Slabs: at most 2048 cells. */
} rtrom_precond;

/* Time discretisation (Sec. 2.1). */
typedef enum {
  RTROM_BE = 0,  /* backward Euler (eq. time_discrete) */
  RTROM_BDF2 = 1 /* BDF2, (3 f^n - 4 f^{n-1} + f^{n-2}) / (2 dt), started with
                    one backward-Euler step (which is not a ROM snapshot: it
                    solves with another operator).  Slabs: at most 2048 cells. */
} rtrom_time_scheme;

/* Spatial discretisation (Sec. 2.1, eq. DG). */
typedef enum {
  RTROM_FV = 0,  /* piecewise constants (K = 0): first-order upwind finite volume */
  RTROM_DG1 = 1  /* piecewise linears (K = 1) on slabs: two unknowns per cell
                    (the cell average and the slope coefficient of the
                    orthonormal basis 1, sqrt(3) xi), so rho, f and b~ hold
                    2 nx values per ordinate, cell-major; DSA by the modified
                    interior-penalty discretisation of the correction's
                    diffusion limit.  Slabs of at most 1024 cells. */
} rtrom_scheme;

/* flags */
#define RTROM_F_ABS_UP_NORM 0x1ull /* error indicators in the paper's absolute
                                      2-norm instead of relative to ||rho^n|| */
#define RTROM_F_SINGLE_WG 0x2ull   /* 1D: run the SI loop on one workgroup even
                                      when the problem is marched on its own
                                      (by default such a march splits the
                                      ordinate pairs over up to 16 co-resident
                                      workgroups; batches and the server always
                                      use one workgroup per problem).  Results
                                      are deterministic either way; the two
                                      modes differ at rounding level. */

typedef struct rtrom_problem rtrom_problem; /* opaque */

/* Problem statement: the paper's eq. rte (one group, isotropic scattering,
 * isotropic inflow g and initial state f0) on a uniform mesh, S_N ordinates
 * (Gauss-Legendre in 1D; Chebyshev-Legendre CL(n_azim, n_polar) in 2D,
 * App. A), backward Euler with step dt (Sec. 2.1), first-order upwind finite
 * volumes (the piecewise-constant member of eq. DG), solver parameters of
 * Alg. 1 / Alg. 2. */
typedef struct {
  int32_t dim;        /* 1 = slab [0,lx]; 2 = rectangle [0,lx] x [0,ly] */
  int32_t nx, ny;     /* cells; ny must be 1 when dim == 1 */
  double lx, ly;      /* domain lengths (> 0); ly ignored in 1D */
  int32_t n_polar;    /* 1D: Gauss-Legendre order; 2D: N_z.  Even, >= 2 */
  int32_t n_azim;     /* 1D: must be 1; 2D: N_phi, a multiple of 4 */
  const double *sigma_s, *sigma_a, *source; /* [ny*nx], >= 0 (source finite) */
  const double *f0;   /* [ny*nx] isotropic initial state, NULL = 0 */
  double inflow[4];   /* isotropic inflow g on x-lo, x-hi, y-lo, y-hi */
  double dt;          /* > 0 */
  double tol;         /* eps_SISA, > 0: stop when ||y - rho||_inf < tol ||y||_inf */
  int32_t max_iter;   /* N_iter >= 1 */
  int32_t method;     /* rtrom_method */
  int32_t precision;  /* rtrom_precision */
  double eps_ig, eps_pc, eps_up; /* eq. ig_stop, eq. pc_stop, update threshold */
  int32_t r_max;      /* ROM rank cap, 1 .. 20 */
  uint64_t flags;     /* RTROM_F_* */
  /* Fields added after the paper's default configuration; zero keeps it. */
  int32_t precond;     /* rtrom_precond */
  int32_t time_scheme; /* rtrom_time_scheme */
  int32_t pc_levels;   /* correction ROMs for iterations 1..pc_levels, built
                          one after the other (Sec. 3.2, key feature 1): the
                          ROM of iteration l takes the pairs rho^n -
                          rho^{(l-1/2)}, rho^{(l-1/2)} - rho^{(l-1)} once the
                          ROMs below it are complete.  0 or 1: the paper's
                          single level; at most 4 */
  int32_t mh_rank;     /* McClarren-Haut pairs per model (a full model restarts
                          from the newest pair), 0 = r_max; at most 20 */
  int32_t scheme;      /* rtrom_scheme */
  int32_t pad_;        /* zero */
  double lu_tol;       /* a reduced ROM system (Sec. 3.2, eq. dmd-ig / dmd-sa)
                          whose LU meets a pivot below lu_tol times its largest
                          entry is singular, and the step falls back to the
                          plain initial guess or DSA for that ROM (counted in
                          rom_fallbacks).  0 = 1e-14; must be finite and >= 0.
                          A value >= 1 makes every reduced system singular,
                          which forces the fallback path (a test of it) */
} rtrom_problem_desc;

typedef struct {
  int64_t steps;              /* time steps taken */
  int64_t si_iters_total;     /* SI sweeps (Alg. 1 iterations), all steps */
  int64_t sweeps_total;       /* SI sweeps + 2 per step (RHS and final f) */
  int32_t si_iters_last;      /* SI sweeps of the last step */
  int32_t phase;              /* 1, 2 or 3 (Sec. 3.2) for the next step */
  int32_t n0, n1;             /* eq. ig_stop step N0; eq. pc_stop count N1 */
  int32_t rank_ig, rank_pc;   /* current ROM ranks */
  int32_t nonconverged_steps;
  int32_t rom_fallbacks;      /* times a ROM due to apply (initial guess,
                                 correction, correction level) met a singular
                                 reduced system, so that its step took the
                                 plain initial guess or DSA instead */
  int64_t ig_updates, pc_updates; /* snapshots added to each ROM */
  int64_t fp32_sweeps;        /* mixed mode: SI sweeps done in FP32 */
  double last_residual;       /* ||y - rho||_inf / ||y||_inf of the last step */
  double t_total_s;           /* device time of all march/step calls (events) */
  int32_t dsa_iters;          /* 2D: Chebyshev iterations per DSA solve (fixed
                                 by the operator's Gershgorin bounds for a
                                 1e-14 error bound); 1D: 0 (direct solve) */
  int32_t reserved_;
} rtrom_stats;

/* Per-step record (rtrom_get_history). */
typedef struct {
  int32_t iters, phase, converged, ig_update, pc_update, rank_ig, rank_pc, fallback;
  double e_ig, e_pc; /* error indicators (negative when not evaluated) */
  double residual;
} rtrom_step_record;

/* Create a problem: validates `d`, builds the quadrature, uploads materials,
 * expands f0 to every ordinate and runs the first RHS sweep (b~^0, Sec. 2.3).
 * On success *out owns the problem.  Errors: EINVAL (description), ENOMEM,
 * EDEVICE. */
rtrom_status rtrom_create_problem(const rtrom_problem_desc *d, rtrom_problem **out);

/* Advance one time step n -> n+1 (Alg. 2 around Alg. 1).  Synchronous.
 * Returns ENOCONV when the step hit max_iter (the state still advanced). */
rtrom_status rtrom_step(rtrom_problem *p);

/* Advance nsteps >= 0 steps on the problem's stream, then synchronise.
 * ENOCONV if any step hit max_iter. */
rtrom_status rtrom_march(rtrom_problem *p, int32_t nsteps);

/* Advance every problem of `ps` (n >= 1 distinct handles, any mix of sizes
 * and ordinate counts of the same dimension) by nsteps, fusing them into
 * shared launches (one workgroup per 1D instance, the largest dispatched
 * first).  Each problem's result is bitwise what it gets marched alone in
 * one-workgroup mode, whatever it is batched with and wherever it sits in
 * `ps`.  All handles must live on the same device.  ENOCONV if any step of
 * any problem hit max_iter. */
rtrom_status rtrom_march_batch(rtrom_problem *const *ps, int32_t n, int32_t nsteps);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same as
 * rtrom_march_batch (same kernels, bitwise the same results) but it allocates
 * nothing: the batch's descriptor table and state copies live in a static
 * device array of the library, sized for RTROM_NOALLOC_MAX_BATCH problems
 * (about 1 MiB, one copy per device, held until the process ends), and the
 * problems' step histories are never grown.
 * Errors: EINVAL for n > RTROM_NOALLOC_MAX_BATCH, or when a problem's step
 * history cannot hold steps + nsteps records (histories hold 1024 steps from
 * creation and grow only in rtrom_march / rtrom_march_batch); nothing is
 * marched then.  Every call on a device shares that device's array: calls
 * that overlap on one device (several host threads) race and must be
 * serialised by the caller. */
#define RTROM_NOALLOC_MAX_BATCH 1024
rtrom_status rtrom_march_batch_noalloc(rtrom_problem *const *ps, int32_t n, int32_t nsteps);

/* rho^n (the converged density of the last step, Alg. 1's returned iterate),
 * n >= the number of unknowns: nx*ny, or 2*nx for RTROM_DG1 (per cell the
 * average, then the slope coefficient). */
rtrom_status rtrom_get_scalar_flux(const rtrom_problem *p, double *rho, int64_t n);

/* f^n, [ordinate][unknown] with the ordinate order of rtrom_get_quadrature,
 * n >= n_ord * unknowns doubles. */
rtrom_status rtrom_get_angular_flux(const rtrom_problem *p, double *f, int64_t n);

/* Right-hand side b~ of the next step (eq. implicit_linear_system_rho),
 * n >= unknowns doubles. */
rtrom_status rtrom_get_rhs(const rtrom_problem *p, double *b, int64_t n);

/* Quadrature used by the problem: n >= n_ord doubles each (oy, oz may be NULL
 * in 1D).  ox = mu in 1D. */
rtrom_status rtrom_get_quadrature(const rtrom_problem *p, double *ox, double *oy,
                                  double *oz, double *w, int64_t n);

/* Host-only quadrature builders (no device needed): Gauss-Legendre with
 * weights summing to one, and CL(n_azim, n_polar) in App. A order. */
rtrom_status rtrom_gauss_legendre(int32_t n, double *mu, double *w);
rtrom_status rtrom_cl_quadrature(int32_t n_azim, int32_t n_polar, double *ox,
                                 double *oy, double *oz, double *w);

/* Counters of the march so far (library bookkeeping; the counts are the
 * quantities Sec. 4 reports: SI sweeps per step, N0, N1, ranks). */
rtrom_status rtrom_stats_get(const rtrom_problem *p, rtrom_stats *out);

/* Correction ROMs of iterations 1..L (L = max(1, pc_levels); Sec. 3.2, key
 * feature 1): for level l, out[4 (l-1) + 0..3] = complete (0/1), steps its
 * construction took (N1 for l = 1), rank, snapshots added.  n: entries of
 * out (at least 4 L); *levels receives L.  Errors: EINVAL. */
rtrom_status rtrom_get_levels(const rtrom_problem *p, int64_t *out, int32_t n, int32_t *levels);

/* Per-step records of the last min(n, steps) steps in order. *written gets the
 * number of records copied. */
rtrom_status rtrom_get_history(const rtrom_problem *p, rtrom_step_record *out,
                               int64_t n, int64_t *written);

/* Replace the isotropic inflow for the following steps; b~ of the next step
 * is rebuilt with it (time-dependent boundary data).  g: 4 doubles. */
rtrom_status rtrom_set_inflow(rtrom_problem *p, const double *g);

/* Launch on `hip_stream` (a hipStream_t, e.g. torch's current stream) from now
 * on; NULL selects the problem's own stream.  Library plumbing, no passage of
 * the paper. */
rtrom_status rtrom_set_stream(rtrom_problem *p, void *hip_stream);

/* Bytes of device memory owned by the problem (library plumbing). */
rtrom_status rtrom_device_bytes(const rtrom_problem *p, uint64_t *bytes);

/* Bytes a problem with description d would own (for admission control). */
rtrom_status rtrom_estimate_bytes(const rtrom_problem_desc *d, uint64_t *bytes);

void rtrom_destroy_problem(rtrom_problem *p); /* NULL -> no-op */

/* Kernel timing (library instrumentation, no passage of the paper).  While enabled, every kernel launch of every problem is
 * bracketed by HIP events on the stream it runs on, and the device time and
 * launch count of each kernel kind accumulate process-wide (read after the
 * march returns).  Kinds: 0 slab SI solve, 1 slab f-pass, 2 ROM bookkeeping and
 * incremental-SVD projections, 3 plane sweep, 4 plane DSA, 5 plane f-pass,
 * 6 plane other, 7 ROM basis rotation.  Enabling or disabling resets the
 * totals. */
#define RTROM_NKINDS 8
rtrom_status rtrom_profile_enable(int32_t on);
rtrom_status rtrom_profile_read(double *seconds, int64_t *launches, int32_t nkinds);

const char *rtrom_last_error(void);

/* ---- serving: continuous batching of independent problems ---------------
 * (Sec. 4 runs one problem at a time; serving many is this library's.)
 * A request is one time-marching problem (desc + nsteps).  Requests queue in
 * submission order; max_slots worker threads admit the head of the queue as
 * soon as a slot is free and its device footprint (rtrom_estimate_bytes plus
 * its step history) fits the rest of hbm_budget_bytes.  Admitted problems
 * march concurrently, each on its own streams, so their kernels overlap on
 * the device; a finished march copies rho and the statistics to the host and
 * releases the device state, freeing budget.  A result depends only on its
 * own request (own state, fixed launch shapes, fixed-order reductions): it is
 * the same alone and in the mix.  Handles are thread-safe; profiling
 * (rtrom_profile_enable) must stay off while a server runs. */
typedef struct rtrom_server rtrom_server;
typedef struct {
  uint64_t hbm_budget_bytes; /* admission budget for problem state */
  int32_t max_slots;         /* concurrent problems (worker threads), 1..256 */
  int32_t device;            /* HIP device ordinal */
  int32_t steps_per_tick;    /* reserved (problems advance one step at a time) */
} rtrom_server_desc;

enum { RTROM_REQ_QUEUED = 0, RTROM_REQ_RUNNING = 1, RTROM_REQ_DONE = 2, RTROM_REQ_FAILED = 3 };

/* Initialises the HIP runtime on the calling thread and starts the worker
 * threads.  EINVAL on bad arguments, EDEVICE without a usable device. */
rtrom_status rtrom_server_create(const rtrom_server_desc *d, rtrom_server **out);
/* Validates and copies d (the caller may free its arrays on return);
 * non-blocking.  EINVAL for an invalid description, ENOMEM if the request can
 * never fit the budget. */
rtrom_status rtrom_server_submit(rtrom_server *s, const rtrom_problem_desc *d,
                                 int32_t nsteps, uint64_t *ticket);
/* state = RTROM_REQ_*; EINVAL for an unknown (or already fetched) ticket. */
rtrom_status rtrom_server_poll(rtrom_server *s, uint64_t ticket, int32_t *state);
/* Blocks until every submitted request has finished. */
rtrom_status rtrom_server_drain(rtrom_server *s);
/* Copies out a finished request's rho (n >= its unknowns), stats, per-step latencies
 * (seconds, up to nlat) and its march latency from admission to completion,
 * then forgets the ticket.  EBUSY if not finished; a failed request returns
 * its error.  Returns ENOCONV when some step hit max_iter (R8). */
rtrom_status rtrom_server_fetch(rtrom_server *s, uint64_t ticket, double *rho, int64_t n,
                                rtrom_stats *st, double *step_lat_s, int64_t nlat,
                                double *march_lat_s);
/* Stops admitting, ends running marches at their next step, joins the
 * workers.  NULL is a no-op. */
void rtrom_server_destroy(rtrom_server *s);

#ifdef __cplusplus
}
#endif
#endif /* RTROM_H */
