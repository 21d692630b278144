// rt_capi.hip -- the C ABI of librtrom: argument validation, quadrature,
// device arena layout, the time-marching driver and accessors.
#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rt_host.h"

namespace {
thread_local std::string g_err;
std::atomic<int> g_next_id{0};
}

int rt_log_level() {
  static const int level = [] {
    const char *e = std::getenv("RTROM_LOG");
    return e ? std::max(0, std::atoi(e)) : 0;
  }();
  return level;
}

void rt_log(int level, const char *fmt, ...) {
  if (rt_log_level() < level) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "rtrom: %s\n", buf);
  std::fflush(stderr);
}

void rt_mark(const char *msg) { roctxMarkA(msg); }
RtRange::RtRange(const char *name) { roctxRangePushA(name); }
RtRange::~RtRange() { roctxRangePop(); }

void rt_set_error(const std::string &m) {
  g_err = m;
  rt_log(1, "error: %s", m.c_str());
}

extern "C" const char *rtrom_last_error(void) { return g_err.c_str(); }

#define RT_HIP(call, msg)                                                      \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      rt_set_error(std::string(msg) + ": " + hipGetErrorString(e_));           \
      return RTROM_EDEVICE;                                                    \
    }                                                                          \
  } while (0)

static rtrom_status fail(rtrom_status s, const std::string &m) {
  rt_set_error(m);
  return s;
}

// ---------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------
namespace {
struct Prof {
  bool on = false;
  double sec[RT_NKINDS] = {0};
  int64_t cnt[RT_NKINDS] = {0};
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> kinds;  // per event pair
};
Prof g_prof;
hipEvent_t prof_event() {
  if (g_prof.used == g_prof.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
  }
  return g_prof.pool[g_prof.used++];
}
}  // namespace

namespace {
std::mutex g_prof_mu;  // concurrent 2D batch members record from several threads
}
void rt_prof_begin(int kind, hipStream_t s) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = prof_event();
  if (e) (void)hipEventRecord(e, s);
  g_prof.kinds.push_back(kind);
}
void rt_prof_end(int kind, hipStream_t s) {
  (void)kind;
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t e = prof_event();
  if (e) (void)hipEventRecord(e, s);
}
bool rt_prof_on() { return g_prof.on; }
void rt_prof_collect() {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (size_t k = 0; k < g_prof.kinds.size() && 2 * k + 1 < g_prof.used; ++k) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, g_prof.pool[2 * k], g_prof.pool[2 * k + 1]) == hipSuccess) {
      g_prof.sec[g_prof.kinds[k]] += ms * 1e-3;
      g_prof.cnt[g_prof.kinds[k]] += 1;
    }
  }
  g_prof.kinds.clear();
  g_prof.used = 0;
}

extern "C" rtrom_status rtrom_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  for (int k = 0; k < RT_NKINDS; ++k) {
    g_prof.sec[k] = 0.0;
    g_prof.cnt[k] = 0;
  }
  g_prof.kinds.clear();
  g_prof.used = 0;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_profile_read(double *seconds, int64_t *launches, int32_t nkinds) {
  if (!seconds || !launches || nkinds < 0) return fail(RTROM_EINVAL, "bad argument");
  for (int k = 0; k < nkinds; ++k) {
    seconds[k] = k < RT_NKINDS ? g_prof.sec[k] : 0.0;
    launches[k] = k < RT_NKINDS ? g_prof.cnt[k] : 0;
  }
  return RTROM_OK;
}

// ---------------------------------------------------------------------------
// Quadrature (host, FP64)
// ---------------------------------------------------------------------------

// Gauss-Legendre nodes by Newton's method on P_n from Tricomi's asymptotic
// initial guess; weights 2 / ((1 - x^2) P_n'(x)^2) scaled to sum to one.
extern "C" rtrom_status rtrom_gauss_legendre(int32_t n, double *mu, double *w) {
  if (n < 1 || !mu || !w) return fail(RTROM_EINVAL, "gauss_legendre: n >= 1 and non-null outputs required");
  const double pi = 3.14159265358979323846;
  for (int k = 1; k <= n; ++k) {
    // k-th largest root
    double th = pi * (4.0 * k - 1.0) / (4.0 * n + 2.0);
    double x = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
      double pm1 = 1.0, p = x;  // P_0, P_1
      for (int j = 2; j <= n; ++j) {
        double pn = ((2 * j - 1) * x * p - (j - 1) * pm1) / j;
        pm1 = p;
        p = pn;
      }
      if (n == 1) {
        p = x;
        pm1 = 1.0;
      }
      dp = n * (pm1 - x * p) / (1.0 - x * x);
      double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) <= 4e-16 * std::fabs(x) + 1e-300) {
        // one more evaluation of the derivative at the converged node
        pm1 = 1.0;
        p = x;
        for (int j = 2; j <= n; ++j) {
          double pn = ((2 * j - 1) * x * p - (j - 1) * pm1) / j;
          pm1 = p;
          p = pn;
        }
        dp = (n == 1) ? 1.0 : n * (pm1 - x * p) / (1.0 - x * x);
        break;
      }
    }
    mu[n - k] = x;
    w[n - k] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  // exact symmetry of the rule (nodes +-x share a weight)
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (std::fabs(mu[i]) + std::fabs(mu[n - 1 - i]));
    double ww = 0.5 * (w[i] + w[n - 1 - i]);
    mu[i] = -a;
    mu[n - 1 - i] = a;
    w[i] = w[n - 1 - i] = ww;
  }
  if (n % 2) mu[n / 2] = 0.0;
  return RTROM_OK;
}

// CL(N_phi, N_z) (App. A): azimuths (2k-1) pi / N_phi with weight 1/N_phi,
// Gauss-Legendre in z; ordering j = j2 * N_phi + j1.
extern "C" rtrom_status rtrom_cl_quadrature(int32_t n_azim, int32_t n_polar, double *ox, double *oy,
                                            double *oz, double *w) {
  if (n_azim < 1 || n_polar < 1 || !ox || !oy || !oz || !w)
    return fail(RTROM_EINVAL, "cl_quadrature: positive orders and non-null outputs required");
  std::vector<double> z(n_polar), wz(n_polar);
  rtrom_gauss_legendre(n_polar, z.data(), wz.data());
  const double pi = 3.14159265358979323846;
  for (int j2 = 0; j2 < n_polar; ++j2) {
    double sn = std::sqrt(std::max(0.0, 1.0 - z[j2] * z[j2]));
    for (int j1 = 0; j1 < n_azim; ++j1) {
      double phi = (2.0 * j1 + 1.0) * pi / n_azim;
      int j = j2 * n_azim + j1;
      ox[j] = std::cos(phi) * sn;
      oy[j] = std::sin(phi) * sn;
      oz[j] = z[j2];
      w[j] = wz[j2] / n_azim;
    }
  }
  return RTROM_OK;
}

// ---------------------------------------------------------------------------
// Validation (host only, before any device call)
// ---------------------------------------------------------------------------

static rtrom_status validate(const rtrom_problem_desc *d);
rtrom_status rt_validate(const rtrom_problem_desc *d) { return validate(d); }

static rtrom_status validate(const rtrom_problem_desc *d) {
  if (!d) return fail(RTROM_EINVAL, "null description");
  if (d->dim != 1 && d->dim != 2) return fail(RTROM_EINVAL, "dim must be 1 or 2");
  if (d->nx < 1 || d->ny < 1) return fail(RTROM_EINVAL, "nx, ny must be >= 1");
  if (d->dim == 1 && d->ny != 1) return fail(RTROM_EINVAL, "ny must be 1 in 1D");
  if (d->dim == 1 && d->nx > RT_SLAB_MAX_CELLS)
    return fail(RTROM_EINVAL, "1D problems are limited to 4096 cells");
  if (d->dim == 2 && ((int64_t)d->nx * d->ny > (1 << 22)))
    return fail(RTROM_EINVAL, "2D problems are limited to 4194304 cells");
  if (!(d->lx > 0.0) || !std::isfinite(d->lx)) return fail(RTROM_EINVAL, "lx must be > 0");
  if (d->dim == 2 && (!(d->ly > 0.0) || !std::isfinite(d->ly))) return fail(RTROM_EINVAL, "ly must be > 0");
  if (d->dim == 2 && rt_plane_needs_cyclic(d->ny) && d->nx > rt_plane_max_nx_cyclic())
    return fail(RTROM_EINVAL, "2D grids with more than 1024 rows are limited to nx <= 3840");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(RTROM_EINVAL, "dt must be > 0");
  if (!(d->tol > 0.0) || !std::isfinite(d->tol)) return fail(RTROM_EINVAL, "tol must be > 0");
  if (d->max_iter < 1) return fail(RTROM_EINVAL, "max_iter must be >= 1");
  if (d->n_polar < 2 || d->n_polar % 2) return fail(RTROM_EINVAL, "n_polar must be even and >= 2");
  if (d->n_polar > 256) return fail(RTROM_EINVAL, "n_polar must be <= 256");
  if (d->dim == 1 && d->n_azim != 1) return fail(RTROM_EINVAL, "n_azim must be 1 in 1D");
  if (d->dim == 2 && (d->n_azim < 4 || d->n_azim % 4 || d->n_azim > 256))
    return fail(RTROM_EINVAL, "n_azim must be a multiple of 4 in 4..256");
  if (d->method < 0 || d->method > 2) return fail(RTROM_EINVAL, "unknown method");
  if (d->precision < 0 || d->precision > 1) return fail(RTROM_EINVAL, "unknown precision");
  if (d->r_max < 1 || d->r_max > RT_RMAX) return fail(RTROM_EINVAL, "r_max must be in 1..20");
  if (!(d->eps_ig >= 0.0) || !(d->eps_pc >= 0.0) || !(d->eps_up >= 0.0))
    return fail(RTROM_EINVAL, "eps_ig, eps_pc, eps_up must be >= 0");
  if (!d->sigma_s || !d->sigma_a || !d->source) return fail(RTROM_EINVAL, "sigma_s, sigma_a, source required");
  const int64_t nc = (int64_t)d->nx * d->ny;
  for (int64_t i = 0; i < nc; ++i) {
    if (!(d->sigma_s[i] >= 0.0) || !std::isfinite(d->sigma_s[i]))
      return fail(RTROM_EINVAL, "sigma_s must be finite and >= 0");
    if (!(d->sigma_a[i] >= 0.0) || !std::isfinite(d->sigma_a[i]))
      return fail(RTROM_EINVAL, "sigma_a must be finite and >= 0");
    if (!std::isfinite(d->source[i])) return fail(RTROM_EINVAL, "source must be finite");
    if (d->f0 && !std::isfinite(d->f0[i])) return fail(RTROM_EINVAL, "f0 must be finite");
  }
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(d->inflow[k])) return fail(RTROM_EINVAL, "inflow must be finite");
  if (d->precond != RTROM_PC_DSA && d->precond != RTROM_PC_MH) return fail(RTROM_EINVAL, "unknown precond");
  if (d->time_scheme != RTROM_BE && d->time_scheme != RTROM_BDF2) return fail(RTROM_EINVAL, "unknown time_scheme");
  if (d->pc_levels < 0 || d->pc_levels > 4) return fail(RTROM_EINVAL, "pc_levels must be in 0..4");
  if (d->mh_rank < 0 || d->mh_rank > RT_RMAX) return fail(RTROM_EINVAL, "mh_rank must be in 0..20");
  if (!(d->lu_tol >= 0.0) || !std::isfinite(d->lu_tol)) return fail(RTROM_EINVAL, "lu_tol must be finite and >= 0");
  const bool variant = d->precond == RTROM_PC_MH || d->time_scheme == RTROM_BDF2;
  if (variant && d->dim == 1 && d->nx > RT_WAVE_MAX_CELLS)
    return fail(RTROM_EINVAL, "McClarren-Haut and BDF2 run on slabs of at most 2048 cells");
  if (d->pc_levels > 1 && d->dim == 1 && d->nx > RT_WAVE_MAX_CELLS)
    return fail(RTROM_EINVAL, "correction ROMs beyond the first iteration run on slabs of at most 2048 cells");
  if (d->scheme != RTROM_FV && d->scheme != RTROM_DG1) return fail(RTROM_EINVAL, "unknown scheme");
  if (d->scheme == RTROM_DG1) {
    if (d->dim != 1) return fail(RTROM_EINVAL, "the DG-P1 scheme runs on slabs only");
    if (d->nx > RT_DG_MAX_CELLS) return fail(RTROM_EINVAL, "DG-P1 slabs are limited to 1024 cells");
  }
  return RTROM_OK;
}

// unknowns of the scalar flux: cells, or two per cell for DG-P1
static size_t unknowns_of(const rtrom_problem_desc *d) {
  return (size_t)d->nx * d->ny * (d->scheme == RTROM_DG1 ? 2 : 1);
}

// ---------------------------------------------------------------------------
// Arena layout
// ---------------------------------------------------------------------------
namespace {
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

// Threads an instance's cells are split over: about eight cells per thread
// up to 2048 cells (at most 256 threads: short scans, and a batch of such
// instances fits two workgroups per CU), about four above (up to 1024
// threads); a multiple of 64.  Fixed per instance at creation, so its
// arithmetic does not depend on what it is batched with.
int slab_instance_threads(int nc) {
  const int cpt = nc <= 2048 ? 8 : 4;
  int nt = (nc + cpt - 1) / cpt;
  const char *env = std::getenv("RTROM_SLAB_CELLS_PER_THREAD");
  if (env && std::atoi(env) >= 1 && std::atoi(env) <= 8) nt = (nc + std::atoi(env) - 1) / std::atoi(env);
  nt = ((nt + 63) / 64) * 64;
  return std::max(64, std::min(1024, nt));
}

// Launch geometry of a fused launch over instances with the given thread
// counts: the block holds the largest instance; CMAX covers every chunk.
int slab_launch_threads(const int *nthr, const int *nc, int n, int *cmax) {
  int nt = 64, c = 1;
  for (int i = 0; i < n; ++i) {
    nt = std::max(nt, nthr[i]);
    c = std::max(c, (nc[i] + nthr[i] - 1) / nthr[i]);
  }
  *cmax = c <= 4 ? 4 : 8;
  return nt;  // cmax 8 only with nt <= 512: the caller splits batches that mix both
}
}  // namespace

// Certification factor of mixed precision: the FP32-refined iterate and its
// FP64 certification sweep must pass Alg. 1's stop test at theta * tol.  An
// FP64 run that stops at tol leaves an error anywhere between about the
// contraction factor times tol and tol itself (in the stop test's own
// measure), depending on how far below tol its last residual fell; the FP32
// loop instead stops as soon as its (rounded) residual drops below the
// threshold, which puts the accepted iterate at the top of that range, and
// the residual test sees the error of the slowly converging modes only
// damped by (1 - their eigenvalue), so what the FP32 increments leave there
// passes it and accumulates over the steps.  theta = 1/16 keeps mixed results
// within the distance the FP64 run keeps from the converged solution at every
// step of every tested march (1/8 did not: a 100-step batch march drifted to
// 1.2x that distance).  Overridden by RTROM_MIXED_CERT (a factor in (0, 1])
// for experiments.
double rt_mixed_cert_factor() {
  const char *env = std::getenv("RTROM_MIXED_CERT");
  if (env) {
    const double v = std::atof(env);
    if (v > 0.0 && v <= 1.0) return v;
  }
  return 0.0625;
}

// Pair groups of the cooperative slab SI: up to 16 workgroups, each sweeping
// pg consecutive ordinate pairs.  ng = 0: one workgroup (no cooperation).
static void slab_groups(const rtrom_problem_desc *d, int nv, int *ng, int *pg) {
  const int npair = nv / 2;
  *ng = 0;
  *pg = npair;
  if (d->dim != 1 || (d->flags & RTROM_F_SINGLE_WG) || npair < 2) return;
  // the variants and DG run in the one-workgroup kernels
  if (d->precond == RTROM_PC_MH || d->time_scheme == RTROM_BDF2 || d->pc_levels > 1 || d->scheme == RTROM_DG1)
    return;
  const int g = std::min(16, npair);
  *pg = (npair + g - 1) / g;
  *ng = (npair + *pg - 1) / *pg;
}

// Partial-sum rows of each ROM's projection passes: 2D instances use
// 256-cell blocks, the cooperative 1D passes blocks of 64 cells per wave pair
// (at least 64 cells).
static size_t part_rows(int dim, size_t nc) { return dim == 1 ? (nc + 63) / 64 : (nc + 255) / 256; }

static int mh_cap_of(const rtrom_problem_desc *d) { return d->mh_rank > 0 ? d->mh_rank : d->r_max; }

static size_t slab_bytes(const rtrom_problem_desc *d, int nv) {
  const size_t nc = unknowns_of(d);
  const size_t ld = (nc + 31) & ~size_t(31);
  Layout L;
  for (int k = 0; k < 13; ++k) L.take(nc * 8);
  L.take(5 * nc * 8);
  L.take((size_t)nv * 8 * 6);
  if (d->dim == 1) {  // 2D keeps its folded f in the plane buffers
    L.take((size_t)nv * nc * 8);
    L.take((size_t)(nv / 2) * nc * 8);
    if (d->time_scheme == RTROM_BDF2) {  // f^{n-1}, three DSA factor arrays
      L.take((size_t)nv * nc * 8);
      for (int k = 0; k < 3; ++k) L.take(nc * 8);
    }
  }
  if (d->time_scheme == RTROM_BDF2) L.take(nc * 8);  // sigma_t + 3/(2 dt)
  if (d->precond == RTROM_PC_MH) {  // Q, Z
    L.take((size_t)mh_cap_of(d) * ld * 8);
    L.take((size_t)mh_cap_of(d) * ld * 8);
  }
  if (d->dim == 1) {
    if (d->scheme == RTROM_DG1) L.take(12 * (size_t)d->nx * 8);  // block DSA factors
    if (d->scheme == RTROM_DG1 && d->time_scheme == RTROM_BDF2) L.take(12 * (size_t)d->nx * 8);  // of BDF2
    int ng, pg;
    slab_groups(d, nv, &ng, &pg);
    if (ng > 1) {
      L.take(2 * (size_t)ng * nc * 8);
      L.take(2 * (size_t)ng * nc * 4);
      L.take(2 * nc * 8);
      L.take(2 * nc * 4);
      L.take(2 * (size_t)ng * RT_RMAX * 8);
      L.take(8 * 8);
    }
  }
  const int nrom = 1 + std::max(1, (int)d->pc_levels);
  for (int r = 0; r < nrom; ++r) {
    L.take((RT_RMAX + 1) * ld * 8);
    L.take((RT_RMAX + 1) * ld * 8);
    L.take((RT_RMAX + 1) * 8);
    L.take(RT_RMAX * RT_RMAX * 8);
    L.take(RT_RMAX * RT_RMAX * 8);
    L.take(RT_RMAX * 4);
    L.take(sizeof(RomPend));
    L.take(sizeof(RomWork));
    L.take(3 * part_rows(d->dim, nc) * RT_NPART * 8);
  }
  for (int k = 0; k + 2 < nrom; ++k) {  // y_l, rho^{(l-1)}, the correction, three work rows
    for (int q = 0; q < 3; ++q) L.take(nc * 8);
    L.take(3 * nc * 8);
  }
  L.take(sizeof(RtState));
  L.take(sizeof(Inst));
  return L.off;
}

// b~ of the next step from the stored f (creation, a new inflow).  The kernel
// depends on the size only (the wave-per-pair f-pass up to RT_WAVE_MAX_CELLS
// cells), never on how the problem is marched later, so a problem batched
// and the same problem marched alone start from bitwise the same b~.
static hipError_t slab_rhs(rtrom_problem *p) {
  const Inst &I = p->hinst;
  if (p->nc <= RT_WAVE_MAX_CELLS)
    return rt_launch_slab_fpass_wave(p->dinst, 1, 1, I.dg ? (I.bdf2 ? 16 : 4) : (I.bdf2 ? 2 : 1), p->stream);
  int cmax;
  const int nt = slab_launch_threads(&I.nthr, &p->nc, 1, &cmax);
  return rt_launch_slab_rhs(p->dinst, 1, nt, cmax, I.npair, p->nc, p->stream);
}

extern "C" rtrom_status rtrom_estimate_bytes(const rtrom_problem_desc *d, uint64_t *bytes) {
  if (!d || !bytes) return fail(RTROM_EINVAL, "null argument");
  if (d->dim != 1 && d->dim != 2) return fail(RTROM_EINVAL, "dim must be 1 or 2");
  if (d->nx < 1 || d->ny < 1 || d->n_polar < 1 || d->n_azim < 1) return fail(RTROM_EINVAL, "bad sizes");
  int nv = d->dim == 1 ? d->n_polar : d->n_polar * d->n_azim;
  size_t b = slab_bytes(d, nv) + (d->dim == 2 ? rt_plane_extra_bytes(d) : 0) + 1024 * sizeof(RtStepRec);
  *bytes = b;
  return RTROM_OK;
}

static rtrom_status upload_inst(rtrom_problem *p) {
  RT_HIP(hipMemcpyAsync(p->dinst, &p->hinst, sizeof(Inst), hipMemcpyHostToDevice, p->stream), "upload descriptor");
  return RTROM_OK;
}

extern "C" void rtrom_destroy_problem(rtrom_problem *p) {
  if (!p) return;
  rt_log(2, "problem %d destroyed after %lld steps", p->id, (long long)p->steps);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->d.dim == 2) rt_plane_destroy(p);
  if (p->arena) (void)hipFree(p->arena);
  if (p->dhist) (void)hipFree(p->dhist);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->ev_si) (void)hipEventDestroy(p->ev_si);
  if (p->ev_rom) (void)hipEventDestroy(p->ev_rom);
  if (p->aux_stream) {
    (void)hipStreamSynchronize(p->aux_stream);
    (void)hipStreamDestroy(p->aux_stream);
  }
  if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
  delete p;
}

// Step history: grown geometrically, so a long march reallocates a handful
// of times at most.  Plain hipMalloc / hipFree only: no stream-ordered pool
// allocations anywhere in the library, so nothing is left in a pool tied to
// streams that problems destroy (served problems create and destroy theirs
// on worker threads).
static rtrom_status ensure_hist(rtrom_problem *p, int64_t need, hipStream_t s) {
  if (need <= p->hist_cap) return RTROM_OK;
  int64_t cap = std::max<int64_t>(need, std::max<int64_t>(1024, 2 * p->hist_cap));
  RtStepRec *nh = nullptr;
  if (hipMalloc((void **)&nh, cap * sizeof(RtStepRec)) != hipSuccess)
    return fail(RTROM_ENOMEM, "history allocation failed");
  RT_HIP(hipMemsetAsync(nh, 0, cap * sizeof(RtStepRec), s), "clear history");
  if (p->dhist && p->hist_cap > 0) {
    RT_HIP(hipMemcpyAsync(nh, p->dhist, p->hist_cap * sizeof(RtStepRec), hipMemcpyDeviceToDevice, s),
           "copy history");
    RT_HIP(hipStreamSynchronize(s), "history copy sync");
    RT_HIP(hipFree(p->dhist), "free history");
  }
  p->dhist = nh;
  p->hist_cap = cap;
  p->hinst.hist = nh;
  p->hinst.hist_cap = (int)std::min<int64_t>(cap, 0x7fffffff);
  RT_HIP(hipMemcpyAsync(p->dinst, &p->hinst, sizeof(Inst), hipMemcpyHostToDevice, s), "upload descriptor");
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_create_problem(const rtrom_problem_desc *d, rtrom_problem **out) {
  if (!out) return fail(RTROM_EINVAL, "null output handle");
  *out = nullptr;
  rtrom_status v = validate(d);
  if (v != RTROM_OK) return v;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(RTROM_EDEVICE, "no HIP device");
  rtrom_problem *p = new rtrom_problem();
  p->d = *d;
  p->d.sigma_s = p->d.sigma_a = p->d.source = p->d.f0 = nullptr;
  (void)hipGetDevice(&p->device);
  const int nc = (int)unknowns_of(d);  // == cells except for DG-P1
  const int ncell = d->nx * d->ny, ndof = nc / ncell;
  const int nv = d->dim == 1 ? d->n_polar : d->n_polar * d->n_azim;
  p->nc = nc;
  p->nv = nv;
  p->ox.assign(nv, 0.0);
  p->oy.assign(nv, 0.0);
  p->oz.assign(nv, 0.0);
  p->w.assign(nv, 0.0);
  if (d->dim == 1)
    rtrom_gauss_legendre(nv, p->ox.data(), p->w.data());
  else
    rtrom_cl_quadrature(d->n_azim, d->n_polar, p->ox.data(), p->oy.data(), p->oz.data(), p->w.data());

  auto bail = [&](rtrom_status s, const std::string &m) {
    rtrom_destroy_problem(p);
    return fail(s, m);
  };
  if (hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(RTROM_EDEVICE, "stream creation failed");
  p->stream = p->own_stream;
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
    return bail(RTROM_EDEVICE, "event creation failed");
  if (hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_si, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_rom, hipEventDisableTiming) != hipSuccess)
    return bail(RTROM_EDEVICE, "auxiliary stream creation failed");

  // --- arena ------------------------------------------------------------
  const size_t ld = ((size_t)nc + 31) & ~size_t(31);
  p->arena_bytes = slab_bytes(d, nv);
  if (hipMalloc(&p->arena, p->arena_bytes) != hipSuccess) return bail(RTROM_ENOMEM, "device allocation failed");
  if (hipMemsetAsync(p->arena, 0, p->arena_bytes, p->stream) != hipSuccess)
    return bail(RTROM_EDEVICE, "clear arena failed");
  Layout L;
  auto D = [&](size_t bytes) { return (double *)(p->arena + L.take(bytes)); };
  Inst &I = p->hinst;
  memset(&I, 0, sizeof(I));
  double *ss = D(nc * 8), *sa = D(nc * 8), *G = D(nc * 8), *ct = D(nc * 8);
  double *fe = D(nc * 8), *bg = D(nc * 8), *invd = D(nc * 8);
  I.rho = D(nc * 8);
  I.bt2[0] = D(nc * 8);
  I.bt2[1] = D(nc * 8);
  I.rho0 = D(nc * 8);
  I.rhalf = D(nc * 8);
  I.dpc = D(nc * 8);
  I.work = D(5 * (size_t)nc * 8);
  double *qbuf = D((size_t)nv * 8 * 6);
  I.f = d->dim == 1 ? D((size_t)nv * nc * 8) : nullptr;
  I.fpart = d->dim == 1 ? D((size_t)(nv / 2) * nc * 8) : nullptr;
  double *ctb = nullptr;
  if (d->time_scheme == RTROM_BDF2) {
    ctb = D(nc * 8);
    I.ct_b = ctb;
  }
  if (d->dim == 1 && d->time_scheme == RTROM_BDF2) {
    I.fb[0] = I.f;
    I.fb[1] = D((size_t)nv * nc * 8);
    I.dsa_fe_b = D(nc * 8);
    I.dsa_bg_b = D(nc * 8);
    I.dsa_invd_b = D(nc * 8);
  }
  if (d->precond == RTROM_PC_MH) {
    I.mh_cap = mh_cap_of(d);
    I.mhQ = D((size_t)I.mh_cap * ld * 8);
    I.mhZ = D((size_t)I.mh_cap * ld * 8);
  }
  if (d->dim == 1 && d->scheme == RTROM_DG1) I.dsa_blk = D(12 * (size_t)ncell * 8);
  if (d->dim == 1 && d->scheme == RTROM_DG1 && d->time_scheme == RTROM_BDF2) I.dsa_blk_b = D(12 * (size_t)ncell * 8);
  I.dg = d->scheme == RTROM_DG1;
  I.ncell = ncell;
  slab_groups(d, nv, &I.ng, &I.pg);
  if (I.ng > 1) {
    I.sip = D(2 * (size_t)I.ng * nc * 8);
    I.sip32 = (float *)D(2 * (size_t)I.ng * nc * 4);
    I.sips = D(2 * (size_t)nc * 8);
    I.sips32 = (float *)D(2 * (size_t)nc * 4);
    I.apx = D(2 * (size_t)I.ng * RT_RMAX * 8);
    I.bar = (unsigned long long *)D(8 * 8);
  }
  const int nrom = 1 + std::max(1, (int)d->pc_levels);
  RomDev *roms[2 + RT_XLEV] = {&I.ig, &I.pc, &I.pl[0], &I.pl[1], &I.pl[2]};
  static_assert(RT_XLEV == 3, "one RomDev pointer per level");
  RomWork rom_work_init[2 + RT_XLEV];
  for (int r = 0; r < nrom; ++r) {
    roms[r]->U = D((RT_RMAX + 1) * ld * 8);
    roms[r]->W = D((RT_RMAX + 1) * ld * 8);
    roms[r]->S = D((RT_RMAX + 1) * 8);
    roms[r]->M = D(RT_RMAX * RT_RMAX * 8);
    roms[r]->LU = D(RT_RMAX * RT_RMAX * 8);
    roms[r]->perm = (int *)D(RT_RMAX * 4);
    roms[r]->pend = (RomPend *)D(sizeof(RomPend));
    roms[r]->work = (RomWork *)D(sizeof(RomWork));
    roms[r]->lu_tol = d->lu_tol > 0.0 ? d->lu_tol : 1e-14;
    {
      const size_t nb = part_rows(d->dim, nc);
      double *parts = D(3 * nb * RT_NPART * 8);
      RomWork wk;
      memset(&wk, 0, sizeof(wk));
      wk.part1 = parts;
      wk.part2 = parts + nb * RT_NPART;
      wk.part3 = parts + 2 * nb * RT_NPART;
      rom_work_init[r] = wk;
    }
  }
  for (int k = 0; k + 2 < nrom; ++k) {
    I.ylev[k] = D(nc * 8);
    I.rlev[k] = D(nc * 8);
    I.dlev[k] = D(nc * 8);
    I.wlev[k] = D(3 * (size_t)nc * 8);
  }
  I.nlev = nrom - 1;
  I.st = (RtState *)D(sizeof(RtState));
  p->dinst = (Inst *)D(sizeof(Inst));

  I.dim = d->dim;
  I.nx = d->nx;
  I.ny = d->ny;
  I.nc = nc;
  I.nv = nv;
  I.npair = nv / 2;
  I.post_fused = d->dim == 1 && nc <= RT_POST_FUSED_NC;
  I.post_nb = I.post_fused ? 1 : rt_pass_blocks(nc);
  I.max_iter = d->max_iter;
  I.method = d->method;
  I.precision = d->precision;
  I.r_max = d->r_max;
  I.abs_up = (d->flags & RTROM_F_ABS_UP_NORM) ? 1 : 0;
  I.ld = (int)ld;
  I.nthr = d->dim == 1 ? slab_instance_threads(nc) : 256;
  if (I.ng > 1) {  // the pair-group kernels need all their workgroups resident at once
    int cmax;
    const int nt = slab_launch_threads(&I.nthr, &nc, 1, &cmax);
    if (!rt_slab_coop_fits(p->device, I.ng, nt, cmax, I.npair, nc)) I.ng = 0;
  }
  I.hx = d->lx / d->nx;
  I.hy = d->dim == 2 ? d->ly / d->ny : 1.0;
  I.dt = d->dt;
  I.inv_dt = 1.0 / d->dt;
  I.tol = d->tol;
  {
    const double theta = d->precision == RTROM_MIXED ? rt_mixed_cert_factor() : 1.0;
    I.tol_cert = theta * d->tol;
    I.tol32 = theta * d->tol;
  }
  I.eps_ig = d->eps_ig;
  I.eps_pc = d->eps_pc;
  I.eps_up = d->eps_up;
  I.precond = d->precond;
  I.bdf2 = d->time_scheme == RTROM_BDF2;
  I.adt_b = 1.5 / d->dt;
  for (int k = 0; k < 4; ++k) I.g[k] = d->inflow[k];
  I.ss = ss;
  I.sa = sa;
  I.G = G;
  I.ct = ct;
  I.dsa_fe = fe;
  I.dsa_bg = bg;
  I.dsa_invd = invd;

  // --- host-side staging of per-cell and per-ordinate data ----------------
  // per unknown: the cell's value (DG-P1: both unknowns; the source and f0
  // are constant on the cell, so their slope unknowns are zero)
  std::vector<double> h_ss(nc), h_sa(nc), h_G(nc), h_ct(nc), h_q((size_t)nv * 6, 0.0);
  for (int u = 0; u < nc; ++u) {
    const int i = u / ndof;
    h_ss[u] = d->sigma_s[i];
    h_sa[u] = d->sigma_a[i];
    h_G[u] = u % ndof == 0 ? d->source[i] : 0.0;
    h_ct[u] = d->sigma_s[i] + d->sigma_a[i] + 1.0 / d->dt;
  }
  if (d->dim == 1) {
    // ordinates sorted ascending: pair p = (p, nv-1-p) are mirrors
    for (int q = 0; q < nv / 2; ++q) {
      h_q[q] = std::fabs(p->ox[q]) / I.hx;
      h_q[nv + q] = p->w[q];
    }
    I.pm = qbuf;
    I.pw = qbuf + nv;
  }
  auto H2D = [&](void *dst, const void *src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, p->stream) == hipSuccess;
  };
  bool ok = H2D(ss, h_ss.data(), nc * 8) && H2D(sa, h_sa.data(), nc * 8) && H2D(G, h_G.data(), nc * 8) &&
            H2D(ct, h_ct.data(), nc * 8) && H2D(qbuf, h_q.data(), h_q.size() * 8);
  std::vector<double> h_ctb;
  if (ctb) {  // the BDF2 operator: sigma_t + 3 / (2 dt)
    h_ctb.resize(nc);
    for (int u = 0; u < nc; ++u) h_ctb[u] = h_ss[u] + h_sa[u] + 1.5 / d->dt;
    ok = ok && H2D(ctb, h_ctb.data(), nc * 8);
  }
  std::vector<double> rho0(nc, 0.0);
  if (d->f0)
    for (int u = 0; u < nc; u += ndof) rho0[u] = d->f0[u / ndof];
  ok = ok && H2D(I.rho, rho0.data(), nc * 8);
  if (d->f0)
    for (int j = 0; j < nv && ok && d->dim == 1; ++j) ok = H2D(I.f + (size_t)j * nc, rho0.data(), nc * 8);
  // initial phase-machine state: everything zero, Phase I ahead
  RtState st0;
  memset(&st0, 0, sizeof(st0));
  st0.phase = 1;
  ok = ok && H2D(I.st, &st0, sizeof(st0));
  for (int r = 0; r < nrom && ok; ++r) ok = H2D(roms[r]->work, &rom_work_init[r], sizeof(RomWork));
  if (!ok) return bail(RTROM_EDEVICE, "upload failed");
  if (ensure_hist(p, 1024, p->stream) != RTROM_OK) {
    std::string m = g_err;
    return bail(RTROM_ENOMEM, m);
  }
  if (d->dim == 1) {
    if (upload_inst(p) != RTROM_OK) return bail(RTROM_EDEVICE, "upload descriptor failed");
    for (int alt = 0; alt <= (I.bdf2 ? 1 : 0); ++alt) {  // alt: the BDF2 operator's factors
      const hipError_t e = I.dg ? rt_launch_setup_dsa_dg(p->dinst, 1, alt, p->stream)
                                : rt_launch_slab_setup(p->dinst, 1, nc, alt, p->stream);
      if (e != hipSuccess) return bail(RTROM_EDEVICE, "setup launch failed");
    }
    if (slab_rhs(p) != hipSuccess) return bail(RTROM_EDEVICE, "initial RHS launch failed");
  } else {
    if (upload_inst(p) != RTROM_OK) return bail(RTROM_EDEVICE, "upload descriptor failed");
    int s = rt_plane_create(p);
    if (s != RTROM_OK) {
      std::string m = g_err;
      return bail((rtrom_status)s, m);
    }
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return bail(RTROM_EDEVICE, "create sync failed");
  p->id = g_next_id.fetch_add(1);
  if (rt_log_level() >= 2) {
    static const char *methods[] = {"si_dsa", "rom", "si"};  // rtrom_method order
    rt_log(2, "problem %d created: %dD, %d x %d cells, %d ordinates, %s, %s precision, %s, %s, %s, %.1f MiB",
           p->id, d->dim, d->nx, d->dim == 2 ? d->ny : 1, p->nv,
           methods[std::min(2, std::max(0, (int)d->method))], d->precision == RTROM_FP64 ? "fp64" : "mixed",
           d->precond == RTROM_PC_MH ? "McClarren-Haut" : "DSA", d->time_scheme == RTROM_BDF2 ? "BDF2" : "BE",
           d->scheme == RTROM_DG1 ? "DG-P1" : "FV", (double)(p->arena_bytes + (d->dim == 2 ? rt_plane_extra_bytes(d) : 0)) / (1 << 20));
  }
  *out = p;
  return RTROM_OK;
}

// ---------------------------------------------------------------------------
// Marching
// ---------------------------------------------------------------------------
static rtrom_status read_state(const rtrom_problem *p, RtState *st) {
  RT_HIP(hipMemcpyAsync(st, p->hinst.st, sizeof(RtState), hipMemcpyDeviceToHost, p->stream), "read state");
  RT_HIP(hipStreamSynchronize(p->stream), "state sync");
  return RTROM_OK;
}

// Device scratch of the allocation-free batch march: the batch's descriptor
// table and the gathered per-instance states, in a file-scope device array
// (one copy per device, held until the process ends).  Host code never
// passes the array's name to a kernel or a copy: it takes the array's device
// address from hipGetSymbolAddress once per device and uses that.
#define RT_NOALLOC_BYTES (RTROM_NOALLOC_MAX_BATCH * (sizeof(Inst) + sizeof(RtState)) + 512)
static __device__ __align__(256) unsigned char scratch[RT_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

// The scratch array's device address on `device` (the current device).
static rtrom_status scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return fail(RTROM_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RTROM_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return RTROM_OK;
}

// noalloc: take the descriptor table and states from the device scratch array
// instead of allocating them, and never grow a step history.
static rtrom_status march_one_kind(rtrom_problem *const *ps_in, int n, int nsteps, bool noalloc = false) {
  const RtRange range(n == 1 ? "rtrom_march" : "rtrom_march_batch");
  // all handles of one dimension; 1D: fused launches over the instance array.
  // A 1D batch is laid out largest first (cells x ordinate pairs): workgroups
  // are dispatched in instance order, so the longest ones start first and
  // the launches' tails shorten.  Every instance computes the same thing
  // wherever it sits.
  // Instances of more than RT_WAVE_MAX_CELLS cells come first: they run the
  // kernels with cells split over the threads in contiguous runs, the others
  // the kernels with ordinate pairs spread over waves, as two launches.
  std::vector<rtrom_problem *> order(ps_in, ps_in + n);
  if (n > 1 && ps_in[0]->d.dim == 1)
    std::stable_sort(order.begin(), order.end(), [](const rtrom_problem *a, const rtrom_problem *b) {
      const bool wa = a->nc > RT_WAVE_MAX_CELLS, wb = b->nc > RT_WAVE_MAX_CELLS;
      if (wa != wb) return wa;
      return (long long)a->nc * a->hinst.npair > (long long)b->nc * b->hinst.npair;
    });
  rtrom_problem *const *ps = order.data();
  hipStream_t s = ps[0]->stream;
  for (int i = 0; i < n; ++i)
    if (ps[i]->stream != s) RT_HIP(hipStreamSynchronize(ps[i]->stream), "sync member stream");
  for (int i = 0; i < n; ++i) {
    if (noalloc) {
      if (ps[i]->steps + nsteps > ps[i]->hist_cap)
        return fail(RTROM_EINVAL, "march_batch_noalloc: the march would outgrow a problem's step history "
                                  "(capacity " + std::to_string(ps[i]->hist_cap) + " steps); it never allocates");
      continue;
    }
    rtrom_status e = ensure_hist(ps[i], ps[i]->steps + nsteps, s);
    if (e != RTROM_OK) return e;
  }
  // descriptor uploads of grown histories went on s; members may launch on
  // their own streams
  RT_HIP(hipStreamSynchronize(s), "history sync");
  // phase-machine states before the march (for the non-convergence count)
  std::vector<RtState> before(n);
  Inst *dinsts = nullptr;
  RtState *dstates = nullptr;
  // batch descriptor and state buffers, released on every return path (after
  // the stream has drained on the normal one)
  struct BatchBufs {
    hipStream_t s;
    void *a = nullptr, *b = nullptr;
    ~BatchBufs() {
      if (a || b) (void)hipStreamSynchronize(s);
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
    }
  } bufs{s};
  if (ps[0]->d.dim == 1 && n > 1) {
    std::vector<Inst> h(n);
    for (int i = 0; i < n; ++i) h[i] = ps[i]->hinst;
    if (noalloc) {
      void *base = nullptr;
      rtrom_status e = scratch_address(ps[0]->device, &base);
      if (e != RTROM_OK) return e;
      dinsts = (Inst *)base;
      dstates = (RtState *)((char *)base + (((size_t)n * sizeof(Inst) + 255) & ~size_t(255)));
    } else {
      if (hipMalloc((void **)&dinsts, n * sizeof(Inst)) != hipSuccess)
        return fail(RTROM_ENOMEM, "batch descriptor allocation failed");
      bufs.a = dinsts;
      if (hipMalloc((void **)&dstates, n * sizeof(RtState)) != hipSuccess)
        return fail(RTROM_ENOMEM, "batch states allocation failed");
      bufs.b = dstates;
    }
    RT_HIP(hipMemcpyAsync(dinsts, h.data(), n * sizeof(Inst), hipMemcpyHostToDevice, s), "upload batch");
    RT_HIP(rt_launch_gather_states(dinsts, n, dstates, s), "gather states");
    RT_HIP(hipMemcpyAsync(before.data(), dstates, n * sizeof(RtState), hipMemcpyDeviceToHost, s), "read states");
    RT_HIP(hipStreamSynchronize(s), "state sync");
  } else {
    for (int i = 0; i < n; ++i) {
      rtrom_status e = read_state(ps[i], &before[i]);
      if (e != RTROM_OK) return e;
    }
  }
  RT_HIP(hipEventRecord(ps[0]->ev0, s), "event");
  if (ps[0]->d.dim == 1) {
    std::vector<int> nthr(n), ncs(n);
    for (int i = 0; i < n; ++i) {
      nthr[i] = ps[i]->hinst.nthr;
      ncs[i] = ps[i]->nc;
    }
    if (n == 1) dinsts = ps[0]->dinst;
    // launch groups: [0, nA) instances of more than RT_WAVE_MAX_CELLS cells
    // (contiguous-run kernels), [nA, n) the rest (wave-per-pair kernels)
    int nA = 0;
    while (nA < n && ncs[nA] > RT_WAVE_MAX_CELLS) ++nA;
    struct Group {
      int off, cnt, nt, cmax, nc_max, npair_max, pairs_total, wave;
      int si_kinds, fp_kinds;  // wave kernels: bit 0 default instances, bit 1 variants (MH; BDF2), bit 2 DG,
                               // bit 3 DG with McClarren-Haut (SI only), bit 4 DG with BDF2 (f-pass only)
    };
    std::vector<Group> groups;
    for (int g = 0; g < 2; ++g) {
      Group G{g ? nA : 0, g ? n - nA : nA, 0, 0, 0, 1, 0, g, 0, 0};
      if (G.cnt == 0) continue;
      G.nt = slab_launch_threads(nthr.data() + G.off, ncs.data() + G.off, G.cnt, &G.cmax);
      for (int i = G.off; i < G.off + G.cnt; ++i) {
        G.nc_max = std::max(G.nc_max, ncs[i]);
        G.npair_max = std::max(G.npair_max, ps[i]->hinst.npair);
        G.pairs_total += ps[i]->hinst.npair;
        const bool mh = ps[i]->hinst.precond == RT_PC_MH;
        G.si_kinds |= ps[i]->hinst.dg ? (mh ? 8 : 4) : (mh ? 2 : 1);
        G.fp_kinds |= ps[i]->hinst.dg ? (ps[i]->hinst.bdf2 ? 16 : 4) : (ps[i]->hinst.bdf2 ? 2 : 1);
      }
      groups.push_back(G);
    }
    const int nt = groups[0].nt, cmax = groups[0].cmax;  // a problem marched alone: one group
    int any_rom = 0, any_fused = 0, nc_grid = 0, nrom = 2;
    for (int i = 0; i < n; ++i) {
      const int rom_i = ps[i]->d.method == RTROM_ROM_SI_DSA;
      any_rom |= rom_i;
      if (rom_i) nrom = std::max(nrom, 1 + ps[i]->hinst.nlev);
      if (rom_i && ps[i]->hinst.post_fused) any_fused = 1;
      if (rom_i && !ps[i]->hinst.post_fused) nc_grid = std::max(nc_grid, ncs[i]);
    }
    // Per step: SI solve (which also takes the step's ROM decisions), then
    // the f-pass (main stream) and the ROM work (auxiliary stream) run
    // concurrently -- they touch disjoint state: the f-pass writes f^n and the
    // other b~ buffer, the ROM work reads rho's and b~^{n-1} -- and the next
    // SI solve waits for both.
    hipStream_t s2 = any_rom ? ps[0]->aux_stream : s;
    // A problem marched on its own with pair groups runs each step as two
    // cooperative launches: the SI solve with the ROM decisions and
    // projection passes, then everything else (cores alongside the f-pass,
    // LU alongside the rotation and b~).
    const bool coop = n == 1 && ps[0]->hinst.ng > 1;
    for (int k = 0; k < nsteps && coop; ++k) {
      rt_prof_begin(RT_K_SLAB_SI, s);
      RT_HIP(rt_launch_slab_si_coop(dinsts, ps[0]->hinst.ng, nt, cmax, s), "cooperative SI launch");
      rt_prof_end(RT_K_SLAB_SI, s);
      rt_prof_begin(RT_K_POST, s);
      RT_HIP(rt_launch_slab_tail_coop(dinsts, ps[0]->hinst.npair, ps[0]->nc, nt, cmax, s), "cooperative tail launch");
      rt_prof_end(RT_K_POST, s);
    }
    // one step's launches on s (SI solve, f-pass) and s2 (ROM post), joined
    // by events; every kernel takes its step from the device state, so the
    // sequence is the same each step
    auto enqueue_step = [&]() -> rtrom_status {
      rt_prof_begin(RT_K_SLAB_SI, s);
      for (const Group &G : groups) {
        if (G.wave) RT_HIP(rt_launch_slab_si_wave(dinsts + G.off, G.cnt, G.si_kinds, s), "SI launch");
        else RT_HIP(rt_launch_slab_si(dinsts + G.off, G.cnt, G.nt, G.cmax, s), "SI launch");
      }
      rt_prof_end(RT_K_SLAB_SI, s);
      if (s2 != s) {
        RT_HIP(hipEventRecord(ps[0]->ev_si, s), "event");
        RT_HIP(hipStreamWaitEvent(s2, ps[0]->ev_si, 0), "event wait");
      }
      if (any_rom) {
        rt_prof_begin(RT_K_POST, s2);
        RT_HIP(rt_launch_rom_slab(dinsts, n, any_fused, nc_grid, nrom, s2), "ROM launch");
        rt_prof_end(RT_K_POST, s2);
        if (nc_grid > 0) {  // instances without a fused post
          rt_prof_begin(RT_K_ROM_UPDATE, s2);
          RT_HIP(rt_launch_rom_update(dinsts, n, nc_grid, 2, s2), "ROM update launch");
          rt_prof_end(RT_K_ROM_UPDATE, s2);
        }
      }
      rt_prof_begin(RT_K_SLAB_FPASS, s);
      for (const Group &G : groups) {
        if (G.wave) RT_HIP(rt_launch_slab_fpass_wave(dinsts + G.off, G.cnt, 0, G.fp_kinds, s), "f-pass launch");
        else
          RT_HIP(rt_launch_slab_fpass(dinsts + G.off, G.cnt, G.nt, G.cmax, G.npair_max, G.nc_max, G.pairs_total, s),
                 "f-pass launch");
      }
      rt_prof_end(RT_K_SLAB_FPASS, s);
      if (s2 != s) {
        RT_HIP(hipEventRecord(ps[0]->ev_rom, s2), "event");
        RT_HIP(hipStreamWaitEvent(s, ps[0]->ev_rom, 0), "event wait");
      }
      return RTROM_OK;
    };
    // A march of several steps captures one step in a HIP graph and replays
    // it: the per-step launch cost is paid once per march (kernel timing
    // brackets every launch with events, so it runs the steps eagerly).
    // RTROM_GRAPH=0 keeps eager launches; a capture the runtime refuses falls
    // back to them as well, and so does the allocation-free march (building
    // a graph allocates).
    const char *genv = std::getenv("RTROM_GRAPH");
    bool graph_done = false;
    if (!coop && !noalloc && nsteps >= 2 && !rt_prof_on() && !(genv && std::atoi(genv) == 0)) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const rtrom_status es = enqueue_step();
        ok = hipStreamEndCapture(s, &graph) == hipSuccess && es == RTROM_OK && graph;
      }
      ok = ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      (void)hipGetLastError();  // a refused capture leaves the steps to the eager loop
      if (ok) {
        bool launched = true;
        for (int k = 0; k < nsteps && launched; ++k) launched = hipGraphLaunch(exec, s) == hipSuccess;
        const bool synced = hipStreamSynchronize(s) == hipSuccess;
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (!launched || !synced) return fail(RTROM_EDEVICE, "step graph launch failed");
        graph_done = true;
      } else {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
      }
    }
    for (int k = 0; k < nsteps && !coop && !graph_done; ++k) {
      const rtrom_status es = enqueue_step();
      if (es != RTROM_OK) return es;
    }
  } else if (n == 1) {
    int e = rt_plane_step(ps[0], nsteps);
    if (e != RTROM_OK) return (rtrom_status)e;
  } else {
    // 2D batch: every problem marches on its own streams, from up to eight
    // host threads at once, so the members' kernels overlap on the device
    // (each 2D step's loop is steered from the host by its residual norms).
    // A problem's arithmetic does not depend on what runs beside it.
    const int nt = std::min(n, 8);
    std::vector<int> errs(nt, RTROM_OK);
    std::vector<std::string> msgs(nt);
    std::vector<std::thread> pool;
    const int dev = ps[0]->device;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t] {
        if (hipSetDevice(dev) != hipSuccess) {
          errs[t] = RTROM_EDEVICE;
          msgs[t] = "cannot select the device";
          return;
        }
        for (int i = t; i < n && errs[t] == RTROM_OK; i += nt) {
          const int e = rt_plane_step(ps[i], nsteps);
          if (e != RTROM_OK) {
            errs[t] = e;
            msgs[t] = g_err;  // thread-local message of the worker
          }
        }
        if (errs[t] == RTROM_OK) {
          for (int i = t; i < n; i += nt)
            if (hipStreamSynchronize(ps[i]->stream) != hipSuccess) {
              errs[t] = RTROM_EDEVICE;
              msgs[t] = "member stream sync failed";
            }
        }
      });
    for (auto &th : pool) th.join();
    for (int t = 0; t < nt; ++t)
      if (errs[t] != RTROM_OK) return fail((rtrom_status)errs[t], msgs[t]);
  }
  RT_HIP(hipEventRecord(ps[0]->ev1, s), "event");
  RT_HIP(hipStreamSynchronize(s), "march sync");
  rt_prof_collect();
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, ps[0]->ev0, ps[0]->ev1);
  std::vector<RtState> after(n);
  if (dstates) {
    RT_HIP(rt_launch_gather_states(dinsts, n, dstates, s), "gather states");
    RT_HIP(hipMemcpyAsync(after.data(), dstates, n * sizeof(RtState), hipMemcpyDeviceToHost, s), "read states");
    RT_HIP(hipStreamSynchronize(s), "state sync");
  } else {
    for (int i = 0; i < n; ++i) {
      rtrom_status e = read_state(ps[i], &after[i]);
      if (e != RTROM_OK) return e;
    }
  }
  rtrom_status res = RTROM_OK;
  for (int i = 0; i < n; ++i) {
    ps[i]->steps += nsteps;
    ps[i]->t_total += ms * 1e-3 / n;
    if (after[i].nonconv != before[i].nonconv) res = RTROM_ENOCONV;
    if (after[i].fault) {
      rt_set_error("a cooperative grid barrier timed out; the problem's state is invalid");
      return RTROM_EDEVICE;
    }
  }
  // diagnostics: ROM phase changes (roctx marks, RTROM_LOG >= 2) and one
  // line per step (RTROM_LOG >= 3)
  for (int i = 0; i < n; ++i) {
    if (after[i].phase != before[i].phase) {
      char msg[160];
      std::snprintf(msg, sizeof(msg), "problem %d: ROM phase %d -> %d within steps %lld..%lld (N0 %d, N1 %d)",
                    ps[i]->id, before[i].phase, after[i].phase, (long long)(ps[i]->steps - nsteps + 1),
                    (long long)ps[i]->steps, after[i].n0, after[i].n1);
      rt_mark(msg);
      rt_log(2, "%s", msg);
    }
    if (rt_log_level() >= 3 && ps[i]->steps <= ps[i]->hist_cap) {
      std::vector<RtStepRec> rec(nsteps);
      RT_HIP(hipMemcpy(rec.data(), ps[i]->dhist + (ps[i]->steps - nsteps), nsteps * sizeof(RtStepRec),
                       hipMemcpyDeviceToHost), "read step records");
      for (int k = 0; k < nsteps; ++k)
        rt_log(3, "problem %d step %lld: %d sweeps, phase %d, %s, residual %.3e, ranks %d / %d%s", ps[i]->id,
               (long long)(ps[i]->steps - nsteps + k + 1), rec[k].iters, rec[k].phase,
               rec[k].converged ? "converged" : "NOT converged", rec[k].residual, rec[k].rank_ig, rec[k].rank_pc,
               rec[k].fallback ? ", ROM fallback" : "");
    }
  }
  if (res == RTROM_ENOCONV) rt_set_error("a time step reached max_iter without meeting the tolerance");
  return res;
}

extern "C" rtrom_status rtrom_march(rtrom_problem *p, int32_t nsteps) {
  if (!p) return fail(RTROM_EINVAL, "null problem");
  if (nsteps < 0) return fail(RTROM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return RTROM_OK;
  return march_one_kind(&p, 1, nsteps);
}

extern "C" rtrom_status rtrom_step(rtrom_problem *p) { return rtrom_march(p, 1); }

static rtrom_status check_batch(rtrom_problem *const *ps, int32_t n, int32_t nsteps) {
  if (!ps || n < 1) return fail(RTROM_EINVAL, "need at least one problem");
  if (nsteps < 0) return fail(RTROM_EINVAL, "nsteps must be >= 0");
  for (int i = 0; i < n; ++i) {
    if (!ps[i]) return fail(RTROM_EINVAL, "null problem in batch");
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) return fail(RTROM_EINVAL, "duplicate problem in batch");
    if (ps[i]->d.dim != ps[0]->d.dim) return fail(RTROM_EINVAL, "batch mixes 1D and 2D problems");
    if (ps[i]->device != ps[0]->device) return fail(RTROM_EINVAL, "batch spans devices");
  }
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_march_batch_noalloc(rtrom_problem *const *ps, int32_t n, int32_t nsteps) {
  rtrom_status v = check_batch(ps, n, nsteps);
  if (v != RTROM_OK) return v;
  if (n > RTROM_NOALLOC_MAX_BATCH)
    return fail(RTROM_EINVAL, "march_batch_noalloc: at most " + std::to_string(RTROM_NOALLOC_MAX_BATCH) +
                                  " problems per call");
  if (nsteps == 0) return RTROM_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(RTROM_EDEVICE, "no current device");
  if (cur != ps[0]->device && hipSetDevice(ps[0]->device) != hipSuccess)
    return fail(RTROM_EDEVICE, "cannot select the problems' device");
  rtrom_status r = march_one_kind(ps, n, nsteps, true);
  if (cur != ps[0]->device) (void)hipSetDevice(cur);
  return r;
}

extern "C" rtrom_status rtrom_march_batch(rtrom_problem *const *ps, int32_t n, int32_t nsteps) {
  if (!ps || n < 1) return fail(RTROM_EINVAL, "need at least one problem");
  if (nsteps < 0) return fail(RTROM_EINVAL, "nsteps must be >= 0");
  for (int i = 0; i < n; ++i) {
    if (!ps[i]) return fail(RTROM_EINVAL, "null problem in batch");
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) return fail(RTROM_EINVAL, "duplicate problem in batch");
    if (ps[i]->d.dim != ps[0]->d.dim) return fail(RTROM_EINVAL, "batch mixes 1D and 2D problems");
    if (ps[i]->device != ps[0]->device) return fail(RTROM_EINVAL, "batch spans devices");
  }
  if (nsteps == 0) return RTROM_OK;
  return march_one_kind(ps, n, nsteps);
}

// ---------------------------------------------------------------------------
// Accessors
// ---------------------------------------------------------------------------
static rtrom_status d2h(const rtrom_problem *p, void *dst, const void *src, size_t bytes) {
  RT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, p->stream), "download");
  RT_HIP(hipStreamSynchronize(p->stream), "download sync");
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_get_scalar_flux(const rtrom_problem *p, double *rho, int64_t n) {
  if (!p || !rho) return fail(RTROM_EINVAL, "null argument");
  if (n < p->nc) return fail(RTROM_EINVAL, "output buffer too small");
  return d2h(p, rho, p->hinst.rho, (size_t)p->nc * 8);
}

extern "C" rtrom_status rtrom_get_rhs(const rtrom_problem *p, double *b, int64_t n) {
  if (!p || !b) return fail(RTROM_EINVAL, "null argument");
  if (n < p->nc) return fail(RTROM_EINVAL, "output buffer too small");
  return d2h(p, b, p->hinst.bt2[p->steps & 1], (size_t)p->nc * 8);
}

extern "C" rtrom_status rtrom_get_angular_flux(const rtrom_problem *p, double *f, int64_t n) {
  if (!p || !f) return fail(RTROM_EINVAL, "null argument");
  if (n < (int64_t)p->nc * p->nv) return fail(RTROM_EINVAL, "output buffer too small");
  if (p->d.dim == 2) return (rtrom_status)rt_plane_unfold(p, f);
  const double *src = p->hinst.bdf2 ? p->hinst.fb[p->steps & 1] : p->hinst.f;  // BDF2: f^n in fb[n & 1]
  return d2h(p, f, src, (size_t)p->nc * p->nv * 8);
}

extern "C" rtrom_status rtrom_get_quadrature(const rtrom_problem *p, double *ox, double *oy, double *oz,
                                             double *w, int64_t n) {
  if (!p || !ox || !w) return fail(RTROM_EINVAL, "null argument");
  if (n < p->nv) return fail(RTROM_EINVAL, "output buffer too small");
  memcpy(ox, p->ox.data(), p->nv * 8);
  memcpy(w, p->w.data(), p->nv * 8);
  if (oy) memcpy(oy, p->oy.data(), p->nv * 8);
  if (oz) memcpy(oz, p->oz.data(), p->nv * 8);
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_stats_get(const rtrom_problem *p, rtrom_stats *out) {
  if (!p || !out) return fail(RTROM_EINVAL, "null argument");
  RtState st;
  rtrom_status e = read_state(p, &st);
  if (e != RTROM_OK) return e;
  memset(out, 0, sizeof(*out));
  out->steps = st.steps;
  out->si_iters_total = st.si_total;
  out->sweeps_total = st.sweeps_total;
  out->si_iters_last = st.iters;
  out->phase = !st.flag_ig ? 1 : (!st.flag_pc ? 2 : 3);
  for (int k = 0; k + 2 <= p->hinst.nlev; ++k) out->phase += (out->phase == k + 3 && st.flag_pl[k]) ? 1 : 0;
  out->n0 = st.n0;
  out->n1 = st.n1;
  out->rank_ig = st.rank_ig;
  out->rank_pc = st.rank_pc;
  out->nonconverged_steps = st.nonconv;
  out->rom_fallbacks = st.fallbacks;
  out->ig_updates = st.ig_updates;
  out->pc_updates = st.pc_updates;
  out->fp32_sweeps = st.fp32_sweeps;
  out->last_residual = st.residual;
  out->t_total_s = p->t_total;
  out->dsa_iters = p->d.dim == 2 ? rt_plane_dsa_iters(p) : 0;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_get_levels(const rtrom_problem *p, int64_t *out, int32_t n, int32_t *levels) {
  if (!p || !out || !levels) return fail(RTROM_EINVAL, "null argument");
  const int L = std::max(1, p->hinst.nlev);
  if (n < 4 * L) return fail(RTROM_EINVAL, "output buffer too small");
  RtState st;
  rtrom_status e = read_state(p, &st);
  if (e != RTROM_OK) return e;
  for (int l = 1; l <= L; ++l) {
    int64_t *o = out + 4 * (l - 1);
    if (l == 1) {
      o[0] = st.flag_pc;
      o[1] = st.n1;
      o[2] = st.rank_pc;
      o[3] = st.pc_updates;
    } else {
      o[0] = st.flag_pl[l - 2];
      o[1] = st.n_pl[l - 2];
      o[2] = st.rank_pl[l - 2];
      o[3] = st.upd_pl[l - 2];
    }
  }
  *levels = L;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_get_history(const rtrom_problem *p, rtrom_step_record *out, int64_t n,
                                          int64_t *written) {
  if (!p || !out || n < 0) return fail(RTROM_EINVAL, "bad argument");
  int64_t m = std::min<int64_t>(n, std::min<int64_t>(p->steps, p->hist_cap));
  int64_t first = std::min<int64_t>(p->steps, p->hist_cap) - m;
  static_assert(sizeof(rtrom_step_record) == sizeof(RtStepRec), "record layout");
  if (m > 0) {
    rtrom_status e = d2h(p, out, p->dhist + first, (size_t)m * sizeof(RtStepRec));
    if (e != RTROM_OK) return e;
  }
  if (written) *written = m;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_set_inflow(rtrom_problem *p, const double *g) {
  if (!p || !g) return fail(RTROM_EINVAL, "null argument");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(g[k])) return fail(RTROM_EINVAL, "inflow must be finite");
  for (int k = 0; k < 4; ++k) {
    p->d.inflow[k] = g[k];
    p->hinst.g[k] = g[k];
  }
  rtrom_status e = upload_inst(p);
  if (e != RTROM_OK) return e;
  if (p->d.dim == 1) {
    RT_HIP(slab_rhs(p), "RHS launch");
  } else {
    int s = rt_plane_rhs(p);
    if (s != RTROM_OK) return (rtrom_status)s;
  }
  RT_HIP(hipStreamSynchronize(p->stream), "inflow sync");
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_set_stream(rtrom_problem *p, void *hip_stream) {
  if (!p) return fail(RTROM_EINVAL, "null problem");
  RT_HIP(hipStreamSynchronize(p->stream), "stream switch sync");
  p->stream = hip_stream ? (hipStream_t)hip_stream : p->own_stream;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_device_bytes(const rtrom_problem *p, uint64_t *bytes) {
  if (!p || !bytes) return fail(RTROM_EINVAL, "null argument");
  *bytes = p->arena_bytes + (uint64_t)p->hist_cap * sizeof(RtStepRec) +
           (p->d.dim == 2 ? rt_plane_extra_bytes(&p->d) : 0);
  return RTROM_OK;
}
