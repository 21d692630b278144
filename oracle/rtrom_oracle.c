/*
 * rtrom_oracle.c -- plain, slow, FP64 CPU oracle for on-the-fly ROM-accelerated
 * SI-DSA (Liu & Peng, "On-the-Fly ROM-Based Acceleration of SI-DSA for Implicit
 * Time Marching of the Radiative Transfer Equation", arXiv 2603.19647).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * Everything here is written from the paper's equations and algorithms, in
 * their order, single threaded, with true divisions and no blocking or fusion:
 *   - S_N discrete ordinates, weights summing to one (Sec. 2.1, eq. rte discrete)
 *   - Gauss-Legendre (1D slab) and Chebyshev-Legendre CL(N_phi, N_z) (App. A)
 *   - backward Euler (Sec. 2.1, eq. time_discrete)
 *   - upwind DG with the K = 0 (piecewise constant) space, i.e. first-order
 *     upwind finite volume (Sec. 2.1, eq. DG with the upwind flux H-hat)
 *   - memory-efficient SI-SA on rho only (Sec. 2.3, eq. implicit_linear_system_rho,
 *     eq. SI_rho, Alg. 1), DSA correction (eq. rho_residual)
 *   - final sweep for f^n (eq. sweep_to_obtain_f) and the RHS b~ (Sec. 2.3)
 *   - DMD reduced operator (Sec. 3.1, eq. dmd-operator), incremental SVD
 *     (App. B, eq. svd_core), phases 1-3 and error-indicator updates
 *     (Sec. 3.2, eq. ig_stop, eq. dmd-ig, eq. correction_snapshot, eq. pc_stop,
 *     eq. dmd-sa, Alg. 2).
 *
 * Readings where the paper is silent are listed next to the code that takes
 * them (DSA discretisation for finite volume, relative stop test, which iterate
 * is returned, truncation rule, normalised indicators, rank-deficient snapshots).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)

#define ORC_SI_DSA 0
#define ORC_ROM_SI_DSA 1
#define ORC_SI_PLAIN 2

/* correction used where DSA would be (Sec. 3.3, Sec. 4.5) */
#define ORC_PC_DSA 0
#define ORC_PC_MH 1

/* time discretisation (Sec. 2.1) */
#define ORC_BE 0
#define ORC_BDF2 1

#define ORC_MAX_LEVELS 4

/* spatial discretisation (Sec. 2.1, eq. DG) */
#define ORC_FV 0   /* K = 0: piecewise constants = first-order upwind finite volume */
#define ORC_DG1 1  /* K = 1: piecewise linear upwind DG (slabs) */

typedef struct {
  int32_t dim, nx, ny;
  double lx, ly;
  int32_t n_polar, n_azim;
  const double *sigma_s, *sigma_a, *source, *f0; /* [ny*nx], x fastest */
  double inflow[4];                              /* x-lo, x-hi, y-lo, y-hi */
  double dt, tol;
  int32_t max_iter;
  int32_t method;
  double eps_ig, eps_pc, eps_up;
  int32_t r_max;
  int32_t abs_up_norm;
  int32_t precond;     /* ORC_PC_DSA or ORC_PC_MH */
  int32_t time_scheme; /* ORC_BE or ORC_BDF2 */
  int32_t pc_levels;   /* sequential correction ROMs for iterations 1..pc_levels (0 = 1) */
  int32_t mh_rank;     /* McClarren-Haut pairs per model (0 = r_max) */
  int32_t scheme;      /* ORC_FV or ORC_DG1 */
  int32_t pad_;
  double lu_tol;       /* singular-pivot threshold of the reduced ROM systems
                          relative to their largest entry (0 = 1e-14) */
} orc_desc;

typedef struct {
  int32_t iters;     /* SI sweeps used in this step (l at convergence) */
  int32_t phase;     /* 1, 2 or 3 at the start of the step */
  int32_t converged; /* 1 if the stop test passed */
  int32_t ig_update; /* 1 if a snapshot was added to the IG ROM */
  int32_t pc_update; /* 1 if a snapshot was added to the PC ROM */
  int32_t rank_ig, rank_pc;
  int32_t fallback;  /* 1 if a singular reduced system forced plain IG/DSA */
  double e_ig, e_pc; /* error indicators (-1 when not evaluated) */
  double residual;   /* last ||y - rho_prev||_inf / ||y||_inf */
} orc_step_rec;

/* ------------------------------------------------------------------------ */
/* Quadrature                                                                */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n(x) and its derivative, three-term recurrence. */
static void legendre_eval(int n, double x, double *pn, double *dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *pn = 1.0;
    *dpn = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

/* n-point Gauss-Legendre rule on [-1,1] with weights normalised to sum 1
 * (Sec. 2.1: weights sum to one).  Nodes ascending. */
int orc_gauss_legendre(int n, double *mu, double *w) {
  if (n < 1) return ORC_EINVAL;
  for (int i = 0; i < n; ++i) {
    /* Chebyshev-type initial guess for the i-th root (descending), Newton */
    double x = cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn, dpn;
    for (int it = 0; it < 100; ++it) {
      legendre_eval(n, x, &pn, &dpn);
      double dx = pn / dpn;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    legendre_eval(n, x, &pn, &dpn);
    /* standard weight 2/((1-x^2) P_n'(x)^2), halved so the weights sum to 1 */
    double wi = 1.0 / ((1.0 - x * x) * dpn * dpn);
    mu[n - 1 - i] = x;
    w[n - 1 - i] = wi;
  }
  return ORC_OK;
}

/* CL(N_phi, N_z) on the unit sphere (App. A): phi_k = (2k-1) pi / N_phi,
 * weight 1/N_phi, times the normalised N_z-point Gauss-Legendre rule in z;
 * ordering j = (j2-1) N_phi + j1 (App. A). */
int orc_cl_quadrature(int nphi, int nz, double *ox, double *oy, double *oz,
                      double *w) {
  if (nphi < 1 || nz < 1) return ORC_EINVAL;
  double *z = (double *)malloc(sizeof(double) * nz);
  double *wz = (double *)malloc(sizeof(double) * nz);
  orc_gauss_legendre(nz, z, wz);
  for (int j2 = 0; j2 < nz; ++j2) {
    double st = sqrt(1.0 - z[j2] * z[j2]);
    for (int j1 = 0; j1 < nphi; ++j1) {
      double phi = (2.0 * (j1 + 1) - 1.0) * M_PI / nphi;
      int j = j2 * nphi + j1;
      ox[j] = cos(phi) * st;
      oy[j] = sin(phi) * st;
      oz[j] = z[j2];
      w[j] = wz[j2] / nphi;
    }
  }
  free(z);
  free(wz);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (the oracle's own; pinned against numpy)       */
/* ------------------------------------------------------------------------ */

/* One-sided (Hestenes) Jacobi SVD of a rows x cols matrix K (row-major),
 * rows <= cols.  Right rotations orthogonalise the columns of B = K V; the
 * singular values are the column norms.  Outputs, sorted by descending
 * singular value: s[cols], V[cols x cols] (row-major, column j = j-th right
 * singular vector), Uc[rows x cols] (column j = B_j / s_j, zero if s_j = 0). */
void orc_jacobi_svd(int rows, int cols, const double *K, double *Uc, double *s,
                    double *V) {
  double *B = (double *)malloc(sizeof(double) * rows * cols);
  double *Vw = (double *)malloc(sizeof(double) * cols * cols);
  memcpy(B, K, sizeof(double) * rows * cols);
  for (int i = 0; i < cols; ++i)
    for (int j = 0; j < cols; ++j) Vw[i * cols + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < cols - 1; ++p) {
      for (int q = p + 1; q < cols; ++q) {
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int i = 0; i < rows; ++i) {
          double bp = B[i * cols + p], bq = B[i * cols + q];
          alpha += bp * bp;
          beta += bq * bq;
          gamma += bp * bq;
        }
        if (gamma == 0.0 || fabs(gamma) <= 1e-15 * sqrt(alpha * beta)) continue;
        rotated = 1;
        double zeta = (beta - alpha) / (2.0 * gamma);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        double sn = c * t;
        for (int i = 0; i < rows; ++i) {
          double bp = B[i * cols + p], bq = B[i * cols + q];
          B[i * cols + p] = c * bp - sn * bq;
          B[i * cols + q] = sn * bp + c * bq;
        }
        for (int i = 0; i < cols; ++i) {
          double vp = Vw[i * cols + p], vq = Vw[i * cols + q];
          Vw[i * cols + p] = c * vp - sn * vq;
          Vw[i * cols + q] = sn * vp + c * vq;
        }
      }
    }
    if (!rotated) break;
  }
  /* column norms, then a selection sort into descending order */
  double *nrm = (double *)malloc(sizeof(double) * cols);
  int *ord = (int *)malloc(sizeof(int) * cols);
  for (int j = 0; j < cols; ++j) {
    double a = 0.0;
    for (int i = 0; i < rows; ++i) a += B[i * cols + j] * B[i * cols + j];
    nrm[j] = sqrt(a);
    ord[j] = j;
  }
  for (int a = 0; a < cols; ++a) {
    int best = a;
    for (int b = a + 1; b < cols; ++b)
      if (nrm[ord[b]] > nrm[ord[best]]) best = b;
    int tmp = ord[a];
    ord[a] = ord[best];
    ord[best] = tmp;
  }
  for (int jj = 0; jj < cols; ++jj) {
    int j = ord[jj];
    s[jj] = nrm[j];
    for (int i = 0; i < cols; ++i) V[i * cols + jj] = Vw[i * cols + j];
    for (int i = 0; i < rows; ++i)
      Uc[i * cols + jj] = (nrm[j] > 0.0) ? B[i * cols + j] / nrm[j] : 0.0;
  }
  free(nrm);
  free(ord);
  free(B);
  free(Vw);
}

/* LU factorisation with partial pivoting, in place (row-major n x n).
 * Returns 0 on success, 1 if a pivot is below tol * max|A| (singular). */
static int lu_factor_tol(int n, double *A, int *piv, double tol) {
  double amax = 0.0;
  for (int i = 0; i < n * n; ++i)
    if (fabs(A[i]) > amax) amax = fabs(A[i]);
  int bad = (amax == 0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    double akk = A[k * n + k];
    if (fabs(akk) < tol * amax || akk == 0.0) {
      bad = 1;
      continue;
    }
    for (int i = k + 1; i < n; ++i) {
      double l = A[i * n + k] / akk;
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return bad;
}

int orc_lu_factor(int n, double *A, int *piv) { return lu_factor_tol(n, A, piv, 1e-14); }

void orc_lu_solve(int n, const double *LU, const int *piv, double *b) {
  for (int k = 0; k < n; ++k) {
    int p = piv[k];
    if (p != k) {
      double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
    b[i] /= LU[i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* Incremental SVD + DMD reduced operator (Sec. 3.1, App. B)                 */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nc, rmax, rank;
  double *U;  /* column k at U + k*nc, k < rank */
  double *S;  /* singular values, descending */
  double *W;  /* W = B V, column k at W + k*nc */
  double *Ar; /* LU factors of the reduced operator U^T W S^{-1} (rank x rank) */
  int *piv;
  int lu_ok;
  int last_deficient;
  double lu_tol; /* singular-pivot threshold of the reduced system (R17) */
} orc_rom;

static int rom_init(orc_rom *m, int nc, int rmax) {
  memset(m, 0, sizeof(*m));
  m->nc = nc;
  m->rmax = rmax;
  m->lu_tol = 1e-14;
  m->U = (double *)calloc((size_t)(rmax + 1) * nc, sizeof(double));
  m->W = (double *)calloc((size_t)(rmax + 1) * nc, sizeof(double));
  m->S = (double *)calloc(rmax + 1, sizeof(double));
  m->Ar = (double *)calloc((size_t)(rmax + 1) * (rmax + 1), sizeof(double));
  m->piv = (int *)calloc(rmax + 1, sizeof(int));
  if (!m->U || !m->W || !m->S || !m->Ar || !m->piv) return ORC_ENOMEM;
  return ORC_OK;
}

static void rom_free(orc_rom *m) {
  free(m->U);
  free(m->W);
  free(m->S);
  free(m->Ar);
  free(m->piv);
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Reduced operator of eq. dmd-operator: A_r = U^T (B V) S^{-1}, then its LU. */
static void rom_refresh(orc_rom *m) {
  int r = m->rank, nc = m->nc;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      m->Ar[i * r + j] = dot(nc, m->U + (size_t)i * nc, m->W + (size_t)j * nc) / m->S[j];
  m->lu_ok = (r > 0) && !lu_factor_tol(r, m->Ar, m->piv, m->lu_tol);
}

/* Add snapshot pair (x, b) per App. B.  truncate: keep s_i / sum(s) > eps.
 * The rank is always capped at rmax.  Returns 1 if the new column lay in
 * span(U) (rank-deficient snapshot), 0 otherwise, -1 if x = 0 at rank 0. */
int orc_rom_add(orc_rom *m, const double *x, const double *b, int truncate,
                double eps) {
  int nc = m->nc, r = m->rank;
  double xn = sqrt(dot(nc, x, x));
  if (r == 0) {
    if (xn == 0.0) return -1;
    for (int i = 0; i < nc; ++i) {
      m->U[i] = x[i] / xn;
      m->W[i] = b[i];
    }
    m->S[0] = xn;
    m->rank = 1;
    m->last_deficient = 0;
    rom_refresh(m);
    return 0;
  }
  /* projection onto span(U), classical Gram-Schmidt applied twice */
  double *a = (double *)calloc(r, sizeof(double));
  double *a2 = (double *)calloc(r, sizeof(double));
  double *p = (double *)malloc(sizeof(double) * nc);
  for (int k = 0; k < r; ++k) a[k] = dot(nc, m->U + (size_t)k * nc, x);
  for (int i = 0; i < nc; ++i) {
    double v = x[i];
    for (int k = 0; k < r; ++k) v -= m->U[(size_t)k * nc + i] * a[k];
    p[i] = v;
  }
  for (int k = 0; k < r; ++k) a2[k] = dot(nc, m->U + (size_t)k * nc, p);
  for (int i = 0; i < nc; ++i) {
    double v = p[i];
    for (int k = 0; k < r; ++k) v -= m->U[(size_t)k * nc + i] * a2[k];
    p[i] = v;
  }
  for (int k = 0; k < r; ++k) a[k] += a2[k];
  double nu = sqrt(dot(nc, p, p));
  int deficient = !(nu > 1e-12 * xn);
  int rows = deficient ? r : r + 1, cols = r + 1;
  /* core matrix [[diag S, U^T x], [0, nu]] (eq. svd_core) */
  double *K = (double *)calloc((size_t)rows * cols, sizeof(double));
  for (int i = 0; i < r; ++i) {
    K[i * cols + i] = m->S[i];
    K[i * cols + r] = a[i];
  }
  if (!deficient) K[r * cols + r] = nu;
  double *Uc = (double *)malloc(sizeof(double) * rows * cols);
  double *sc = (double *)malloc(sizeof(double) * cols);
  double *Vc = (double *)malloc(sizeof(double) * cols * cols);
  orc_jacobi_svd(rows, cols, K, Uc, sc, Vc);
  int k = rows;
  if (truncate) {
    double tot = 0.0;
    for (int i = 0; i < rows; ++i) tot += sc[i];
    int kk = 0;
    for (int i = 0; i < rows; ++i)
      if (sc[i] / tot > eps) kk = i + 1;
    k = kk > 0 ? kk : 1;
  }
  if (k > m->rmax) k = m->rmax;
  /* U <- [U, p/nu] Uc[:, :k];  W <- [W, b] Vc[:, :k] */
  double *Un = (double *)calloc((size_t)k * nc, sizeof(double));
  double *Wn = (double *)calloc((size_t)k * nc, sizeof(double));
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < nc; ++i) {
      double u = 0.0;
      for (int q = 0; q < r; ++q) u += m->U[(size_t)q * nc + i] * Uc[q * cols + j];
      if (!deficient) u += (p[i] / nu) * Uc[r * cols + j];
      Un[(size_t)j * nc + i] = u;
      double w = 0.0;
      for (int q = 0; q < r; ++q) w += m->W[(size_t)q * nc + i] * Vc[q * cols + j];
      w += b[i] * Vc[r * cols + j];
      Wn[(size_t)j * nc + i] = w;
    }
  }
  memcpy(m->U, Un, sizeof(double) * (size_t)k * nc);
  memcpy(m->W, Wn, sizeof(double) * (size_t)k * nc);
  for (int j = 0; j < k; ++j) m->S[j] = sc[j];
  m->rank = k;
  m->last_deficient = deficient;
  rom_refresh(m);
  free(a);
  free(a2);
  free(p);
  free(K);
  free(Uc);
  free(sc);
  free(Vc);
  free(Un);
  free(Wn);
  return deficient;
}

/* smallest retained singular value over the sum (eq. ig_stop, eq. pc_stop) */
static double rom_tail_ratio(const orc_rom *m) {
  double tot = 0.0;
  for (int i = 0; i < m->rank; ++i) tot += m->S[i];
  return tot > 0.0 ? m->S[m->rank - 1] / tot : 0.0;
}

/* y = U * LU^{-1} (U^T rhs): the ROM solve shared by eq. dmd-ig and eq. dmd-sa */
static void rom_apply(const orc_rom *m, const double *rhs, double *out) {
  int r = m->rank, nc = m->nc;
  double *c = (double *)malloc(sizeof(double) * (r > 0 ? r : 1));
  for (int k = 0; k < r; ++k) c[k] = dot(nc, m->U + (size_t)k * nc, rhs);
  orc_lu_solve(r, m->Ar, m->piv, c);
  for (int i = 0; i < nc; ++i) {
    double v = 0.0;
    for (int k = 0; k < r; ++k) v += m->U[(size_t)k * nc + i] * c[k];
    out[i] = v;
  }
  free(c);
}

/* standalone ROM object for unit pins of the incremental SVD */
void *orc_rom_new(int nc, int rmax) {
  orc_rom *m = (orc_rom *)malloc(sizeof(orc_rom));
  if (!m) return NULL;
  if (rom_init(m, nc, rmax)) {
    rom_free(m);
    free(m);
    return NULL;
  }
  return m;
}
void orc_rom_delete(void *h) {
  if (!h) return;
  rom_free((orc_rom *)h);
  free(h);
}
int orc_rom_push(void *h, const double *x, const double *b, int truncate, double eps) {
  return orc_rom_add((orc_rom *)h, x, b, truncate, eps);
}
int orc_rom_rank(void *h) { return ((orc_rom *)h)->rank; }
int orc_rom_lu_ok(void *h) { return ((orc_rom *)h)->lu_ok; }
void orc_rom_get(void *h, double *U, double *S, double *W) {
  orc_rom *m = (orc_rom *)h;
  memcpy(U, m->U, sizeof(double) * (size_t)m->rank * m->nc);
  memcpy(W, m->W, sizeof(double) * (size_t)m->rank * m->nc);
  memcpy(S, m->S, sizeof(double) * m->rank);
}
/* reduced operator A_r = U^T W S^{-1} recomputed (not the LU) */
void orc_rom_reduced(void *h, double *Ar) {
  orc_rom *m = (orc_rom *)h;
  int r = m->rank;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      Ar[i * r + j] = dot(m->nc, m->U + (size_t)i * m->nc, m->W + (size_t)j * m->nc) / m->S[j];
}
void orc_rom_solve(void *h, const double *rhs, double *out) {
  rom_apply((orc_rom *)h, rhs, out);
}

/* ------------------------------------------------------------------------ */
/* McClarren-Haut DMD across iterations (Sec. 3.3)                          */
/* ------------------------------------------------------------------------ */

/* McClarren-Haut model of the sweep operator T Sigma_s built from the pairs
 * of one time step's iterations (Sec. 3.3): input differences
 * rho^{(k-1)} - rho^{(k-2)} and their images y_k - y_{k-1}, each pair scaled
 * by the input's 2-norm.  Reading: the pairs' DMD is computed through a QR
 * factorisation of the inputs (X = Q R, Gram-Schmidt applied twice) instead
 * of an SVD; without truncation both give the same reduced operator
 * Q^T T Sigma_s Q = Q^T Z R^{-1}. */
typedef struct {
  int nc, cap, m;
  double *Q; /* orthonormal inputs, column k at Q + k*nc */
  double *Z; /* scaled outputs, column k at Z + k*nc */
  double *R; /* upper triangular, R[i*cap + j] */
} orc_mh;

/* Reading: a pair whose scaled input has an orthogonal remainder at or below
 * this fraction of its norm adds no new direction and is skipped (its image
 * would be dominated by rounding). */
#define ORC_MH_DEP 1e-6

static int mh_init(orc_mh *M, int nc, int cap) {
  memset(M, 0, sizeof(*M));
  M->nc = nc;
  M->cap = cap;
  M->Q = (double *)calloc((size_t)cap * nc, sizeof(double));
  M->Z = (double *)calloc((size_t)cap * nc, sizeof(double));
  M->R = (double *)calloc((size_t)cap * cap, sizeof(double));
  return (M->Q && M->Z && M->R) ? ORC_OK : ORC_ENOMEM;
}

static void mh_free(orc_mh *M) {
  free(M->Q);
  free(M->Z);
  free(M->R);
}

/* Add the pair (x, z = T Sigma_s x), both scaled by 1/||x||_2.  A full model
 * (cap pairs) restarts from this pair.  Returns 1 when the pair was skipped. */
static int mh_push(orc_mh *M, const double *x, const double *z, double *p) {
  const int nc = M->nc;
  const double xn = sqrt(dot(nc, x, x));
  if (!(xn > 0.0)) return 1;
  if (M->m == M->cap) M->m = 0;
  const int m = M->m;
  double a[64], a2[64];
  for (int k = 0; k < m; ++k) a[k] = dot(nc, M->Q + (size_t)k * nc, x) / xn;
  for (int i = 0; i < nc; ++i) {
    double v = x[i] / xn;
    for (int k = 0; k < m; ++k) v -= M->Q[(size_t)k * nc + i] * a[k];
    p[i] = v;
  }
  for (int k = 0; k < m; ++k) a2[k] = dot(nc, M->Q + (size_t)k * nc, p);
  for (int i = 0; i < nc; ++i) {
    double v = p[i];
    for (int k = 0; k < m; ++k) v -= M->Q[(size_t)k * nc + i] * a2[k];
    p[i] = v;
  }
  const double nu = sqrt(dot(nc, p, p));
  if (!(nu > ORC_MH_DEP)) return 1;
  for (int i = 0; i < nc; ++i) {
    M->Q[(size_t)m * nc + i] = p[i] / nu;
    M->Z[(size_t)m * nc + i] = z[i] / xn;
  }
  for (int k = 0; k < m; ++k) M->R[k * M->cap + m] = a[k] + a2[k];
  M->R[m * M->cap + m] = nu;
  for (int k = m + 1; k < M->cap; ++k) M->R[k * M->cap + m] = 0.0;
  M->m = m + 1;
  return 0;
}

/* Correction from the model: with A~ = Q^T Z R^{-1} (the pairs' DMD of
 * T Sigma_s on span(Q)), the ideal correction equation (I - T Sigma_s) d =
 * T Sigma_s r (eq. ideal_correct) restricted to span(Q) gives
 * d = Q (I - A~)^{-1} A~ Q^T r.  Returns 0 when applied, 1 when there is no
 * model or I - A~ is singular (out = 0 then). */
static int mh_correct(const orc_mh *M, const double *r, double *out) {
  const int nc = M->nc, m = M->m, cap = M->cap;
  memset(out, 0, sizeof(double) * nc);
  if (m == 0) return 1;
  double B[64 * 64], At[64 * 64], Mi[64 * 64], g[64], qr[64];
  int piv[64];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) B[i * m + j] = dot(nc, M->Q + (size_t)i * nc, M->Z + (size_t)j * nc);
  /* A~ R = B, R upper triangular: column by column */
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double v = B[i * m + j];
      for (int k = 0; k < j; ++k) v -= At[i * m + k] * M->R[k * cap + j];
      At[i * m + j] = v / M->R[j * cap + j];
    }
  for (int k = 0; k < m; ++k) qr[k] = dot(nc, M->Q + (size_t)k * nc, r);
  for (int i = 0; i < m; ++i) {
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += At[i * m + k] * qr[k];
    g[i] = v;
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Mi[i * m + j] = (i == j ? 1.0 : 0.0) - At[i * m + j];
  if (orc_lu_factor(m, Mi, piv)) return 1;
  orc_lu_solve(m, Mi, piv, g);
  for (int i = 0; i < nc; ++i) {
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += M->Q[(size_t)k * nc + i] * g[k];
    out[i] = v;
  }
  return 0;
}

/* standalone model for the unit pins */
void *orc_mh_new(int nc, int cap) {
  orc_mh *M = (orc_mh *)malloc(sizeof(orc_mh));
  if (!M) return NULL;
  if (cap < 1 || cap > 64 || mh_init(M, nc, cap)) {
    mh_free(M);
    free(M);
    return NULL;
  }
  return M;
}
void orc_mh_delete(void *h) {
  if (!h) return;
  mh_free((orc_mh *)h);
  free(h);
}
int orc_mh_push(void *h, const double *x, const double *z) {
  orc_mh *M = (orc_mh *)h;
  double *p = (double *)malloc(sizeof(double) * M->nc);
  int r = mh_push(M, x, z, p);
  free(p);
  return r;
}
int orc_mh_size(void *h) { return ((orc_mh *)h)->m; }
int orc_mh_correct(void *h, const double *r, double *out) { return mh_correct((orc_mh *)h, r, out); }

/* ------------------------------------------------------------------------ */
/* Problem state                                                             */
/* ------------------------------------------------------------------------ */


typedef struct {
  orc_desc d;
  int nc, nv;   /* nc: unknowns of rho (N_x of Sec. 2.2: cells x DoFs per cell) */
  int ncell, ndof;
  double hx, hy;
  double *ox, *oy, *oz, *w; /* ordinates (1D: ox = mu) */
  double *ss, *sa, *G, *ct; /* per unknown: sigma_s, sigma_a, source, sigma_t + alpha/dt
                               (DG: the cell's values on both DoFs; the source's
                               slope DoF is zero) */
  double alpha;             /* time-derivative weight of the current operator:
                               1 (backward Euler, and the first BDF2 step) or 3/2 */
  double *f;                /* f^n, [nv][nc] */
  double *fold;             /* BDF2: f^{n-1}, [nv][nc] */
  double *rho;              /* rho^n */
  double *bt;               /* b~^{n-1}: right-hand side of the next step */
  /* DSA */
  double *dlo, *ddi, *dup;  /* 1D tridiagonal */
  double *band;             /* 2D: banded Cholesky factor, [nc][bw+1] */
  int bw;
  /* ROM: initial guess and the correction ROMs of iterations 1..L */
  int nlev;
  orc_rom ig, pc[ORC_MAX_LEVELS];
  int flag_ig, flag_pc[ORC_MAX_LEVELS], n0, nl[ORC_MAX_LEVELS];
  orc_mh mh;
  /* counters */
  int64_t steps, si_total, sweeps_total;
  int nonconv, fallbacks;
  int64_t ig_updates, pc_updates[ORC_MAX_LEVELS];
  orc_step_rec *hist;
  int64_t hist_cap;
  /* vectors of the last step, kept for the pins of Alg. 2: rho^{(0)},
   * rho^{(1/2)}, the ROM correction delta rho^{(1)}_DMD (zero when the step
   * did not apply it) and b~^{n-1} */
  double *last_rho0, *last_rhalf, *last_dpc, *last_bt;
  int last_used_pc;
  /* work */
  double *w0, *w1, *w2, *w3, *w4, *w5, *w6, *fcol;
  double *yl[ORC_MAX_LEVELS + 1];   /* rho^{(l-1/2)}, l = 1..L+1 */
  double *rl[ORC_MAX_LEVELS + 1];   /* rho^{(l-1)}, l = 1..L+1 */
  double *dl[ORC_MAX_LEVELS];       /* ROM corrections of iterations 1..L */
  double *yprev, *rprev2;           /* McClarren-Haut: y_{l-1}, rho^{(l-2)} */
} orc_problem;

static int desc_valid(const orc_desc *d) {
  if (d->dim != 1 && d->dim != 2) return 0;
  if (d->nx < 1 || d->ny < 1) return 0;
  if (d->dim == 1 && d->ny != 1) return 0;
  if (!(d->lx > 0.0) || (d->dim == 2 && !(d->ly > 0.0))) return 0;
  if (!(d->dt > 0.0) || !(d->tol > 0.0) || d->max_iter < 1) return 0;
  if (d->n_polar < 2 || d->n_polar % 2) return 0;
  if (d->dim == 2 && (d->n_azim < 4 || d->n_azim % 4)) return 0;
  if (d->method < 0 || d->method > 2) return 0;
  if (d->r_max < 1) return 0;
  if (d->precond != ORC_PC_DSA && d->precond != ORC_PC_MH) return 0;
  if (d->time_scheme != ORC_BE && d->time_scheme != ORC_BDF2) return 0;
  if (d->pc_levels < 0 || d->pc_levels > ORC_MAX_LEVELS) return 0;
  if (d->mh_rank < 0 || d->mh_rank > 64) return 0;
  if (!(d->lu_tol >= 0.0) || !isfinite(d->lu_tol)) return 0;
  if (d->scheme != ORC_FV && !(d->scheme == ORC_DG1 && d->dim == 1)) return 0;
  if (!d->sigma_s || !d->sigma_a || !d->source) return 0;
  size_t nc = (size_t)d->nx * d->ny;
  for (size_t i = 0; i < nc; ++i) {
    if (!(d->sigma_s[i] >= 0.0) || !isfinite(d->sigma_s[i])) return 0;
    if (!(d->sigma_a[i] >= 0.0) || !isfinite(d->sigma_a[i])) return 0;
    if (!isfinite(d->source[i])) return 0;
    if (d->f0 && !isfinite(d->f0[i])) return 0;
  }
  for (int k = 0; k < 4; ++k)
    if (!isfinite(d->inflow[k])) return 0;
  return 1;
}

/* Inflow value seen by ordinate j on its upwind x / y boundary. */
static double inflow_x(const orc_problem *P, int j) {
  return P->ox[j] > 0.0 ? P->d.inflow[0] : P->d.inflow[1];
}
static double inflow_y(const orc_problem *P, int j) {
  return P->oy[j] > 0.0 ? P->d.inflow[2] : P->d.inflow[3];
}

/* One transport sweep for ordinate j (Sec. 2.3: a single upwind-ordered pass
 * of block Gauss-Seidel).  s: per-cell right-hand side; out: f_j per cell.
 * zero_inflow: the correction / SI sweeps use zero inflow, since the boundary
 * data already sit in b~ (eq. dg_discrete1, G~_j).
 * 1D cell i, mu > 0: (1/dt + sigma_t + mu/h) f_i = s_i + (mu/h) f_{i-1}. */
static void sweep_one(const orc_problem *P, int j, const double *s, int zero_inflow,
                      double *out) {
  const int nx = P->d.nx, ny = P->d.ny;
  if (P->d.scheme == ORC_DG1) {
    /* eq. DG with K = 1 on the slab: on each cell f = u0 + sqrt(3) u1 xi
     * (xi in [-1, 1]; the basis 1, sqrt(3) xi is orthonormal for the cell
     * average), tested with both basis functions, upwind flux H-hat.  For
     * mu > 0, with c = sigma_t + alpha/dt, h the cell width, f_in the value
     * entering from the upwind face and s = s0 + sqrt(3) s1 xi:
     *   (c h + mu) u0 + sqrt(3) mu u1 = h s0 + mu f_in
     *   -sqrt(3) mu u0 + (c h + 3 mu) u1 = h s1 - sqrt(3) mu f_in
     * and the value leaving the cell is u0 + sqrt(3) u1.  mu < 0 is the
     * mirror image (xi -> -xi, so u1 and s1 change sign). */
    const double mu = fabs(P->ox[j]), h = P->hx, r3 = sqrt(3.0);
    const int pos = P->ox[j] > 0.0;
    double fin = zero_inflow ? 0.0 : inflow_x(P, j);
    for (int k = 0; k < nx; ++k) {
      const int i = pos ? k : nx - 1 - k;
      const double c = P->ct[2 * i];
      const double s0 = s[2 * i], s1 = pos ? s[2 * i + 1] : -s[2 * i + 1];
      const double a11 = c * h + mu, a12 = r3 * mu, a21 = -r3 * mu, a22 = c * h + 3.0 * mu;
      const double b1 = h * s0 + mu * fin, b2 = h * s1 - r3 * mu * fin;
      const double det = a11 * a22 - a12 * a21;
      const double u0 = (b1 * a22 - a12 * b2) / det;
      const double u1 = (a11 * b2 - a21 * b1) / det;
      out[2 * i] = u0;
      out[2 * i + 1] = pos ? u1 : -u1;
      fin = u0 + r3 * u1;
    }
    return;
  }
  if (P->d.dim == 1) {
    double m = fabs(P->ox[j]) / P->hx;
    double fin = zero_inflow ? 0.0 : inflow_x(P, j);
    if (P->ox[j] > 0.0) {
      for (int i = 0; i < nx; ++i) {
        out[i] = (s[i] + m * fin) / (P->ct[i] + m);
        fin = out[i];
      }
    } else {
      for (int i = nx - 1; i >= 0; --i) {
        out[i] = (s[i] + m * fin) / (P->ct[i] + m);
        fin = out[i];
      }
    }
    return;
  }
  double mx = fabs(P->ox[j]) / P->hx, my = fabs(P->oy[j]) / P->hy;
  double gx = zero_inflow ? 0.0 : inflow_x(P, j);
  double gy = zero_inflow ? 0.0 : inflow_y(P, j);
  int sx = P->ox[j] > 0.0 ? 1 : -1, sy = P->oy[j] > 0.0 ? 1 : -1;
  for (int a = 0; a < ny; ++a) {
    int iy = sy > 0 ? a : ny - 1 - a;
    for (int b = 0; b < nx; ++b) {
      int ix = sx > 0 ? b : nx - 1 - b;
      double fx = (b == 0) ? gx : out[iy * nx + (ix - sx)];
      double fy = (a == 0) ? gy : out[(iy - sy) * nx + ix];
      int c = iy * nx + ix;
      out[c] = (s[c] + mx * fx + my * fy) / (P->ct[c] + mx + my);
    }
  }
}

/* rho-moment of a sweep with an ordinate-independent source and zero
 * inflow: out = T (src)  (Sec. 2.3: T = sum_j w_j (M/dt + D_j + Sigma_t)^{-1}) */
static void apply_T(orc_problem *P, const double *src, double *out) {
  memset(out, 0, sizeof(double) * P->nc);
  for (int j = 0; j < P->nv; ++j) {
    sweep_one(P, j, src, 1, P->fcol);
    for (int i = 0; i < P->nc; ++i) out[i] += P->w[j] * P->fcol[i];
  }
}

/* ------------------------------------------------------------------------ */
/* DSA (eq. rho_residual) for upwind finite volume.                          */
/* Reading: the paper's consistent DSA is DG-specific and defined outside   */
/* the paper; for cell-centred FV we take the diffusion limit (Sec. 2,      */
/* D = 1/(3 sigma)) of the correction equation, whose absorption is         */
/* sigma_a + 1/dt (Sec. 2.3), with D_P = 1/(3 sigma~_t) + h/4 (the upwind   */
/* scheme's numerical diffusion <|Omega.e|> h / 2 with <|Omega.e|> = 1/2),  */
/* harmonic face coefficients and Marshak vacuum faces J.n = rho_b / 2.     */
/* DSA only preconditions: the fixed point does not depend on it.           */
/* ------------------------------------------------------------------------ */

static double dsa_D(const orc_problem *P, int c, double h) {
  return 1.0 / (3.0 * P->ct[c]) + 0.25 * h;
}
static double face_k(double Dp, double Dq, double h) {
  return 2.0 * Dp * Dq / (h * (Dp + Dq));
}
static double bdry_k(double Dp, double h) { return 2.0 * Dp / (h + 4.0 * Dp); }

/* matrix entry of the DSA operator, used by both the 1D setup and 2D factor */
static double dsa_entry(const orc_problem *P, int r, int c) {
  const int nx = P->d.nx, ny = P->d.ny;
  double sat = P->sa[r] + P->alpha / P->d.dt;
  int rx = r % nx, ry = r / nx, cx = c % nx, cy = c / nx;
  double hx = P->hx, hy = P->hy;
  if (r == c) {
    double v = sat;
    double Dx = dsa_D(P, r, hx);
    v += (rx > 0 ? face_k(Dx, dsa_D(P, r - 1, hx), hx) : bdry_k(Dx, hx)) / hx;
    v += (rx < nx - 1 ? face_k(Dx, dsa_D(P, r + 1, hx), hx) : bdry_k(Dx, hx)) / hx;
    if (P->d.dim == 2) {
      double Dy = dsa_D(P, r, hy);
      v += (ry > 0 ? face_k(Dy, dsa_D(P, r - nx, hy), hy) : bdry_k(Dy, hy)) / hy;
      v += (ry < ny - 1 ? face_k(Dy, dsa_D(P, r + nx, hy), hy) : bdry_k(Dy, hy)) / hy;
    }
    return v;
  }
  if (ry == cy && abs(rx - cx) == 1)
    return -face_k(dsa_D(P, r, hx), dsa_D(P, c, hx), hx) / hx;
  if (P->d.dim == 2 && rx == cx && abs(ry - cy) == 1)
    return -face_k(dsa_D(P, r, hy), dsa_D(P, c, hy), hy) / hy;
  return 0.0;
}

/* DSA for upwind DG-P1 (slabs).  Reading: the paper's "fully consistent"
 * DSA is defined in a reference outside the paper; here the correction
 * equation's diffusion limit, -(D d')' + sigma~_a d = sigma_s (rho^{l-1/2} -
 * rho^{l-1}) with D = 1/(3 sigma~_t), is discretised in the same DG-P1 space
 * by the modified interior penalty method: symmetric interior penalty with
 * the penalty max(D_L / h + D_R / h, 1/4) on interior faces, and Marshak
 * vacuum faces (a boundary term u v / 2).  Entry (r, c) of the bilinear form
 * a(phi_c, phi_r) divided by h, so that the right-hand side is sigma_s times
 * the DoF-wise difference (the mass matrix of the orthonormal basis is h I).
 * The matrix is SPD; the fixed point does not depend on it. */
static double mip_entry(const orc_problem *P, int r, int c) {
  const int N = P->ncell;
  const double h = P->hx, r3 = sqrt(3.0);
  const int ci = r / 2, k = r % 2, cj = c / 2, m = c % 2;
  if (abs(ci - cj) > 1) return 0.0;
  const double phiR[2] = {1.0, r3}, phiL[2] = {1.0, -r3};  /* values at xi = +1, -1 */
  const double dphi[2] = {0.0, 2.0 * r3 / h};              /* derivatives d/dx */
  double a = 0.0;
  if (ci == cj) {
    const double D = 1.0 / (3.0 * P->ct[2 * ci]);
    const double sat = P->sa[2 * ci] + P->alpha / P->d.dt;
    a += D * dphi[m] * dphi[k] * h + (k == m ? sat * h : 0.0);
  }
  /* faces f = p + 1/2 between cells p and p + 1 touching both rows' cells */
  for (int p = -1; p < N; ++p) {
    const int L = p, R = p + 1;
    /* jump [u] = u_L(+1) - u_R(-1) and the mean flux {D u'} of a basis
     * function of cell q */
    double ju = 0.0, jv = 0.0, fu = 0.0, fv = 0.0;
    const int touches_c = (cj == L || cj == R), touches_r = (ci == L || ci == R);
    if (!touches_c || !touches_r) continue;
    if (L < 0 || R >= N) {  /* vacuum face: Marshak, (1/2) u v */
      const double uc = (cj == L) ? phiR[m] : phiL[m];
      const double vr = (ci == L) ? phiR[k] : phiL[k];
      a += 0.5 * uc * vr;
      continue;
    }
    const double DL = 1.0 / (3.0 * P->ct[2 * L]), DR = 1.0 / (3.0 * P->ct[2 * R]);
    double kap = DL / h + DR / h;
    if (kap < 0.25) kap = 0.25;
    if (cj == L) {
      ju = phiR[m];
      fu = 0.5 * DL * dphi[m];
    } else {
      ju = -phiL[m];
      fu = 0.5 * DR * dphi[m];
    }
    if (ci == L) {
      jv = phiR[k];
      fv = 0.5 * DL * dphi[k];
    } else {
      jv = -phiL[k];
      fv = 0.5 * DR * dphi[k];
    }
    a += kap * ju * jv - fu * jv - fv * ju;
  }
  return a / h;
}

static double dsa_matrix_entry(const orc_problem *P, int r, int c) {
  return P->d.scheme == ORC_DG1 ? mip_entry(P, r, c) : dsa_entry(P, r, c);
}

static int dsa_setup(orc_problem *P) {
  int nc = P->nc;
  free(P->dlo);
  free(P->ddi);
  free(P->dup);
  free(P->band);
  P->dlo = P->ddi = P->dup = P->band = NULL;
  if (P->d.dim == 1 && P->d.scheme == ORC_FV) {
    P->dlo = (double *)calloc(nc, sizeof(double));
    P->ddi = (double *)calloc(nc, sizeof(double));
    P->dup = (double *)calloc(nc, sizeof(double));
    if (!P->dlo || !P->ddi || !P->dup) return ORC_ENOMEM;
    for (int i = 0; i < nc; ++i) {
      P->ddi[i] = dsa_entry(P, i, i);
      P->dlo[i] = i > 0 ? dsa_entry(P, i, i - 1) : 0.0;
      P->dup[i] = i < nc - 1 ? dsa_entry(P, i, i + 1) : 0.0;
    }
    return ORC_OK;
  }
  /* 2D: banded Cholesky of the SPD 5-point matrix, lower bandwidth nx;
   * DG-P1 slabs: of the MIP matrix, lower bandwidth 3 (two DoFs per cell,
   * neighbouring cells coupled) */
  int bw = P->d.scheme == ORC_DG1 ? 3 : P->d.nx;
  P->bw = bw;
  P->band = (double *)calloc((size_t)nc * (bw + 1), sizeof(double));
  if (!P->band) return ORC_ENOMEM;
#define L(i, j) P->band[(size_t)(i) * (bw + 1) + ((i) - (j))]
  for (int i = 0; i < nc; ++i) {
    int j0 = i - bw > 0 ? i - bw : 0;
    for (int j = j0; j <= i; ++j) {
      double s = dsa_matrix_entry(P, i, j);
      int k0 = (i - bw > j - bw ? i - bw : j - bw);
      if (k0 < 0) k0 = 0;
      for (int k = k0; k < j; ++k) s -= L(i, k) * L(j, k);
      if (i == j) {
        if (!(s > 0.0)) return ORC_EINVAL;
        L(i, i) = sqrt(s);
      } else {
        L(i, j) = s / L(j, j);
      }
    }
  }
#undef L
  return ORC_OK;
}

/* exact solve of C x = rhs (Thomas in 1D, banded Cholesky in 2D) */
static void dsa_solve(orc_problem *P, const double *rhs, double *x) {
  int n = P->nc;
  if (P->d.dim == 1 && P->d.scheme == ORC_FV) {
    double *cp = P->w5, *dp = P->w6;
    cp[0] = P->dup[0] / P->ddi[0];
    dp[0] = rhs[0] / P->ddi[0];
    for (int i = 1; i < n; ++i) {
      double den = P->ddi[i] - P->dlo[i] * cp[i - 1];
      cp[i] = P->dup[i] / den;
      dp[i] = (rhs[i] - P->dlo[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return;
  }
  int bw = P->bw;
#define L(i, j) P->band[(size_t)(i) * (bw + 1) + ((i) - (j))]
  for (int i = 0; i < n; ++i) {
    double s = rhs[i];
    int k0 = i - bw > 0 ? i - bw : 0;
    for (int k = k0; k < i; ++k) s -= L(i, k) * x[k];
    x[i] = s / L(i, i);
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    int k1 = i + bw < n - 1 ? i + bw : n - 1;
    for (int k = i + 1; k <= k1; ++k) s -= L(k, i) * x[k];
    x[i] = s / L(i, i);
  }
#undef L
}

/* ------------------------------------------------------------------------ */
/* RHS and final sweeps                                                      */
/* ------------------------------------------------------------------------ */

/* Known part of the time derivative for the step about to be taken: f_j/dt
 * (backward Euler, Sec. 2.1 eq. time_discrete), or (4 f^{n-1}_j - f^{n-2}_j)
 * / (2 dt) for BDF2 (Sec. 2.1 names BDF as the alternative; its operator
 * carries 3/(2 dt)).  Reading: BDF2 starts with one backward-Euler step. */
static double hist_term(const orc_problem *P, int bdf2, size_t k) {
  if (bdf2) return (4.0 * P->f[k] - P->fold[k]) / (2.0 * P->d.dt);
  return P->f[k] / P->d.dt;
}

/* whether step number n (1-based) uses the BDF2 formula */
static int bdf2_step(const orc_problem *P, int64_t n) {
  return P->d.time_scheme == ORC_BDF2 && n >= 2;
}

/* b~ = sum_j w_j (alpha M/dt + D_j + Sigma_t)^{-1} (history_j + G~_j)
 * (Sec. 2.3) for step number n */
static void compute_rhs(orc_problem *P, int64_t n, double *bt) {
  int nc = P->nc;
  const int b2 = bdf2_step(P, n);
  memset(bt, 0, sizeof(double) * nc);
  for (int j = 0; j < P->nv; ++j) {
    for (int i = 0; i < nc; ++i) P->w0[i] = hist_term(P, b2, (size_t)j * nc + i) + P->G[i];
    sweep_one(P, j, P->w0, 0, P->fcol);
    for (int i = 0; i < nc; ++i) bt[i] += P->w[j] * P->fcol[i];
  }
}

/* f^n_j from rho^n (eq. sweep_to_obtain_f) for step number n; BDF2 keeps
 * f^{n-1} as the older level */
static void final_sweep(orc_problem *P, int64_t n, const double *rho) {
  int nc = P->nc;
  const int b2 = bdf2_step(P, n);
  for (int j = 0; j < P->nv; ++j) {
    double *fj = P->f + (size_t)j * nc;
    for (int i = 0; i < nc; ++i) P->w0[i] = P->ss[i] * rho[i] + hist_term(P, b2, (size_t)j * nc + i) + P->G[i];
    sweep_one(P, j, P->w0, 0, P->fcol);
    if (P->fold) memcpy(P->fold + (size_t)j * nc, fj, sizeof(double) * nc);
    memcpy(fj, P->fcol, sizeof(double) * nc);
  }
}

/* transport and DSA operators for the time weight alpha (1 or 3/2) */
static int set_alpha(orc_problem *P, double alpha) {
  P->alpha = alpha;
  for (int i = 0; i < P->nc; ++i) P->ct[i] = P->ss[i] + P->sa[i] + alpha / P->d.dt;
  return dsa_setup(P);
}

/* ------------------------------------------------------------------------ */
/* Create / destroy                                                          */
/* ------------------------------------------------------------------------ */

void orc_destroy(void *h);

void *orc_create(const orc_desc *d) {
  if (!d || !desc_valid(d)) return NULL;
  orc_problem *P = (orc_problem *)calloc(1, sizeof(orc_problem));
  if (!P) return NULL;
  P->d = *d;
  P->d.sigma_s = P->d.sigma_a = P->d.source = P->d.f0 = NULL;
  const int ncell = d->nx * d->ny, ndof = d->scheme == ORC_DG1 ? 2 : 1;
  int nc = ncell * ndof;
  P->ncell = ncell;
  P->ndof = ndof;
  P->nc = nc;
  P->hx = d->lx / d->nx;
  P->hy = d->dim == 2 ? d->ly / d->ny : 1.0;
  P->nv = d->dim == 1 ? d->n_polar : d->n_polar * d->n_azim;
  int nv = P->nv;
  P->ox = (double *)calloc(nv, sizeof(double));
  P->oy = (double *)calloc(nv, sizeof(double));
  P->oz = (double *)calloc(nv, sizeof(double));
  P->w = (double *)calloc(nv, sizeof(double));
  P->ss = (double *)malloc(sizeof(double) * nc);
  P->sa = (double *)malloc(sizeof(double) * nc);
  P->G = (double *)malloc(sizeof(double) * nc);
  P->ct = (double *)malloc(sizeof(double) * nc);
  P->f = (double *)malloc(sizeof(double) * (size_t)nv * nc);
  P->rho = (double *)malloc(sizeof(double) * nc);
  P->bt = (double *)malloc(sizeof(double) * nc);
  P->w0 = (double *)malloc(sizeof(double) * nc);
  P->w1 = (double *)malloc(sizeof(double) * nc);
  P->w2 = (double *)malloc(sizeof(double) * nc);
  P->w3 = (double *)malloc(sizeof(double) * nc);
  P->w4 = (double *)malloc(sizeof(double) * nc);
  P->w5 = (double *)malloc(sizeof(double) * nc);
  P->w6 = (double *)malloc(sizeof(double) * nc);
  P->fcol = (double *)malloc(sizeof(double) * nc);
  P->nlev = d->pc_levels > 0 ? d->pc_levels : 1;
  for (int k = 0; k <= P->nlev; ++k) {
    P->yl[k] = (double *)calloc(nc, sizeof(double));
    P->rl[k] = (double *)calloc(nc, sizeof(double));
    if (k < P->nlev) P->dl[k] = (double *)calloc(nc, sizeof(double));
    if (!P->yl[k] || !P->rl[k] || (k < P->nlev && !P->dl[k])) {
      orc_destroy(P);
      return NULL;
    }
  }
  if (d->precond == ORC_PC_MH) {
    P->yprev = (double *)calloc(nc, sizeof(double));
    P->rprev2 = (double *)calloc(nc, sizeof(double));
    if (!P->yprev || !P->rprev2 || mh_init(&P->mh, nc, d->mh_rank > 0 ? d->mh_rank : d->r_max)) {
      orc_destroy(P);
      return NULL;
    }
  }
  if (d->time_scheme == ORC_BDF2) {
    P->fold = (double *)calloc((size_t)nv * nc, sizeof(double));
    if (!P->fold) {
      orc_destroy(P);
      return NULL;
    }
  }
  P->last_rho0 = (double *)calloc(nc, sizeof(double));
  P->last_rhalf = (double *)calloc(nc, sizeof(double));
  P->last_dpc = (double *)calloc(nc, sizeof(double));
  P->last_bt = (double *)calloc(nc, sizeof(double));
  if (!P->last_rho0 || !P->last_rhalf || !P->last_dpc || !P->last_bt) {
    orc_destroy(P);
    return NULL;
  }
  if (!P->ox || !P->oy || !P->oz || !P->w || !P->ss || !P->sa || !P->G || !P->ct ||
      !P->f || !P->rho || !P->bt || !P->w0 || !P->w1 || !P->w2 || !P->w3 || !P->w4 ||
      !P->w5 || !P->w6 || !P->fcol) {
    orc_destroy(P);
    return NULL;
  }
  if (d->dim == 1)
    orc_gauss_legendre(d->n_polar, P->ox, P->w);
  else
    orc_cl_quadrature(d->n_azim, d->n_polar, P->ox, P->oy, P->oz, P->w);
  for (int i = 0; i < nc; ++i) {
    const int cell = i / ndof, dof = i % ndof;
    P->ss[i] = d->sigma_s[cell];
    P->sa[i] = d->sigma_a[cell];
    P->G[i] = dof == 0 ? d->source[cell] : 0.0;
    P->rho[i] = (dof == 0 && d->f0) ? d->f0[cell] : 0.0;
  }
  for (int j = 0; j < nv; ++j)
    for (int i = 0; i < nc; ++i) P->f[(size_t)j * nc + i] = P->rho[i];
  if (set_alpha(P, 1.0) != ORC_OK) {
    orc_destroy(P);
    return NULL;
  }
  int bad = rom_init(&P->ig, nc, d->r_max);
  for (int k = 0; k < P->nlev; ++k) bad |= rom_init(&P->pc[k], nc, d->r_max);
  if (d->lu_tol > 0.0) {
    P->ig.lu_tol = d->lu_tol;
    for (int k = 0; k < P->nlev; ++k) P->pc[k].lu_tol = d->lu_tol;
  }
  if (bad) {
    orc_destroy(P);
    return NULL;
  }
  /* b~^0 from f^0 (the RHS sweep of the first step) */
  compute_rhs(P, 1, P->bt);
  return P;
}

void orc_destroy(void *h) {
  orc_problem *P = (orc_problem *)h;
  if (!P) return;
  free(P->ox); free(P->oy); free(P->oz); free(P->w);
  free(P->ss); free(P->sa); free(P->G); free(P->ct);
  free(P->f); free(P->rho); free(P->bt);
  free(P->w0); free(P->w1); free(P->w2); free(P->w3); free(P->w4); free(P->w5);
  free(P->w6); free(P->fcol);
  free(P->dlo); free(P->ddi); free(P->dup); free(P->band);
  rom_free(&P->ig);
  for (int k = 0; k < ORC_MAX_LEVELS; ++k) rom_free(&P->pc[k]);
  for (int k = 0; k <= ORC_MAX_LEVELS; ++k) {
    free(P->yl[k]);
    free(P->rl[k]);
    if (k < ORC_MAX_LEVELS) free(P->dl[k]);
  }
  mh_free(&P->mh);
  free(P->yprev);
  free(P->rprev2);
  free(P->fold);
  free(P->hist);
  free(P->last_rho0); free(P->last_rhalf); free(P->last_dpc); free(P->last_bt);
  free(P);
}

/* ------------------------------------------------------------------------ */
/* One time step: Alg. 2 around Alg. 1                                       */
/* ------------------------------------------------------------------------ */

static double norm_inf(int n, const double *a) {
  double m = 0.0;
  for (int i = 0; i < n; ++i)
    if (fabs(a[i]) > m) m = fabs(a[i]);
  return m;
}
static double diff_inf(int n, const double *a, const double *b) {
  double m = 0.0;
  for (int i = 0; i < n; ++i)
    if (fabs(a[i] - b[i]) > m) m = fabs(a[i] - b[i]);
  return m;
}
static double diff_2(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
  return sqrt(s);
}

int orc_step(void *h) {
  orc_problem *P = (orc_problem *)h;
  const int nc = P->nc, L = P->nlev;
  const int rom = (P->d.method == ORC_ROM_SI_DSA);
  const int mh = (P->d.precond == ORC_PC_MH);
  const int64_t n = P->steps + 1;
  orc_step_rec rec;
  memset(&rec, 0, sizeof(rec));
  rec.e_ig = rec.e_pc = -1.0;
  /* phases 1 .. L+2: the ROMs are completed one after the other (Sec. 3.2,
   * key feature 1); with one correction level these are phases 1-3 */
  int flags0[ORC_MAX_LEVELS];
  rec.phase = 1 + P->flag_ig;
  for (int k = 0; k < L; ++k) {
    flags0[k] = P->flag_pc[k];
    rec.phase += P->flag_ig && flags0[k];
  }

  double *rho0 = P->w1;     /* rho^{n,(0)} */
  double *rprev = P->w2;    /* rho^{n,(l-1)} */
  double *y = P->w3;        /* rho^{n,(l-1/2)} */
  double *scratch = (double *)malloc(sizeof(double) * nc);
  int applied[ORC_MAX_LEVELS] = {0};

  /* initial guess (Alg. 2: ROM-enhanced when Flag_IG, else rho^{n-1}) */
  if (rom && P->flag_ig && P->ig.lu_ok) {
    rom_apply(&P->ig, P->bt, rho0);
  } else {
    if (rom && P->flag_ig) {
      rec.fallback = 1;
      P->fallbacks++;
    }
    memcpy(rho0, P->rho, sizeof(double) * nc);
  }
  memcpy(rprev, rho0, sizeof(double) * nc);
  if (mh) P->mh.m = 0; /* the McClarren-Haut model lives within one step */

  /* Alg. 1 */
  int l, conv = 0;
  for (l = 1; l <= P->d.max_iter; ++l) {
    for (int i = 0; i < nc; ++i) scratch[i] = P->ss[i] * rprev[i];
    apply_T(P, scratch, y);
    for (int i = 0; i < nc; ++i) y[i] += P->bt[i];
    if (l <= L + 1) { /* rho^{(l-1/2)} and rho^{(l-1)} for the correction ROMs */
      memcpy(P->yl[l - 1], y, sizeof(double) * nc);
      memcpy(P->rl[l - 1], rprev, sizeof(double) * nc);
    }
    /* stop test; reading: relative to ||y||_inf (absolute when y = 0) */
    double dn = diff_inf(nc, y, rprev), yn = norm_inf(nc, y);
    rec.residual = yn > 0.0 ? dn / yn : dn;
    if (yn > 0.0 ? (dn < P->d.tol * yn) : (dn < P->d.tol)) {
      conv = 1;
      break;
    }
    if (l == P->d.max_iter) break;
    /* McClarren-Haut pair of this iteration: (rho^{(l-1)} - rho^{(l-2)},
     * y_l - y_{l-1}), the second the sweep image of the first */
    if (mh && l >= 2) {
      for (int i = 0; i < nc; ++i) {
        P->w0[i] = rprev[i] - P->rprev2[i];
        P->w5[i] = y[i] - P->yprev[i];
      }
      mh_push(&P->mh, P->w0, P->w5, P->w6);
    }
    if (mh) {
      memcpy(P->yprev, y, sizeof(double) * nc);
      memcpy(P->rprev2, rprev, sizeof(double) * nc);
    }
    /* synthetic acceleration: the ROM of iteration l (eq. dmd-sa for l = 1;
     * a level l > 1 applies only after level l - 1 did in this step), else
     * DSA (eq. rho_residual) or the McClarren-Haut correction */
    const int lev = l - 1;
    const int rom_here = rom && l <= L && flags0[lev] && (l == 1 || applied[lev - 1]);
    if (rom_here && P->pc[lev].lu_ok) {
      for (int i = 0; i < nc; ++i) P->w0[i] = y[i] - rprev[i];
      rom_apply(&P->pc[lev], P->w0, P->dl[lev]);
      applied[lev] = 1;
      for (int i = 0; i < nc; ++i) rprev[i] = y[i] + P->dl[lev][i];
    } else {
      if (rom_here) {
        rec.fallback = 1;
        P->fallbacks++;
      }
      if (P->d.method == ORC_SI_PLAIN) {
        memcpy(rprev, y, sizeof(double) * nc);
      } else if (mh) {
        for (int i = 0; i < nc; ++i) P->w0[i] = y[i] - rprev[i];
        mh_correct(&P->mh, P->w0, scratch);
        for (int i = 0; i < nc; ++i) rprev[i] = y[i] + scratch[i];
      } else {
        for (int i = 0; i < nc; ++i) P->w0[i] = P->ss[i] * (y[i] - rprev[i]);
        dsa_solve(P, P->w0, scratch);
        for (int i = 0; i < nc; ++i) rprev[i] = y[i] + scratch[i];
      }
    }
  }
  if (l > P->d.max_iter) l = P->d.max_iter;
  rec.iters = l;
  rec.converged = conv;

  /* rho^n = rho^{n,(l-1/2)}: the correction is not applied to the returned
   * iterate (Alg. 1 returns rho^{(l-1/2)}) */
  memcpy(P->rho, y, sizeof(double) * nc);

  /* f^n and b~^n; keep b~^{n-1} for the IG snapshot pair.  BDF2 switches to
   * its own operator after the backward-Euler start */
  double *bt_prev = (double *)malloc(sizeof(double) * nc);
  memcpy(bt_prev, P->bt, sizeof(double) * nc);
  final_sweep(P, n, P->rho);
  if (P->d.time_scheme == ORC_BDF2 && n == 1) set_alpha(P, 1.5);
  compute_rhs(P, n + 1, P->bt);

  /* ROM bookkeeping, Alg. 2.  Reading: under BDF2 the backward-Euler start
   * step solves with another operator and is not a snapshot. */
  if (rom && !(P->d.time_scheme == ORC_BDF2 && n == 1)) {
    double rn = sqrt(dot(nc, P->rho, P->rho));
    double scale = (P->d.abs_up_norm || rn == 0.0) ? 1.0 : 1.0 / rn;
    if (!P->flag_ig) {
      int dfc = orc_rom_add(&P->ig, P->rho, bt_prev, 0, P->d.eps_ig);
      if (dfc >= 0) {
        rec.ig_update = 1;
        P->ig_updates++;
        if (rom_tail_ratio(&P->ig) <= P->d.eps_ig || P->ig.rank >= P->d.r_max || dfc == 1) {
          P->flag_ig = 1;
          P->n0 = (int)n;
        }
      }
    } else {
      int lower_upd = 0;
      rec.e_ig = diff_2(nc, rho0, P->rho) * scale;
      if (rec.e_ig > P->d.eps_up) {
        orc_rom_add(&P->ig, P->rho, bt_prev, 1, P->d.eps_ig);
        lower_upd = 1;
        rec.ig_update = 1;
        P->ig_updates++;
      }
      /* correction snapshots of iteration lev + 1: x = rho^n - rho^{(lev+1/2)},
       * b = rho^{(lev+1/2)} - rho^{(lev)} (eq. correction_snapshot for lev = 0);
       * none when the step converged at that iteration.  A level collects
       * only once every level below it is complete. */
      for (int lev = 0; lev < L; ++lev) {
        if (lev > 0 && !flags0[lev - 1]) break;
        if (l <= lev + 1) break;
        double *xs = P->w0, *bs = scratch;
        for (int i = 0; i < nc; ++i) {
          xs[i] = P->rho[i] - P->yl[lev][i];
          bs[i] = P->yl[lev][i] - P->rl[lev][i];
        }
        int upd = 0;
        if (!flags0[lev]) {
          int dfc = orc_rom_add(&P->pc[lev], xs, bs, 0, P->d.eps_pc);
          if (dfc >= 0) {
            upd = 1;
            if (rom_tail_ratio(&P->pc[lev]) <= P->d.eps_pc || P->pc[lev].rank >= P->d.r_max || dfc == 1) {
              P->flag_pc[lev] = 1;
              int prior = P->n0;
              for (int k = 0; k < lev; ++k) prior += P->nl[k];
              P->nl[lev] = (int)n - prior;
            }
          }
        } else {
          /* Alg. 2: update when a ROM below was updated or the indicator
           * exceeds eps_UP.  Reading: a step that could not apply this
           * level's correction (singular reduced system) also updates it. */
          double e = -1.0;
          if (applied[lev]) e = diff_2(nc, P->dl[lev], xs) * scale;
          if (lev == 0) rec.e_pc = e;
          if (lower_upd || !applied[lev] || e > P->d.eps_up) {
            orc_rom_add(&P->pc[lev], xs, bs, 1, P->d.eps_pc);
            upd = 1;
          }
        }
        if (upd) {
          P->pc_updates[lev]++;
          if (lev == 0) rec.pc_update = 1;
          lower_upd = 1;
        }
      }
    }
    rec.rank_ig = P->ig.rank;
    rec.rank_pc = P->pc[0].rank;
  }

  P->steps++;
  P->si_total += rec.iters;
  P->sweeps_total += rec.iters + 2;
  if (!conv) P->nonconv++;
  if (P->steps > P->hist_cap) {
    int64_t cap = P->hist_cap ? 2 * P->hist_cap : 64;
    orc_step_rec *nh = (orc_step_rec *)realloc(P->hist, sizeof(orc_step_rec) * cap);
    if (nh) {
      P->hist = nh;
      P->hist_cap = cap;
    }
  }
  if (P->steps <= P->hist_cap) P->hist[P->steps - 1] = rec;
  memcpy(P->last_rho0, rho0, sizeof(double) * nc);
  memcpy(P->last_rhalf, P->yl[0], sizeof(double) * nc);
  if (applied[0])
    memcpy(P->last_dpc, P->dl[0], sizeof(double) * nc);
  else
    memset(P->last_dpc, 0, sizeof(double) * nc);
  memcpy(P->last_bt, bt_prev, sizeof(double) * nc);
  P->last_used_pc = applied[0];
  free(bt_prev);
  free(scratch);
  return conv ? ORC_OK : ORC_ENOCONV;
}

int orc_march(void *h, int nsteps) {
  int st = ORC_OK;
  for (int k = 0; k < nsteps; ++k) {
    int s = orc_step(h);
    if (s != ORC_OK) st = s;
  }
  return st;
}

/* ------------------------------------------------------------------------ */
/* Accessors and unit-level entry points for the pins                        */
/* ------------------------------------------------------------------------ */

int orc_ncells(void *h) { return ((orc_problem *)h)->nc; }
int orc_nord(void *h) { return ((orc_problem *)h)->nv; }
void orc_get_rho(void *h, double *out) {
  orc_problem *P = (orc_problem *)h;
  memcpy(out, P->rho, sizeof(double) * P->nc);
}
void orc_get_f(void *h, double *out) {
  orc_problem *P = (orc_problem *)h;
  memcpy(out, P->f, sizeof(double) * (size_t)P->nc * P->nv);
}
void orc_get_bt(void *h, double *out) {
  orc_problem *P = (orc_problem *)h;
  memcpy(out, P->bt, sizeof(double) * P->nc);
}
void orc_get_quadrature(void *h, double *ox, double *oy, double *oz, double *w) {
  orc_problem *P = (orc_problem *)h;
  memcpy(ox, P->ox, sizeof(double) * P->nv);
  memcpy(oy, P->oy, sizeof(double) * P->nv);
  memcpy(oz, P->oz, sizeof(double) * P->nv);
  memcpy(w, P->w, sizeof(double) * P->nv);
}
/* counters: steps, si_total, sweeps_total, nonconv, fallbacks, ig_updates,
 * pc_updates, n0, n1, flag_ig, flag_pc, rank_ig, rank_pc */
void orc_get_counters(void *h, int64_t *out) {
  orc_problem *P = (orc_problem *)h;
  out[0] = P->steps;
  out[1] = P->si_total;
  out[2] = P->sweeps_total;
  out[3] = P->nonconv;
  out[4] = P->fallbacks;
  out[5] = P->ig_updates;
  out[6] = P->pc_updates[0];
  out[7] = P->n0;
  out[8] = P->nl[0];
  out[9] = P->flag_ig;
  out[10] = P->flag_pc[0];
  out[11] = P->ig.rank;
  out[12] = P->pc[0].rank;
}
/* per correction level k < L: flag, N_k (steps its construction took),
 * rank, updates -- four values per level; returns L */
int orc_get_levels(void *h, int64_t *out) {
  orc_problem *P = (orc_problem *)h;
  for (int k = 0; k < P->nlev; ++k) {
    out[4 * k] = P->flag_pc[k];
    out[4 * k + 1] = P->nl[k];
    out[4 * k + 2] = P->pc[k].rank;
    out[4 * k + 3] = P->pc_updates[k];
  }
  return P->nlev;
}
int orc_get_history(void *h, orc_step_rec *out, int64_t n) {
  orc_problem *P = (orc_problem *)h;
  int64_t m = P->steps < n ? P->steps : n;
  if (m > P->hist_cap) m = P->hist_cap;
  memcpy(out, P->hist, sizeof(orc_step_rec) * m);
  return (int)m;
}
int orc_step_rec_size(void) { return (int)sizeof(orc_step_rec); }
int orc_desc_size(void) { return (int)sizeof(orc_desc); }

/* time-dependent inflow (test only): b~ for the next step is rebuilt with it */
void orc_set_inflow(void *h, const double *g) {
  orc_problem *P = (orc_problem *)h;
  for (int k = 0; k < 4; ++k) P->d.inflow[k] = g[k];
  compute_rhs(P, P->steps + 1, P->bt);
}
/* out = T Sigma_s rho (zero inflow) */
void orc_apply_TSs(void *h, const double *rho, double *out) {
  orc_problem *P = (orc_problem *)h;
  double *s = (double *)malloc(sizeof(double) * P->nc);
  for (int i = 0; i < P->nc; ++i) s[i] = P->ss[i] * rho[i];
  apply_T(P, s, out);
  free(s);
}
/* out = C^{-1} rhs with the DSA operator */
void orc_dsa_apply_inverse(void *h, const double *rhs, double *out) {
  dsa_solve((orc_problem *)h, rhs, out);
}
/* dense DSA matrix entry (for assembling it in tests) */
double orc_dsa_entry(void *h, int r, int c) { return dsa_matrix_entry((orc_problem *)h, r, c); }
/* one sweep of ordinate j with an arbitrary per-cell source */
void orc_sweep(void *h, int j, const double *s, int zero_inflow, double *out) {
  sweep_one((orc_problem *)h, j, s, zero_inflow, out);
}
/* rho^{(0)}, rho^{(1/2)}, delta rho^{(1)}_DMD and b~^{n-1} of the last step;
 * returns 1 if that step applied the ROM correction (eq. dmd-sa) */
int orc_get_step_vectors(void *h, double *rho0, double *rhalf, double *dpc, double *bt_prev) {
  orc_problem *P = (orc_problem *)h;
  size_t bytes = sizeof(double) * P->nc;
  memcpy(rho0, P->last_rho0, bytes);
  memcpy(rhalf, P->last_rhalf, bytes);
  memcpy(dpc, P->last_dpc, bytes);
  memcpy(bt_prev, P->last_bt, bytes);
  return P->last_used_pc;
}
/* the problem's ROM (which = 0: initial guess, k >= 1: correction level k): returns
 * its rank; U, W get rank columns of nc values each, S rank values */
int orc_get_rom(void *h, int which, double *U, double *S, double *W) {
  orc_problem *P = (orc_problem *)h;
  if (which < 0 || which > P->nlev) return 0;
  const orc_rom *m = which ? &P->pc[which - 1] : &P->ig;
  if (U) memcpy(U, m->U, sizeof(double) * (size_t)m->rank * m->nc);
  if (W) memcpy(W, m->W, sizeof(double) * (size_t)m->rank * m->nc);
  if (S) memcpy(S, m->S, sizeof(double) * m->rank);
  return m->rank;
}
