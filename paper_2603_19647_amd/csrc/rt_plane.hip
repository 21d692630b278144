// rt_plane.hip -- X-Y (2D) path of librtrom for gfx950.
//
// Ordinates: Omega_z = +-c pairs sweep identically in X-Y, so f is stored for
// the upper hemisphere only, each with its pair's doubled weight ("folded"
// set, nv / 2 ordinates).
//
// Sweep (Sec. 2.3: one upwind-ordered pass per ordinate): in upwind
// coordinates, f(a, b) = (s + m_x f(a-1, b) + m_y f(a, b-1)) / (sigma~_t +
// m_x + m_y) with m = |Omega| / h.  One workgroup per folded ordinate; one
// wave per band of 64 rows (lane = row), bands in flight on up to 16 waves.
// A wave runs a skewed pipeline across the columns: at step t, row j handles
// column t - j, the value from the row below arrives by a wave-wide DPP shift,
// and the band below hands its top row over through an LDS ring with
// producer / consumer counters (back-pressure keeps the ring bounded).  Cell
// data are prefetched PD steps ahead.  Each workgroup writes its ordinate's
// weighted flux to a per-ordinate partial; a reduce kernel adds the ordinates
// in a fixed order, so results are deterministic.
//
// DSA (eq. rho_residual) uses the cell-centred 5-point operator with
// Jacobi-preconditioned Chebyshev iteration on Gershgorin bounds: no dot
// products, a fixed iteration count for a 1e-14 error bound.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rt_host.h"
#include "rt_rom.h"

namespace {

constexpr int BAND = 64;   // rows of a band: one wave, lane = row
constexpr int MAXW = 16;   // bands in flight per workgroup (waves)
constexpr int RING = 256;  // columns buffered between consecutive bands
constexpr int PUB = 8;     // producers publish every PUB columns
constexpr int CPUB = 16;   // consumers publish every CPUB columns
constexpr int PD = 4;      // prefetch distance in steps (and loop unroll)
constexpr int BLK = 256;   // cells per block of the element-wise kernels

struct PlaneArgs {
  int nx, ny, nc, ndf, nbands, nw, nblk, pad_;
  double inv_dt;
  double g[4];
  const double *mx, *my, *w;  // per folded ordinate
  const int *sx, *sy;         // upwind signs per folded ordinate
  const double *ss, *ct, *G;
  double *f;                  // [ndf][nc]
  void *partial;              // [ndf][nc] of the sweep's partial type
  double *dummy;              // 128 doubles: stores of idle lanes
};

__device__ __forceinline__ double wave_shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ int lds_load(int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_publish(int *p, int v, bool writer) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // earlier LDS traffic complete
  if (writer) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// per-step prefetched cell data
template <typename R>
struct Slot {
  double ct, a1, a2, a3, a4;  // sigma~_t and the mode's other per-cell inputs
  R s;                        // MODE 0 source
  R fb, hb;                   // row-0 inputs from the band below
};

// MODE 0: SI sweep of the source src (zero inflow) -> per-ordinate w f.
// MODE 1: f-pass: final f^n (source sigma_s rho^n + G + f^{n-1}/dt, inflow g)
//         written over f, then the right-hand-side sweep (source f^n/dt + G,
//         inflow g) -> per-ordinate w h.
// MODE 2: right-hand-side sweep only, from the stored f.
template <typename R, int MODE>
__global__ void __launch_bounds__(1024) k_plane_sweep(PlaneArgs A, const R *__restrict__ src,
                                                      const double *__restrict__ rho) {
  constexpr int NF = MODE == 0 ? 1 : 2;
  typedef typename std::conditional<MODE == 0, R, double>::type PT;
  __shared__ R ring[MAXW][RING][NF];
  __shared__ int prod[MAXW], cons[MAXW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < MAXW) {
    prod[threadIdx.x] = 0;
    cons[threadIdx.x] = 0;
  }
  __syncthreads();
  const int NW = A.nw, nx = A.nx, ny = A.ny, nc = A.nc;
  const int dir = blockIdx.x;
  const int sx = A.sx[dir], sy = A.sy[dir];
  const R mx = (R)A.mx[dir], my = (R)A.my[dir], w = (R)A.w[dir];
  const double mxy = A.mx[dir] + A.my[dir];
  const R idt = (R)A.inv_dt;
  const R gx = MODE == 0 ? R(0) : (R)(sx > 0 ? A.g[0] : A.g[1]);
  const R gy = MODE == 0 ? R(0) : (R)(sy > 0 ? A.g[2] : A.g[3]);
  double *fdir = A.f + (size_t)dir * nc;
  PT *part = (PT *)A.partial + (size_t)dir * nc;
  double *dummy = A.dummy;
  const int wout = wv, win = (wv + NW - 1) % NW;
  int seen_prod = 0, seen_cons = 0;  // last counter values read (monotone)

  for (int band = wv; band < A.nbands; band += NW) {
    const int rows = min(BAND, ny - band * BAND);
    const bool rowok = lane < rows;
    const int b = band * BAND + lane;
    const int iy = sy > 0 ? b : ny - 1 - b;
    const int iyc = sy > 0 ? min(b, ny - 1) : max(ny - 1 - b, 0);  // clamped row for idle lanes
    const int c0 = iy * nx + (sx > 0 ? 0 : nx - 1);    // cell of column 0; column a at c0 + sx a
    const int cbase = iyc * nx + (sx > 0 ? 0 : nx - 1);
    const bool has_in = band > 0, has_out = band + 1 < A.nbands;
    const int pin0 = ((band - 1) / NW) * nx;          // ring positions of the band below
    const int pout0 = (band / NW) * nx;               // ring positions of this band

    // Every lane loads every step (clamped cell when idle) and every lane
    // stores every step (to a per-lane dummy when idle): the memory counter
    // then advances identically on all paths and the prefetched loads are
    // waited for individually.
    auto fetch = [&](Slot<R> &q, int t) {
      const int a = min(max(t - lane, 0), nx - 1);
      const int c = cbase + sx * a;
      q.ct = A.ct[c];
      if (MODE == 0) q.s = src[c];
      if (MODE == 1) {
        q.a1 = A.ss[c];
        q.a2 = rho[c];
        q.a3 = A.G[c];
        q.a4 = fdir[c];
      }
      if (MODE == 2) {
        q.a3 = A.G[c];
        q.a4 = fdir[c];
      }
      if (t < nx) {  // row-0 input of column t (uniform)
        if (has_in) {
          const int pos = pin0 + t;
          if (seen_prod <= pos) {
            while ((seen_prod = lds_load(&prod[win])) <= pos) __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          }
          if (lane == 0) {
            q.fb = ring[win][pos & (RING - 1)][0];
            if (NF == 2) q.hb = ring[win][pos & (RING - 1)][NF - 1];
          }
          if (((t + 1) % CPUB) == 0 || t == nx - 1) lds_publish(&cons[win], pos + 1, lane == 0);
        } else {
          q.fb = gy;
          q.hb = gy;
        }
      }
    };

    Slot<R> q[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k) {
      q[k] = Slot<R>{0.0, 0.0, 0.0, 0.0, 0.0, R(0), R(0), R(0)};
      fetch(q[k], k);
    }
    R fl = gx, hl = gx, fprev = R(0), hprev = R(0);
    // steps of the band, rounded up to the unroll (the extra steps are idle)
    const int T = ((nx + rows - 1 + PD - 1) / PD) * PD;
    for (int t0 = 0; t0 < T; t0 += PD) {
#pragma unroll
      for (int k = 0; k < PD; ++k) {
        const int t = t0 + k;
        const int a = t - lane;
        const bool on = rowok && a >= 0 && a < nx;
        R fb = wave_shr1(fprev), hb = NF == 2 ? wave_shr1(hprev) : R(0);
        if (lane == 0) {
          fb = q[k].fb;
          hb = q[k].hb;
        }
        const int c = c0 + sx * a;
        const R inv = rt_rcp((R)(q[k].ct + mxy));
        R f, h = R(0);
        PT v;
        if (MODE == 0) {
          f = (q[k].s + my * fb + mx * fl) * inv;
          v = (PT)(w * f);
        } else {
          if (MODE == 1) {
            const R s1 = (R)(rt_fma(q[k].a1, q[k].a2, q[k].a3) + q[k].a4 * A.inv_dt);
            f = (s1 + my * fb + mx * fl) * inv;
            *(on ? fdir + c : dummy + lane) = (double)f;
          } else {
            f = (R)q[k].a4;
          }
          const R s2 = rt_fma(f, idt, (R)q[k].a3);
          h = (s2 + my * hb + mx * hl) * inv;
          v = (PT)(w * h);
        }
        *(on ? part + c : (PT *)(dummy + 64) + lane) = v;
        if (!on) {
          f = R(0);
          h = R(0);
        } else {
          fl = f;
          hl = h;
        }
        fprev = f;
        hprev = h;
        // the top row finished column t - (BAND - 1): hand it to the band above
        const int ao = t - (BAND - 1);
        if (has_out && ao >= 0 && ao < nx) {
          const int pos = pout0 + ao;
          if (seen_cons < pos - RING + 1) {
            while ((seen_cons = lds_load(&cons[wout])) < pos - RING + 1) __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          }
          if (lane == BAND - 1) {
            ring[wout][pos & (RING - 1)][0] = f;
            if (NF == 2) ring[wout][pos & (RING - 1)][NF - 1] = h;
          }
          if (((ao + 1) % PUB) == 0 || ao == nx - 1) lds_publish(&prod[wout], pos + 1, lane == BAND - 1);
        }
        fetch(q[k], t + PD);
      }
    }
  }
}

// out[c] = sum over ordinates of partial[d][c] (+ add[c], or + out[c] when
// accumulating); optional per-block maxima for the stop test of Alg. 1:
// max|out - rp| and max|out|.
template <typename PT>
__global__ void __launch_bounds__(BLK) k_plane_reduce(PlaneArgs A, double *out, const double *add,
                                                      int accumulate, const double *rp, double *blkmax) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  double d = 0.0, y = 0.0;
  if (c < A.nc) {
    const PT *pp = (const PT *)A.partial + c;
    double s = 0.0;
    for (int g = 0; g < A.ndf; ++g) s += (double)pp[(size_t)g * A.nc];
    if (accumulate) s += out[c];
    else if (add) s += add[c];
    out[c] = s;
    y = fabs(s);
    if (rp) d = fabs(s - rp[c]);
  }
  if (blkmax) {
    __shared__ double red[2 * (BLK / 64)];
    d = wave_max(d);
    y = wave_max(y);
    if ((threadIdx.x & 63) == 0) {
      red[2 * (threadIdx.x >> 6)] = d;
      red[2 * (threadIdx.x >> 6) + 1] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, bb = 0.0;
      for (int w = 0; w < BLK / 64; ++w) {
        a = fmax(a, red[2 * w]);
        bb = fmax(bb, red[2 * w + 1]);
      }
      blkmax[2 * blockIdx.x] = a;
      blkmax[2 * blockIdx.x + 1] = bb;
    }
  }
}

// global maxima of the block maxima -> res[0] = ||y - rp||_inf, res[1] = ||y||_inf
__global__ void __launch_bounds__(256) k_plane_maxreduce(const double *blkmax, int nblk, double *res) {
  __shared__ double red[8];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    a = fmax(a, blkmax[2 * i]);
    b = fmax(b, blkmax[2 * i + 1]);
  }
  a = wave_max(a);
  b = wave_max(b);
  if ((threadIdx.x & 63) == 0) {
    red[2 * (threadIdx.x >> 6)] = a;
    red[2 * (threadIdx.x >> 6) + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      a = fmax(red[0], red[2 * w]);
      b = fmax(red[1], red[2 * w + 1]);
      red[0] = a;
      red[1] = b;
    }
    res[0] = red[0];
    res[1] = red[1];
  }
}

// element-wise helpers ------------------------------------------------------
// src = sigma_s * v (FP64)
__global__ void k_plane_src64(int nc, const double *ss, const double *v, double *src) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) src[c] = ss[c] * v[c];
}
// rn = y + d; src32 = (float)(sigma_s (rn - rp)); rp = rn
__global__ void k_plane_increment(int nc, const double *ss, const double *y, const double *d, double *rp,
                                  float *src32) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) {
    const double rn = y[c] + (d ? d[c] : 0.0);
    src32[c] = (float)(ss[c] * (rn - rp[c]));
    rp[c] = rn;
  }
}
// rp = y + d (d may be null)
__global__ void k_plane_correct(int nc, const double *y, const double *d, double *rp) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) rp[c] = y[c] + (d ? d[c] : 0.0);
}
__global__ void k_plane_copy(int nc, const double *a, double *b) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) b[c] = a[c];
}
// out = a - b
__global__ void k_plane_sub(int nc, const double *a, const double *b, double *out) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) out[c] = a[c] - b[c];
}

// DSA operator: A x = diag x - ax[c] x[c+1] - ax[c-1] x[c-1] - ay[c] x[c+nx] - ay[c-nx] x[c-nx]
struct DsaArgs {
  int nx, ny, nc;
  const double *diag, *ax, *ay;
};

__device__ __forceinline__ double dsa_Ax(const DsaArgs &D, const double *x, int c) {
  const int ix = c % D.nx, iy = c / D.nx;
  double v = D.diag[c] * x[c];
  if (ix + 1 < D.nx) v -= D.ax[c] * x[c + 1];
  if (ix > 0) v -= D.ax[c - 1] * x[c - 1];
  if (iy + 1 < D.ny) v -= D.ay[c] * x[c + D.nx];
  if (iy > 0) v -= D.ay[c - D.nx] * x[c - D.nx];
  return v;
}

// Chebyshev start: r = rhs = sigma_s (y - rp), x = 0, d0 = r / (theta diag)
__global__ void k_dsa_start(DsaArgs D, const double *ss, const double *y, const double *rp, double *r,
                            double *x, double *d, double inv_theta) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < D.nc) {
    const double rhs = ss[c] * (y[c] - rp[c]);
    r[c] = rhs;
    x[c] = 0.0;
    d[c] = inv_theta * rhs / D.diag[c];
  }
}
// one Chebyshev step: x += d; r -= A d; d' = c1 d + c2 r / diag
__global__ void k_dsa_step(DsaArgs D, double *x, double *r, const double *d, double *dn, double c1, double c2) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < D.nc) {
    const double dc = d[c];
    x[c] += dc;
    const double rn = r[c] - dsa_Ax(D, d, c);
    r[c] = rn;
    dn[c] = c1 * dc + c2 * rn / D.diag[c];
  }
}
__global__ void k_dsa_finish(int nc, double *x, const double *d) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) x[c] += d[c];
}

// setup: DSA coefficients (the same reading as the slab DSA, per face
// direction) and per-block Gershgorin ratios sum|offdiag| / diag
__global__ void k_plane_setup(DsaArgs D, const double *ct, const double *sa, double inv_dt, double hx, double hy,
                              double *diag, double *ax, double *ay, double *blkratio) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  double ratio = 0.0;
  if (c < D.nc) {
    const int nx = D.nx, ny = D.ny;
    const int ix = c % nx, iy = c / nx;
    auto Dx = [&](int i) { return 1.0 / (3.0 * ct[i]) + 0.25 * hx; };
    auto Dy = [&](int i) { return 1.0 / (3.0 * ct[i]) + 0.25 * hy; };
    auto face = [&](double Dp, double Dq, double h) { return 2.0 * Dp * Dq / (h * (Dp + Dq)); };
    auto bdry = [&](double Dp, double h) { return 2.0 * Dp / (h + 4.0 * Dp); };
    const double dxp = Dx(c), dyp = Dy(c);
    const double kl = ix > 0 ? face(dxp, Dx(c - 1), hx) : bdry(dxp, hx);
    const double kr = ix + 1 < nx ? face(dxp, Dx(c + 1), hx) : bdry(dxp, hx);
    const double kb = iy > 0 ? face(dyp, Dy(c - nx), hy) : bdry(dyp, hy);
    const double kt = iy + 1 < ny ? face(dyp, Dy(c + nx), hy) : bdry(dyp, hy);
    const double dg = sa[c] + inv_dt + (kl + kr) / hx + (kb + kt) / hy;
    diag[c] = dg;
    ax[c] = ix + 1 < nx ? kr / hx : 0.0;
    ay[c] = iy + 1 < ny ? kt / hy : 0.0;
    double off = 0.0;
    if (ix > 0) off += kl / hx;
    if (ix + 1 < nx) off += kr / hx;
    if (iy > 0) off += kb / hy;
    if (iy + 1 < ny) off += kt / hy;
    ratio = off / dg;
  }
  ratio = wave_max(ratio);
  __shared__ double red[BLK / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ratio;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < BLK / 64; ++w) m = fmax(m, red[w]);
    blkratio[blockIdx.x] = m;
  }
}

// per-step status for the ROM kernels and the counters
__global__ void k_plane_status(RtState *st, int iters, int conv, int used_pc, int ig_fb, int pc_fb, double resid,
                               int n32) {
  st->iters = iters;
  st->conv = conv;
  st->used_pc = used_pc;
  st->ig_fb = ig_fb;
  st->pc_fb = pc_fb;
  st->residual = resid;
  st->phase = !st->flag_ig ? 1 : (!st->flag_pc ? 2 : 3);
  st->cur = (int)(st->steps & 1);
  st->fp32_sweeps += n32;
}

// DMD solve over the grid: coefficient partials, one-workgroup LU solve,
// expansion (eq. dmd-ig, eq. dmd-sa) for a large instance.
__global__ void __launch_bounds__(BLK) k_romapply_coef(RomDev R, const int *rankp, int ld, int nc,
                                                      const double *rhs, double *part) {
  const int rank = *rankp;
  const int c = blockIdx.x * BLK + threadIdx.x;
  double p[RT_RMAX];
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) p[k] = 0.0;
  if (c < nc) {
    const double v = rhs[c];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k)
      if (k < rank) p[k] = R.U[(size_t)k * ld + c] * v;
  }
  __shared__ double red[(BLK / 64) * RT_RMAX], out[RT_RMAX];
  wg_sum_fast<RT_RMAX>(p, red, out);
  if (threadIdx.x < RT_RMAX) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
__global__ void __launch_bounds__(256) k_romapply_solve(RomDev R, const int *rankp, int nblk, const double *part,
                                                        double *coef) {
  const int rank = *rankp;
  __shared__ double vec[RT_RMAX];
  if ((int)threadIdx.x < rank) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b * RT_NPART + threadIdx.x];
    vec[threadIdx.x] = s;
  }
  __syncthreads();
  lu_solve_wave(R.LU, R.perm, rank, vec);  // ends with a barrier
  if ((int)threadIdx.x < rank) coef[threadIdx.x] = vec[threadIdx.x];
}
__global__ void __launch_bounds__(BLK) k_romapply_expand(RomDev R, const int *rankp, int ld, int nc,
                                                        const double *coef, double *out) {
  const int rank = *rankp;
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) {
    double v = 0.0;
    for (int k = 0; k < rank; ++k) v = rt_fma(R.U[(size_t)k * ld + c], coef[k], v);
    out[c] = v;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct PlaneHost {
  PlaneArgs A;
  DsaArgs D;
  int ndf = 0;                    // folded ordinates (nv / 2)
  std::vector<int> fold_of;       // ordinate -> folded index
  double *dmx = nullptr;          // device: mx, my, w
  int *dsign = nullptr;           // device: sx, sy
  double *partial = nullptr;
  double *y = nullptr, *rp = nullptr, *src = nullptr, *dvec = nullptr;
  float *src32 = nullptr;
  double *cr = nullptr, *cx = nullptr, *cd0 = nullptr, *cd1 = nullptr;
  double *diag = nullptr, *ax = nullptr, *ay = nullptr;
  double *fbuf = nullptr;
  double *blkmax = nullptr, *res = nullptr, *res_h = nullptr;
  double *rpart = nullptr, *rcoef = nullptr;
  int cheb_iters = 0;
  double cheb_theta = 1.0, cheb_delta = 0.0;
  std::vector<double> cheb_c1, cheb_c2;
  size_t bytes = 0;
};

static size_t plane_bytes_for(const rtrom_problem_desc *d, int *ndf_out) {
  const size_t nv = (size_t)d->n_polar * d->n_azim;
  const int ndf = (int)(nv / 2);
  const size_t nc = (size_t)d->nx * d->ny;
  const size_t nblk = (nc + BLK - 1) / BLK;
  if (ndf_out) *ndf_out = ndf;
  size_t b = 0;
  auto take = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  take((size_t)ndf * nc * 8);                              // per-ordinate partials
  take(nc * 8 * 8);                                        // y rp src dvec cr cx cd0 cd1
  take(nc * 4);                                            // src32
  take(nc * 8 * 3);                                        // diag ax ay
  take(nblk * 2 * 8 + 64);                                 // blkmax, res
  take(nblk * RT_NPART * 8 + RT_RMAX * 8);                 // rom apply partials, coef
  take((size_t)ndf * 3 * 8 + (size_t)ndf * 2 * 4);         // mx my w, sx sy
  take(128 * 8);                                           // idle-lane store target
  return b;
}

size_t rt_plane_extra_bytes(const rtrom_problem_desc *d) { return plane_bytes_for(d, nullptr); }

// Largest nx for grids with more bands than waves: the bands then cycle
// through the waves, and the band-to-band rings (RING columns, consumers
// publishing every CPUB) must drain before a wave moves to its next band.
int rt_plane_max_nx_cyclic() { return MAXW * (RING - CPUB); }
int rt_plane_needs_cyclic(int ny) { return (ny + BAND - 1) / BAND > MAXW; }

#define PH(call)                                                            \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      rt_set_error(std::string("plane: ") + hipGetErrorString(e_));         \
      return RTROM_EDEVICE;                                                 \
    }                                                                       \
  } while (0)

template <typename PT>
static void launch_reduce(rtrom_problem *p, PlaneHost *H, double *out, const double *add, int accumulate,
                          const double *rp, double *blkmax) {
  hipLaunchKernelGGL((k_plane_reduce<PT>), dim3(H->A.nblk), dim3(BLK), 0, p->stream, H->A, out, add, accumulate,
                     rp, blkmax);
}

static int launch_sweep(rtrom_problem *p, PlaneHost *H, int mode, int fp32, const void *src, const double *rho) {
  PlaneArgs &A = H->A;
  const dim3 grid(A.ndf), block(64 * A.nw);
  hipStream_t s = p->stream;
  if (mode == 0 && fp32)
    hipLaunchKernelGGL((k_plane_sweep<float, 0>), grid, block, 0, s, A, (const float *)src, rho);
  else if (mode == 0)
    hipLaunchKernelGGL((k_plane_sweep<double, 0>), grid, block, 0, s, A, (const double *)src, rho);
  else if (mode == 1)
    hipLaunchKernelGGL((k_plane_sweep<double, 1>), grid, block, 0, s, A, (const double *)nullptr, rho);
  else
    hipLaunchKernelGGL((k_plane_sweep<double, 2>), grid, block, 0, s, A, (const double *)nullptr, rho);
  PH(hipGetLastError());
  return RTROM_OK;
}

int rt_plane_create(rtrom_problem *p) {
  const rtrom_problem_desc *d = &p->d;
  PlaneHost *H = new PlaneHost();
  p->plane = H;
  int ndf;
  H->bytes = plane_bytes_for(d, &ndf);
  H->ndf = ndf;
  const int nx = d->nx, ny = d->ny, nc = nx * ny;
  const int nblk = (nc + BLK - 1) / BLK;
  const int nbands = (ny + BAND - 1) / BAND;
  if (nbands > MAXW && nx > rt_plane_max_nx_cyclic()) {
    rt_set_error("plane: grids with more than 1024 rows are limited to nx <= 3840");
    return RTROM_EINVAL;
  }
  // folded ordinates: the upper hemisphere (Omega_z > 0) in ordinate order;
  // Omega_z < 0 ordinates map to their mirror at the same azimuth
  const int nphi = d->n_azim, nz = d->n_polar;
  const double hx = d->lx / nx, hy = d->ly / ny;
  std::vector<double> hm(3 * (size_t)ndf, 0.0);
  std::vector<int> hs(2 * (size_t)ndf, 1);
  H->fold_of.assign((size_t)nphi * nz, -1);
  int nf = 0;
  for (int j2 = 0; j2 < nz; ++j2)
    for (int j1 = 0; j1 < nphi; ++j1) {
      const int j = j2 * nphi + j1;
      if (p->oz[j] > 0) {
        const int idx = nf++;
        hm[idx] = std::fabs(p->ox[j]) / hx;
        hm[ndf + idx] = std::fabs(p->oy[j]) / hy;
        hm[2 * (size_t)ndf + idx] = 2.0 * p->w[j];
        hs[idx] = p->ox[j] > 0 ? 1 : -1;
        hs[ndf + idx] = p->oy[j] > 0 ? 1 : -1;
        H->fold_of[j] = idx;
      }
    }
  if (nf != ndf) {
    rt_set_error("plane: quadrature is not symmetric in Omega_z");
    return RTROM_EINVAL;
  }
  for (int j2 = 0; j2 < nz; ++j2)
    for (int j1 = 0; j1 < nphi; ++j1) {
      const int j = j2 * nphi + j1;
      if (p->oz[j] < 0) H->fold_of[j] = H->fold_of[(size_t)(nz - 1 - j2) * nphi + j1];
    }
  // device buffers
  char *mem = nullptr;
  PH(hipMalloc(&mem, H->bytes));
  PH(hipMemsetAsync(mem, 0, H->bytes, p->stream));
  size_t off = 0;
  auto take = [&](size_t x) {
    char *q = mem + off;
    off += (x + 255) & ~size_t(255);
    return q;
  };
  H->partial = (double *)take((size_t)ndf * nc * 8);
  char *vecs = take((size_t)nc * 8 * 8);
  H->y = (double *)vecs;
  H->rp = H->y + nc;
  H->src = H->rp + nc;
  H->dvec = H->src + nc;
  H->cr = H->dvec + nc;
  H->cx = H->cr + nc;
  H->cd0 = H->cx + nc;
  H->cd1 = H->cd0 + nc;
  H->src32 = (float *)take((size_t)nc * 4);
  H->diag = (double *)take((size_t)nc * 8 * 3);
  H->ax = H->diag + nc;
  H->ay = H->ax + nc;
  H->blkmax = (double *)take((size_t)nblk * 2 * 8 + 64);
  H->res = H->blkmax + 2 * (size_t)nblk;
  H->rpart = (double *)take((size_t)nblk * RT_NPART * 8 + RT_RMAX * 8);
  H->rcoef = H->rpart + (size_t)nblk * RT_NPART;
  H->dmx = (double *)take((size_t)ndf * 3 * 8 + (size_t)ndf * 2 * 4);
  H->dsign = (int *)(H->dmx + 3 * (size_t)ndf);
  double *dummy = (double *)take(128 * 8);
  Inst &I = p->hinst;
  H->fbuf = I.f;  // f^n of the folded set lives in the first nv/2 ordinate slots
  PH(hipMemcpyAsync(H->dmx, hm.data(), hm.size() * 8, hipMemcpyHostToDevice, p->stream));
  PH(hipMemcpyAsync(H->dsign, hs.data(), hs.size() * 4, hipMemcpyHostToDevice, p->stream));
  PH(hipHostMalloc((void **)&H->res_h, 64, hipHostMallocDefault));
  PlaneArgs &A = H->A;
  memset(&A, 0, sizeof(A));
  A.nx = nx;
  A.ny = ny;
  A.nc = nc;
  A.ndf = ndf;
  A.nbands = nbands;
  A.nw = std::min(nbands, MAXW);
  A.nblk = nblk;
  A.inv_dt = 1.0 / d->dt;
  for (int k = 0; k < 4; ++k) A.g[k] = d->inflow[k];
  A.mx = H->dmx;
  A.my = H->dmx + ndf;
  A.w = H->dmx + 2 * (size_t)ndf;
  A.sx = H->dsign;
  A.sy = H->dsign + ndf;
  A.ss = I.ss;
  A.ct = I.ct;
  A.G = I.G;
  A.f = H->fbuf;
  A.partial = H->partial;
  A.dummy = dummy;
  double *fbuf = H->fbuf;
  // f^0 (isotropic) on every folded ordinate: rebuild from rho
  for (int j = 0; j < ndf; ++j)
    PH(hipMemcpyAsync(fbuf + (size_t)j * nc, I.rho, (size_t)nc * 8, hipMemcpyDeviceToDevice, p->stream));
  // DSA setup and Chebyshev parameters
  H->D.nx = nx;
  H->D.ny = ny;
  H->D.nc = nc;
  H->D.diag = H->diag;
  H->D.ax = H->ax;
  H->D.ay = H->ay;
  hipLaunchKernelGGL(k_plane_setup, dim3(nblk), dim3(BLK), 0, p->stream, H->D, I.ct, I.sa, 1.0 / d->dt,
                     hx, hy, H->diag, H->ax, H->ay, H->blkmax);
  PH(hipGetLastError());
  std::vector<double> ratios(nblk);
  PH(hipMemcpyAsync(ratios.data(), H->blkmax, nblk * 8, hipMemcpyDeviceToHost, p->stream));
  PH(hipStreamSynchronize(p->stream));
  double gmax = 0.0;
  for (double r : ratios) gmax = std::max(gmax, r);
  // eigenvalues of diag^{-1} A lie in [1 - g, 1 + g] (Gershgorin, strict
  // diagonal dominance because sigma_a + 1/dt > 0)
  const double lmin = std::max(1e-12, 1.0 - gmax), lmax = 1.0 + gmax;
  H->cheb_theta = 0.5 * (lmax + lmin);
  H->cheb_delta = 0.5 * (lmax - lmin);
  const double sigma1 = H->cheb_theta / std::max(H->cheb_delta, 1e-300);
  int K = 1;
  if (H->cheb_delta > 0.0) {
    // error bound 2 / T_K(sigma1) <= 1e-14
    K = (int)std::ceil(std::acosh(2e14) / std::acosh(sigma1));
    K = std::max(1, std::min(K, 2000));
  }
  H->cheb_iters = K;
  // coefficients of d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) diag^{-1} r_{k+1}
  H->cheb_c1.assign(K, 0.0);
  H->cheb_c2.assign(K, 0.0);
  double rho_k = 1.0 / sigma1;
  for (int k = 0; k < K; ++k) {
    const double rho_n = 1.0 / (2.0 * sigma1 - rho_k);
    H->cheb_c1[k] = rho_n * rho_k;
    H->cheb_c2[k] = H->cheb_delta > 0.0 ? 2.0 * rho_n / H->cheb_delta : 0.0;
    rho_k = rho_n;
  }
  // b~^0 from f^0
  return rt_plane_rhs(p);
}

void rt_plane_destroy(rtrom_problem *p) {
  PlaneHost *H = (PlaneHost *)p->plane;
  if (!H) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (H->partial) (void)hipFree(H->partial);
  if (H->res_h) (void)hipHostFree(H->res_h);
  delete H;
  p->plane = nullptr;
}

int rt_plane_rhs(rtrom_problem *p) {
  PlaneHost *H = (PlaneHost *)p->plane;
  for (int k = 0; k < 4; ++k) H->A.g[k] = p->d.inflow[k];
  const int nblk = H->A.nblk;
  int e = launch_sweep(p, H, 2, 0, nullptr, p->hinst.rho);
  if (e) return e;
  launch_reduce<double>(p, H, p->hinst.bt2[p->steps & 1], nullptr, 0, nullptr, nullptr);
  PH(hipGetLastError());
  return RTROM_OK;
}

static int dsa_solve(rtrom_problem *p, PlaneHost *H, const double *y, const double *rp, double *out) {
  const int nblk = H->A.nblk, nc = H->A.nc;
  hipStream_t s = p->stream;
  hipLaunchKernelGGL(k_dsa_start, dim3(nblk), dim3(BLK), 0, s, H->D, p->hinst.ss, y, rp, H->cr, H->cx, H->cd0,
                     1.0 / H->cheb_theta);
  double *d0 = H->cd0, *d1 = H->cd1;
  for (int k = 0; k < H->cheb_iters; ++k) {
    hipLaunchKernelGGL(k_dsa_step, dim3(nblk), dim3(BLK), 0, s, H->D, H->cx, H->cr, (const double *)d0, d1,
                       H->cheb_c1[k], H->cheb_c2[k]);
    std::swap(d0, d1);
  }
  hipLaunchKernelGGL(k_dsa_finish, dim3(nblk), dim3(BLK), 0, s, nc, H->cx, (const double *)d0);
  (void)out;
  PH(hipGetLastError());
  return RTROM_OK;
}

static int rom_apply_grid(rtrom_problem *p, PlaneHost *H, const RomDev &R, const int *rank_dev,
                          const double *rhs, double *out) {
  const int nblk = H->A.nblk, nc = H->A.nc;
  hipStream_t s = p->stream;
  hipLaunchKernelGGL(k_romapply_coef, dim3(nblk), dim3(BLK), 0, s, R, rank_dev, p->hinst.ld, nc, rhs, H->rpart);
  hipLaunchKernelGGL(k_romapply_solve, dim3(1), dim3(256), 0, s, R, rank_dev, nblk, (const double *)H->rpart,
                     H->rcoef);
  hipLaunchKernelGGL(k_romapply_expand, dim3(nblk), dim3(BLK), 0, s, R, rank_dev, p->hinst.ld, nc,
                     (const double *)H->rcoef, out);
  PH(hipGetLastError());
  return RTROM_OK;
}

// residual of the current y against rp: returns ||y - rp||_inf, ||y||_inf
static int read_residual(rtrom_problem *p, PlaneHost *H, double *dn, double *yn) {
  hipLaunchKernelGGL(k_plane_maxreduce, dim3(1), dim3(256), 0, p->stream, (const double *)H->blkmax, H->A.nblk,
                     H->res);
  PH(hipGetLastError());
  PH(hipMemcpyAsync(H->res_h, H->res, 16, hipMemcpyDeviceToHost, p->stream));
  PH(hipStreamSynchronize(p->stream));
  *dn = H->res_h[0];
  *yn = H->res_h[1];
  return RTROM_OK;
}

static int plane_one_step(rtrom_problem *p, PlaneHost *H) {
  Inst &I = p->hinst;
  const int nc = H->A.nc, nblk = H->A.nblk;
  hipStream_t s = p->stream;
  // state needed for this step's decisions
  RtState st;
  PH(hipMemcpyAsync(&st, I.st, sizeof(RtState), hipMemcpyDeviceToHost, s));
  PH(hipStreamSynchronize(s));
  const int rom = (I.method == RT_ROM);
  const int mixed = (I.precision == RT_MIXED);
  const int cur = (int)(st.steps & 1);
  const double *bt = I.bt2[cur];
  int ig_fb = 0;
  if (rom && st.flag_ig && st.lu_ok_ig) {
    rt_prof_begin(RT_K_PLANE_OTHER, s);
    int e = rom_apply_grid(p, H, I.ig, &I.st->rank_ig, bt, I.rho0);
    rt_prof_end(RT_K_PLANE_OTHER, s);
    if (e) return e;
  } else {
    ig_fb = rom && st.flag_ig;
    hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)I.rho, I.rho0);
  }
  hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)I.rho0, H->rp);
  int nsweep = 0, n32 = 0, conv = 0, used_pc = 0, pc_fb = 0, exact = 0, first_corr = 1, need64 = 1;
  double resid = 0.0;
  for (;;) {
    if (need64) {
      rt_prof_begin(RT_K_PLANE_SWEEP, s);
      hipLaunchKernelGGL(k_plane_src64, dim3(nblk), dim3(BLK), 0, s, nc, I.ss, (const double *)H->rp, H->src);
      int e = launch_sweep(p, H, 0, 0, H->src, nullptr);
      if (e) return e;
      launch_reduce<double>(p, H, H->y, bt, 0, H->rp, H->blkmax);
      rt_prof_end(RT_K_PLANE_SWEEP, s);
      if (nsweep == 0)
        hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, I.rhalf);
      nsweep++;
      exact = 1;
      need64 = 0;
    }
    double dn, yn;
    int e = read_residual(p, H, &dn, &yn);
    if (e) return e;
    resid = yn > 0.0 ? dn / yn : dn;
    const bool pass = yn > 0.0 ? (dn < I.tol * yn) : (dn < I.tol);
    if (pass) {
      if (exact) {
        conv = 1;
        break;
      }
      if (nsweep >= I.max_iter) break;
      need64 = 1;
      continue;
    }
    if (nsweep >= I.max_iter) break;
    const double *dcorr = nullptr;
    if (rom && first_corr && st.flag_pc && st.lu_ok_pc) {
      rt_prof_begin(RT_K_PLANE_OTHER, s);
      hipLaunchKernelGGL(k_plane_sub, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y,
                         (const double *)I.rho0, I.work);
      e = rom_apply_grid(p, H, I.pc, &I.st->rank_pc, I.work, I.dpc);
      rt_prof_end(RT_K_PLANE_OTHER, s);
      if (e) return e;
      dcorr = I.dpc;
      used_pc = 1;
    } else if (I.method != RT_SI_PLAIN) {
      if (rom && first_corr && st.flag_pc) pc_fb = 1;
      rt_prof_begin(RT_K_PLANE_DSA, s);
      e = dsa_solve(p, H, H->y, H->rp, nullptr);
      rt_prof_end(RT_K_PLANE_DSA, s);
      if (e) return e;
      dcorr = H->cx;
    }
    first_corr = 0;
    if (mixed) {
      rt_prof_begin(RT_K_PLANE_SWEEP, s);
      hipLaunchKernelGGL(k_plane_increment, dim3(nblk), dim3(BLK), 0, s, nc, I.ss, (const double *)H->y, dcorr,
                         H->rp, H->src32);
      e = launch_sweep(p, H, 0, 1, H->src32, nullptr);
      if (e) return e;
      launch_reduce<float>(p, H, H->y, nullptr, 1, H->rp, H->blkmax);
      rt_prof_end(RT_K_PLANE_SWEEP, s);
      exact = 0;
      n32++;
      nsweep++;
    } else {
      hipLaunchKernelGGL(k_plane_correct, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, dcorr, H->rp);
      need64 = 1;
    }
  }
  hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, I.rho);
  hipLaunchKernelGGL(k_plane_status, dim3(1), dim3(1), 0, s, I.st, nsweep, conv, used_pc, ig_fb, pc_fb, resid, n32);
  PH(hipGetLastError());
  // ROM bookkeeping on the auxiliary stream, concurrent with the f-pass
  hipStream_t s2 = rom ? p->aux_stream : s;
  if (s2 != s) {
    PH(hipEventRecord(p->ev_si, s));
    PH(hipStreamWaitEvent(s2, p->ev_si, 0));
  }
  rt_prof_begin(RT_K_POST, s2);
  PH(rt_launch_rom(p->dinst, 1, nc, rom, s2));
  rt_prof_end(RT_K_POST, s2);
  if (rom) {
    rt_prof_begin(RT_K_ROM_UPDATE, s2);
    PH(rt_launch_rom_update(p->dinst, 1, nc, s2));
    rt_prof_end(RT_K_ROM_UPDATE, s2);
  }
  rt_prof_begin(RT_K_PLANE_FPASS, s);
  {
    int e = launch_sweep(p, H, 1, 0, nullptr, I.rho);
    if (e) return e;
    launch_reduce<double>(p, H, I.bt2[cur ^ 1], nullptr, 0, nullptr, nullptr);
    PH(hipGetLastError());
  }
  rt_prof_end(RT_K_PLANE_FPASS, s);
  if (s2 != s) {
    PH(hipEventRecord(p->ev_rom, s2));
    PH(hipStreamWaitEvent(s, p->ev_rom, 0));
  }
  return RTROM_OK;
}

int rt_plane_step(rtrom_problem *p, int nsteps) {
  PlaneHost *H = (PlaneHost *)p->plane;
  for (int k = 0; k < nsteps; ++k) {
    int e = plane_one_step(p, H);
    if (e) return e;
  }
  return RTROM_OK;
}

// folded f -> CL-ordered f for rtrom_get_angular_flux
int rt_plane_unfold(const rtrom_problem *p, double *f_host) {
  const PlaneHost *H = (const PlaneHost *)p->plane;
  const size_t nc = (size_t)p->nc;
  std::vector<double> tmp((size_t)H->ndf * nc);
  PH(hipMemcpyAsync(tmp.data(), H->fbuf, tmp.size() * 8, hipMemcpyDeviceToHost, p->stream));
  PH(hipStreamSynchronize(p->stream));
  for (int j = 0; j < p->nv; ++j) memcpy(f_host + (size_t)j * nc, tmp.data() + (size_t)H->fold_of[j] * nc, nc * 8);
  return RTROM_OK;
}
