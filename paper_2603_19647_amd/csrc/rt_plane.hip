// rt_plane.hip -- X-Y (2D) path of librtrom for gfx950.
//
// Ordinates: Omega_z = +-c pairs sweep identically in X-Y, so f is kept for
// the upper hemisphere only, each with its pair's doubled weight ("folded"
// set, nv / 2 ordinates), grouped by upwind quadrant.
//
// Sweep (Sec. 2.3: one upwind-ordered pass per ordinate): in upwind
// coordinates (column a, row u), f(a, u) = (s + m_x f(a-1, u) + m_y f(a, u-1))
// / (sigma~_t + m_x + m_y) with m = |Omega| / h.  One workgroup per folded
// ordinate, one wave per band of 64 rows (lane = row), up to 16 bands in
// flight.  A wave runs a skewed pipeline: at step t, row j handles column
// t - j; the row below arrives by a wave-wide DPP shift and the band below
// hands its top row over through an LDS ring with producer / consumer
// counters (back-pressure keeps the ring bounded).
//
// Skewed layout: every per-cell array a sweep touches is stored, per upwind
// quadrant, at slot ((band * TT) + t) * 64 + j -- the order in which the
// pipeline visits cells -- so each step of a wave reads and writes 64
// consecutive elements.  Slots outside the grid are padding: idle lanes load
// and store there, which keeps every lane's memory traffic identical and the
// prefetched loads individually waited for.  Per-cell inputs are skewed by
// small gather kernels; per-ordinate results are summed per quadrant in the
// skewed layout and un-skewed once, in a fixed order (deterministic).
//
// DSA (eq. rho_residual) uses the cell-centred 5-point operator with
// Jacobi-preconditioned Chebyshev iteration on Gershgorin bounds: no dot
// products, a fixed iteration count for a 1e-14 error bound.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "rt_host.h"
#include "rt_mh.h"
#include "rt_rom.h"

// Chebyshev iterations the 2D DSA solve may take (its coefficient table is
// sized for them); a problem needing more is rejected at creation.
#define RT_CHEB_MAX 20000

namespace {

constexpr int BAND = 64;   // rows of a band: one wave, lane = row
constexpr int MAXW = 16;   // bands in flight per workgroup (waves)
constexpr int RING = 256;  // columns buffered between consecutive bands
constexpr int CH = 16;     // columns per ring transfer; the step loop is unrolled by CH
constexpr int BLK = 256;   // cells per block of the element-wise kernels

struct PlaneArgs {
  int nx, ny, nc, ndf, nbands, nw, nblk, TT;  // TT: skewed steps per band
  int SQ, nsblk;                              // slots per quadrant, blocks over SQ
  int qstart[5];                              // folded ordinates of quadrant q: [qstart[q], qstart[q+1])
  double inv_dt;
  double g[4];
  const double *mx, *my, *w;  // per folded ordinate
  const double *ctq, *Gq;     // [4][SQ] sigma~_t, G (skewed)
  const float *ctf;           // [4][SQ] sigma~_t in FP32 (skewed)
  double *s1q;                // [4][SQ] sigma_s rho^n + G (skewed, f-pass)
  void *srcq;                 // [4][SQ] SI sweep source (skewed, sweep type)
  double *f;                  // [ndf][SQ] folded f, skewed in its quadrant
  double *fo;                 // BDF2: [ndf][SQ] the older level f^{n-1} (null otherwise)
  void *partial;              // [ndf][SQ] w f per ordinate (skewed)
  double *quadsum;            // [4][SQ] per-quadrant sums (skewed)
};

__device__ __forceinline__ int quad_of(int dir, const PlaneArgs &A) {
  return (dir >= A.qstart[1]) + (dir >= A.qstart[2]) + (dir >= A.qstart[3]);
}
// quadrant q: bit 0 set when the sweep runs in -x, bit 1 when in -y
__device__ __forceinline__ int slot_cell(const PlaneArgs &A, int q, int slot) {
  const int per_band = A.TT * BAND;
  const int band = slot / per_band, rem = slot - band * per_band;
  const int t = rem >> 6, j = rem & 63;
  const int u = band * BAND + j, a = t - j;
  if (u >= A.ny || a < 0 || a >= A.nx) return -1;
  const int iy = (q & 2) ? A.ny - 1 - u : u;
  const int ix = (q & 1) ? A.nx - 1 - a : a;
  return iy * A.nx + ix;
}
__device__ __forceinline__ int cell_slot(const PlaneArgs &A, int q, int ix, int iy) {
  const int u = (q & 2) ? A.ny - 1 - iy : iy;
  const int a = (q & 1) ? A.nx - 1 - ix : ix;
  const int band = u >> 6, j = u & 63;
  return (band * A.TT + a + j) * BAND + j;
}

// lane i gets v of lane i-1; lane 0 gets in0
__device__ __forceinline__ double shr1_in(double v, double in0) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(in0), __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(in0), __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float shr1_in(float v, float in0) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(in0), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
// wave rotations: rol1 -- lane i gets lane i+1 (lane 63 gets lane 0);
// ror1 -- lane i gets lane i-1 (lane 0 gets lane 63)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true),
                          __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <typename R>
__device__ __forceinline__ R rol1(R v) { return dpp_mov<0x134>(v); }
template <typename R>
__device__ __forceinline__ R ror1(R v) { return dpp_mov<0x13C>(v); }
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
  R ct;                   // sigma~_t
  double a1, a2, a3, a4;  // the mode's other per-cell inputs (a4: BDF2's older level)
  R s;                    // MODE 0 source
};

// MODE 0: SI sweep of the source srcq (zero inflow) -> per-ordinate w f.
// MODE 1: f-pass: final f^n (source sigma_s rho^n + G + f^{n-1}/dt, inflow g)
//         written over f, then the right-hand-side sweep (source f^n/dt + G,
//         inflow g) -> per-ordinate w h.
// MODE 2: right-hand-side sweep only, from the stored f.
// MODE 3: the BDF2 f-pass (Sec. 2.1's BDF alternative): f^n from the source
//         sigma_s rho^n + G + (4 f^{n-1} - f^{n-2}) / (2 dt), with f^{n-1} in
//         f and f^{n-2} in fo, written over fo (the caller then swaps f and
//         fo), then the right-hand side of the next step from the source
//         (4 f^n - f^{n-1}) / (2 dt) + G.
// MODE 4: the BDF2 right-hand-side sweep only, from f (f^n) and fo (f^{n-1}).
// The operator (sigma~_t in ctq / ctf) is the caller's: 1/dt or 3/(2 dt).
// Ring traffic moves CH columns at a time: the top row's values are gathered
// into lanes 0..CH-1 of a register, the consumer reads a chunk into lanes
// 0..CH-1 and feeds its lane 0 with readlane.
template <typename R, int MODE, int PD>
__global__ void __launch_bounds__(1024) k_plane_sweep(PlaneArgs A) {
  static_assert(CH % PD == 0, "prefetch slots rotate within a chunk");
  constexpr int NF = MODE == 0 ? 1 : 2;
  constexpr bool FP = MODE == 1 || MODE == 3;  // computes f^n
  constexpr bool RH = MODE == 2 || MODE == 4;  // right-hand side from the stored f
  constexpr bool B2 = MODE >= 3;               // BDF2 history
  typedef typename std::conditional<MODE == 0, R, double>::type PT;
  __shared__ R ring[MAXW][RING][NF];
  __shared__ int prod[MAXW], cons[MAXW];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  if (threadIdx.x < MAXW) {
    prod[threadIdx.x] = 0;
    cons[threadIdx.x] = 0;
  }
  __syncthreads();
  const int NW = A.nw, nx = A.nx, ny = A.ny;
  const unsigned unx = (unsigned)nx;
  const int dir = blockIdx.x;
  const int q = quad_of(dir, A);
  const R mx = (R)A.mx[dir], my = (R)A.my[dir], w = (R)A.w[dir];
  const double mxy = A.mx[dir] + A.my[dir];
  const R idt = (R)A.inv_dt;
  const R gx = MODE == 0 ? R(0) : (R)((q & 1) ? A.g[1] : A.g[0]);
  const R gy = MODE == 0 ? R(0) : (R)((q & 2) ? A.g[3] : A.g[2]);
  const size_t qoff = (size_t)q * A.SQ, doff = (size_t)dir * A.SQ;
  const double *ctq = A.ctq + qoff, *Gq = A.Gq + qoff, *s1q = A.s1q + qoff;
  const float *ctf = A.ctf + qoff;
  const R mxyr = (R)mxy;
  const R *srcq = (const R *)A.srcq + qoff;
  double *fd = A.f + doff;
  double *fod = B2 ? A.fo + doff : nullptr;
  const double hdt = 0.5 * A.inv_dt;  // 1 / (2 dt)
  PT *part = (PT *)A.partial + doff;
  const int wout = wv, win = (wv + NW - 1) % NW;
  int seen_prod = 0, seen_cons = 0;  // last counter values read (monotone)

  for (int band = wv; band < A.nbands; band += NW) {
    const int rows = min(BAND, ny - band * BAND);
    const bool rowok = lane < rows;
    const bool has_in = band > 0, has_out = band + 1 < A.nbands;
    const int pin0 = ((band - 1) / NW) * nx;   // ring positions of the band below
    const int pout0 = (band / NW) * nx;        // ring positions of this band
    const int sbase = band * A.TT * BAND + lane;  // slot of step 0

    // per-lane pointers at step 0 of the band; step t is t * BAND further
    const R *srcb = srcq + sbase;
    const R *ctb = std::is_same<R, float>::value ? (const R *)(ctf + sbase) : (const R *)(ctq + sbase);
    const double *s1b = s1q + sbase, *Gb = Gq + sbase;
    double *fb0 = fd + sbase;
    double *fob0 = B2 ? fod + sbase : nullptr;
    PT *pb0 = part + sbase;
    auto fetch = [&](Slot<R> &sl, int t) {
      const int o = t * BAND;
      sl.ct = ctb[o];
      if (MODE == 0) sl.s = srcb[o];
      if (FP) sl.a1 = s1b[o];
      if (FP || RH) {
        sl.a2 = Gb[o];
        sl.a3 = fb0[o];
      }
      if (B2) sl.a4 = fob0[o];
    };
    // hand the top row's columns (last - cnt, last] to the band above; lane i
    // of rout holds column last - i
    auto flush = [&](int last, int cnt, R rout, R routh) {
      const int pend = pout0 + last + 1;
      if (seen_cons < pend - RING) {
        while ((seen_cons = lds_load(&cons[wout])) < pend - RING) __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      if (lane < cnt) {
        ring[wout][(pout0 + last - lane) & (RING - 1)][0] = rout;
        if (NF == 2) ring[wout][(pout0 + last - lane) & (RING - 1)][NF - 1] = routh;
      }
      lds_publish(&prod[wout], pend, lane == 0);
    };

    Slot<R> sl[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k) fetch(sl[k], k);
    R fl = gx, hl = gx, fprev = R(0), hprev = R(0);
    R rin = gy, rinh = gy, rout = R(0), routh = R(0);
    // steps of the band, rounded up to the chunk (the extra steps are idle)
    const int T = ((nx + rows - 1 + CH - 1) / CH) * CH;
    for (int t0 = 0; t0 < T; t0 += CH) {
      if (has_in && t0 < nx) {  // row-0 inputs of columns t0 .. t0 + CH - 1
        const int need = pin0 + min(t0 + CH, nx);
        if (seen_prod < need) {
          while ((seen_prod = lds_load(&prod[win])) < need) __builtin_amdgcn_s_sleep(1);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (lane < CH) {
          rin = ring[win][(pin0 + t0 + lane) & (RING - 1)][0];
          if (NF == 2) rinh = ring[win][(pin0 + t0 + lane) & (RING - 1)][NF - 1];
        }
        lds_publish(&cons[win], need, lane == 0);
      }
      // chunk-local pointers: the unrolled steps use constant offsets
      const R *srcc = srcb + t0 * BAND, *ctc = ctb + t0 * BAND;
      const double *s1c = s1b + t0 * BAND, *Gc = Gb + t0 * BAND;
      double *fc = fb0 + t0 * BAND;
      double *foc = B2 ? fob0 + t0 * BAND : nullptr;
      PT *pc = pb0 + t0 * BAND;
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int t = t0 + k;
        const Slot<R> &c = sl[k % PD];
        // lane 0 takes the band below's value of column t from rin, which
        // rotates down one lane per step
        const R fb = shr1_in(fprev, rin);
        const R hb = NF == 2 ? shr1_in(hprev, rinh) : R(0);
        rin = rol1(rin);
        if (NF == 2) rinh = rol1(rinh);
        const R inv = rt_rcp(c.ct + mxyr);
        R f, h = R(0);
        PT v;
        if (MODE == 0) {
          // zero source in the padding keeps lanes that have not reached
          // column 0 at exactly zero, which is the zero inflow
          f = (c.s + my * fb + mx * fl) * inv;
          v = (PT)(w * f);
          fl = f;
        } else {
          const bool on = rowok && (unsigned)(t - lane) < unx;
          if (FP) {
            const R s1 = B2 ? (R)(c.a1 + (4.0 * c.a3 - c.a4) * hdt) : (R)(c.a1 + c.a3 * A.inv_dt);
            f = (s1 + my * fb + mx * fl) * inv;
            (B2 ? foc : fc)[k * BAND] = (double)f;  // BDF2: f^n over f^{n-2}
          } else {
            f = (R)c.a3;
          }
          // history of the next step: f^n / dt, or (4 f^n - f^{n-1}) / (2 dt)
          R s2;
          if (!B2) s2 = rt_fma(f, idt, (R)c.a2);
          else s2 = (R)((4.0 * (double)f - (FP ? c.a3 : c.a4)) * hdt + c.a2);
          h = (s2 + my * hb + mx * hl) * inv;
          v = (PT)(w * h);
          fl = on ? f : gx;
          hl = on ? h : gx;
        }
        pc[k * BAND] = v;
        fprev = f;
        hprev = h;
        if (has_out) {
          // the top row finished column ao = t - (BAND - 1); it enters rout at
          // lane 0 while older columns move up one lane
          const int ao = t - (BAND - 1);
          rout = ror1(lane == BAND - 1 ? f : rout);
          if (NF == 2) routh = ror1(lane == BAND - 1 ? h : routh);
          if (k == (BAND - 1 + CH - 1) % CH) {  // ao closes a chunk
            if (ao >= 0 && ao < nx) flush(ao, CH, rout, routh);
          } else if (ao == nx - 1) {
            flush(ao, (ao & (CH - 1)) + 1, rout, routh);
          }
        }
        {  // prefetch step t + PD
          Slot<R> &n = sl[k % PD];
          const int o = (k + PD) * BAND;
          n.ct = ctc[o];
          if (MODE == 0) n.s = srcc[o];
          if (FP) n.a1 = s1c[o];
          if (FP || RH) {
            n.a2 = Gc[o];
            n.a3 = fc[o];
          }
          if (B2) n.a4 = foc[o];
        }
      }
    }
  }
}

// Skew a per-cell quantity into the four quadrant layouts (padding slots 0):
// KIND 0: x[c]; KIND 1: sigma_s[c] x[c]; KIND 2: sigma_s[c] x[c] + G[c].
template <typename R, int KIND, typename X = double>
__global__ void __launch_bounds__(BLK) k_skew(PlaneArgs A, const double *ss, const X *x, const double *G,
                                              R *out) {
  const int slot = blockIdx.x * BLK + threadIdx.x, q = blockIdx.y;
  if (slot >= A.SQ) return;
  const int c = slot_cell(A, q, slot);
  double v = 0.0;
  if (c >= 0) {
    if (KIND == 0) v = (double)x[c];
    if (KIND == 1) v = ss[c] * (double)x[c];
    if (KIND == 2) v = rt_fma(ss[c], (double)x[c], G[c]);
  }
  out[(size_t)q * A.SQ + slot] = (R)v;
}
// f^0: the isotropic initial flux x on every folded ordinate
__global__ void __launch_bounds__(BLK) k_skew_f(PlaneArgs A, const double *x) {
  const int slot = blockIdx.x * BLK + threadIdx.x, dir = blockIdx.y;
  if (slot >= A.SQ) return;
  const int c = slot_cell(A, quad_of(dir, A), slot);
  A.f[(size_t)dir * A.SQ + slot] = c >= 0 ? x[c] : 0.0;
}

// per-quadrant sums of the per-ordinate partials, ordinates in order
template <typename PT>
__global__ void __launch_bounds__(BLK) k_quad_sum(PlaneArgs A) {
  const int slot = blockIdx.x * BLK + threadIdx.x, q = blockIdx.y;
  if (slot >= A.SQ) return;
  const PT *p = (const PT *)A.partial + slot;
  double s = 0.0;
  for (int d = A.qstart[q]; d < A.qstart[q + 1]; ++d) s += (double)p[(size_t)d * A.SQ];
  A.quadsum[(size_t)q * A.SQ + slot] = s;
}

// out[c] = sum over the quadrants (in order) (+ add[c], or + out[c] when
// accumulating); optional per-block maxima for the stop test of Alg. 1:
// max|out - rp| and max|out|.
__global__ void __launch_bounds__(BLK) k_unskew(PlaneArgs A, double *out, const double *add, int accumulate,
                                                const double *rp, double *blkmax) {
  const int c = blockIdx.x * BLK + threadIdx.x;
  double d = 0.0, y = 0.0;
  if (c < A.nc) {
    const int ix = c % A.nx, iy = c / A.nx;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += A.quadsum[(size_t)q * A.SQ + cell_slot(A, q, ix, iy)];
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

// Chebyshev DSA solve in blocks of DS iterations, one launch per block.
// Tiles of TE x TE cells (TE = 32 or 16, chosen per grid shape by the
// autotuner: the smaller tile gives four times the workgroups for twice the
// halo work), one workgroup of DTHR threads per tile.  A launch reads the
// tile's directions and residuals over a halo of DS cells and iterates DS
// times with the directions in LDS and everything pointwise (residual,
// solution, operator coefficients) in registers; the valid region shrinks by
// one cell per iteration.  Each cell sees exactly the arithmetic of one
// global iteration, so the result does not depend on the tiling.  Kernel
// boundaries order the blocks: no grid-wide synchronisation inside a launch.
constexpr int DS = 8;                // iterations per launch (halo)
constexpr int DTHR = 1024;           // threads per workgroup of k_dsa_block
template <int TE>
struct DsaTile {
  static constexpr int E = TE + 2 * DS;                      // extended tile edge
  static constexpr int PT = (E * E + DTHR - 1) / DTHR;       // extended cells per thread
};

struct DsaSolve {
  DsaArgs D;
  const double *ss, *y, *rp;
  double *x;                      // solution, cell layout
  double *r0, *r1, *d0, *d1;      // double-buffered residual / direction
  const double *c1, *c2;          // Chebyshev coefficients per iteration
  int K, ntx, ntiles, pad_;
  double inv_theta;
};

// r = sigma_s (y - rp), x = 0, d = r / (theta diag); TE x TE threads per tile
template <int TE>
__global__ void __launch_bounds__(TE * TE) k_dsa_init(DsaSolve S) {
  const DsaArgs &D = S.D;
  const int tile = blockIdx.x;
  const int tx = tile % S.ntx, ty = tile / S.ntx;
  const int ix = tx * TE + (int)threadIdx.x % TE, iy = ty * TE + (int)threadIdx.x / TE;
  if (ix < D.nx && iy < D.ny) {
    const int c = iy * D.nx + ix;
    const double rhs = S.ss[c] * (S.y[c] - S.rp[c]);
    S.r0[c] = rhs;
    S.x[c] = 0.0;
    S.d0[c] = S.inv_theta * rhs / D.diag[c];
  }
}

// iterations done .. done + nit - 1, reading buffer cur and writing cur ^ 1;
// the last block closes x with the final direction
template <int TE>
__global__ void __launch_bounds__(DTHR) k_dsa_block(DsaSolve S, int done, int nit, int last, int cur) {
  constexpr int DT = TE, DE = DsaTile<TE>::E, DPT = DsaTile<TE>::PT;
  __shared__ double sd[DE * DE];
  const DsaArgs &D = S.D;
  const int nx = D.nx, ny = D.ny;
  const double *din = cur ? S.d1 : S.d0, *rin = cur ? S.r1 : S.r0;
  double *dout = cur ? S.d0 : S.d1, *rout = cur ? S.r0 : S.r1;
  const int tile = blockIdx.x;
  const int tx = tile % S.ntx, ty = tile / S.ntx;
  double dg[DPT], idg[DPT], ar[DPT], al[DPT], au[DPT], ad[DPT], r[DPT], xr[DPT];
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int e = threadIdx.x + DTHR * i;
    const int ex = e % DE, ey = e / DE;
    const int ix = tx * DT + ex - DS, iy = ty * DT + ey - DS;
    const bool in = e < DE * DE && ix >= 0 && ix < nx && iy >= 0 && iy < ny;
    const int c = in ? iy * nx + ix : 0;
    // links to out-of-grid neighbours are zero; those cells carry d = 0
    dg[i] = in ? D.diag[c] : 1.0;
    idg[i] = rt_rcp(dg[i]);  // the Jacobi scaling, once per launch
    ar[i] = in ? D.ax[c] : 0.0;
    au[i] = in ? D.ay[c] : 0.0;
    al[i] = in && ix > 0 ? D.ax[c - 1] : 0.0;
    ad[i] = in && iy > 0 ? D.ay[c - nx] : 0.0;
    r[i] = in ? rin[c] : 0.0;
    xr[i] = in && ex >= DS && ex < DS + DT && ey >= DS && ey < DS + DT ? S.x[c] : 0.0;
    if (e < DE * DE) sd[e] = in ? din[c] : 0.0;
  }
  __syncthreads();
  for (int it = 0; it < nit; ++it) {
    const double c1 = S.c1[done + it], c2 = S.c2[done + it];
    double dn[DPT];
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int e = threadIdx.x + DTHR * i;
      const int ex = e % DE, ey = e / DE;
      dn[i] = 0.0;
      if (e < DE * DE && ex > 0 && ex < DE - 1 && ey > 0 && ey < DE - 1) {
        const double dc = sd[e];
        xr[i] += dc;
        double v = dg[i] * dc;
        v -= ar[i] * sd[e + 1];
        v -= al[i] * sd[e - 1];
        v -= au[i] * sd[e + DE];
        v -= ad[i] * sd[e - DE];
        r[i] = r[i] - v;
        dn[i] = c1 * dc + c2 * r[i] * idg[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const int e = threadIdx.x + DTHR * i;
      const int ex = e % DE, ey = e / DE;
      if (e < DE * DE && ex > 0 && ex < DE - 1 && ey > 0 && ey < DE - 1) sd[e] = dn[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int e = threadIdx.x + DTHR * i;
    const int ex = e % DE, ey = e / DE;
    const int ix = tx * DT + ex - DS, iy = ty * DT + ey - DS;
    if (e < DE * DE && ex >= DS && ex < DS + DT && ey >= DS && ey < DS + DT && ix < nx && iy < ny) {
      const int c = iy * nx + ix;
      if (last) {
        S.x[c] = xr[i] + sd[e];  // the closing update with the final direction
      } else {
        S.x[c] = xr[i];
        dout[c] = sd[e];
        rout[c] = r[i];
      }
    }
  }
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
                               int n32, int used_mask, int lv_fb) {
  st->iters = iters;
  st->used_mask = used_mask;
  st->lv_fb = lv_fb;
  st->conv = conv;
  st->used_pc = used_pc;
  st->ig_fb = ig_fb;
  st->pc_fb = pc_fb;
  st->residual = resid;
  // phases 1, 2, 3 and, with correction ROMs of later iterations, one more
  // for each complete level (as the slab kernels count them)
  int ph = !st->flag_ig ? 1 : (!st->flag_pc ? 2 : 3);
  for (int k = 0; k < RT_XLEV; ++k) ph += (ph == k + 3 && st->flag_pl[k]) ? 1 : 0;
  st->phase = ph;
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
    // unconditional loads (finite columns past the rank), masked
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      const double u = R.U[(size_t)k * ld + c];
      p[k] = k < rank ? u * v : 0.0;
    }
  }
  __shared__ double red[(BLK / 64) * RT_RMAX], out[RT_RMAX];
  wg_sum_fast<RT_RMAX>(p, red, out);
  if (threadIdx.x < RT_RMAX) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
__global__ void __launch_bounds__(256) k_romapply_solve(RomDev R, const int *rankp, int nblk, const double *part,
                                                        double *coef) {
  const int rank = *rankp;
  __shared__ double vec[RT_RMAX], scratch[256];
  sum_partials<false>(part, nblk, rank, vec, scratch);
  lu_solve_wave(R.LU, R.perm, rank, vec);  // ends with a barrier
  if ((int)threadIdx.x < RT_RMAX) coef[threadIdx.x] = (int)threadIdx.x < rank ? vec[threadIdx.x] : 0.0;
}
__global__ void __launch_bounds__(BLK) k_romapply_expand(RomDev R, const int *rankp, int ld, int nc,
                                                        const double *coef, double *out) {
  const int rank = *rankp;
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c < nc) {
    // every column loaded; coef is zero past the rank
    double u[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) u[k] = R.U[(size_t)k * ld + c];
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(u[k], coef[k], v);
    out[c] = v;
  }
}

// ---------------------------------------------------------------------------
// McClarren-Haut (Sec. 3.3) over the grid: the model of the one-workgroup
// slab kernel (rt_mh.h) with its cell-wise passes as grid kernels (block
// partial sums, summed in a fixed order by one workgroup) and its O(m^2) /
// O(m^3) work in one workgroup, the state in global memory.  Pair l
// (iterations l >= 2): x = rho^{(l-1)} - rho^{(l-2)}, z = y_l - y_{l-1},
// both scaled by 1/||x||_2, inputs orthonormalised by classical Gram-Schmidt
// applied twice into Q (X = Q R), B = Q^T Z, A~ = B R^{-1}; the correction
// d = Q (I - A~)^{-1} A~ Q^T (y - rho^{(l-1)}).  A pair whose scaled input
// keeps an orthogonal remainder of at most 1e-6 is skipped; a full model
// (mh_cap pairs) restarts from the newest pair.  The model lives within one
// time step.
// ---------------------------------------------------------------------------
struct MhGrid {
  int m, m0, skip, bad;
  double xn, nu;
  double R[RT_RMAX * RT_RMAX];  // R[i * RT_RMAX + j], upper triangular
  double B[RT_RMAX * RT_RMAX];  // B = Q^T Z
  double a1[RT_RMAX], ac[RT_RMAX], qz[RT_RMAX], c[RT_RMAX];
};

__global__ void k_mh_reset(MhGrid *M) {
  if (threadIdx.x == 0) M->m = 0;
}

// pass 1 of a pair: partials of Q^T x, Q^T z, x.x (m0: the model's size
// after a restart of a full one)
__global__ void __launch_bounds__(BLK) k_mh_pass1(Inst I, int nc, const double *rp, const double *rp2,
                                                  const double *y, const double *yp, MhGrid *M, double *part) {
  const int m = M->m, m0 = m == I.mh_cap ? 0 : m, ld = I.ld;
  const int c = blockIdx.x * BLK + threadIdx.x;
  double p[RT_MH_NP];
#pragma unroll
  for (int k = 0; k < RT_MH_NP; ++k) p[k] = 0.0;
  if (c < nc) {
    const double x = rp[c] - rp2[c], z = y[c] - yp[c];
    p[2 * RT_RMAX] = x * x;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k)
      if (k < m0) {
        const double q = I.mhQ[(size_t)k * ld + c];
        p[k] = q * x;
        p[RT_RMAX + k] = q * z;
      }
  }
  __shared__ double red[(BLK / 64) * RT_MH_NP], out[RT_MH_NP];
  wg_sum_fast<RT_MH_NP>(p, red, out);
  if (threadIdx.x < RT_MH_NP) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
__global__ void __launch_bounds__(256) k_mh_small1(Inst I, int nblk, const double *part, MhGrid *M) {
  __shared__ double vec[RT_MH_NP], scratch[256];
  sum_partials<false>(part, nblk, RT_MH_NP, vec, scratch);
  const int m = M->m, m0 = m == I.mh_cap ? 0 : m;
  const double xx = vec[2 * RT_RMAX];
  __syncthreads();
  if (threadIdx.x == 0) {
    M->m0 = m0;
    M->skip = !(xx > 0.0);  // no input difference: nothing to learn
    M->xn = sqrt(fmax(xx, 0.0));
  }
  if ((int)threadIdx.x < RT_RMAX) {
    const int k = threadIdx.x;
    const double ixn = xx > 0.0 ? 1.0 / sqrt(xx) : 0.0;
    M->a1[k] = k < m0 ? vec[k] * ixn : 0.0;
    M->qz[k] = k < m0 ? vec[RT_RMAX + k] : 0.0;
  }
}
// pass 2: p = x / ||x|| - Q a1; partials of Q^T p, p.p
__global__ void __launch_bounds__(BLK) k_mh_pass2(Inst I, int nc, const double *rp, const double *rp2,
                                                  const MhGrid *M, double *part) {
  if (M->skip) return;
  const int m0 = M->m0, ld = I.ld;
  const double ixn = 1.0 / M->xn;
  const int c = blockIdx.x * BLK + threadIdx.x;
  double p[RT_RMAX + 1];
#pragma unroll
  for (int k = 0; k <= RT_RMAX; ++k) p[k] = 0.0;
  if (c < nc) {
    double q[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) q[k] = k < m0 ? I.mhQ[(size_t)k * ld + c] : 0.0;
    double v = (rp[c] - rp2[c]) * ixn;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(-q[k], M->a1[k], v);
    p[RT_RMAX] = v * v;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) p[k] = q[k] * v;
  }
  __shared__ double red[(BLK / 64) * (RT_RMAX + 1)], out[RT_RMAX + 1];
  wg_sum_fast<RT_RMAX + 1>(p, red, out);
  if (threadIdx.x <= RT_RMAX) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
__global__ void __launch_bounds__(256) k_mh_small2(int nblk, const double *part, MhGrid *M) {
  if (M->skip) return;
  __shared__ double vec[RT_RMAX + 1], scratch[256];
  sum_partials<false>(part, nblk, RT_RMAX + 1, vec, scratch);
  if (threadIdx.x == 0) {
    const int m0 = M->m0;
    double a2s = 0.0;
    for (int k = 0; k < m0; ++k) a2s = rt_fma(vec[k], vec[k], a2s);
    const double nu = sqrt(fmax(vec[RT_RMAX] - a2s, 0.0));
    M->nu = nu;
    if (!(nu > RT_MH_DEP)) {
      M->skip = 1;  // in span already
    } else {
      const double ixn = 1.0 / M->xn;
      for (int k = 0; k < m0; ++k) {
        M->ac[k] = M->a1[k] + vec[k];
        M->R[k * RT_RMAX + m0] = M->ac[k];
        M->B[k * RT_RMAX + m0] = M->qz[k] * ixn;
      }
      for (int k = m0; k < RT_RMAX; ++k) M->ac[k] = 0.0;
      M->R[m0 * RT_RMAX + m0] = nu;
    }
  }
}
// pass 3: the new columns of Q and Z; partials of the new row of B,
// q . Z_k and q . z^ as direct dot products
__global__ void __launch_bounds__(BLK) k_mh_pass3(Inst I, int nc, const double *rp, const double *rp2,
                                                  const double *y, const double *yp, const MhGrid *M, double *part) {
  if (M->skip) return;
  const int m0 = M->m0, ld = I.ld;
  const double ixn = 1.0 / M->xn, inu = 1.0 / M->nu;
  const int c = blockIdx.x * BLK + threadIdx.x;
  double p[RT_RMAX + 1];
#pragma unroll
  for (int k = 0; k <= RT_RMAX; ++k) p[k] = 0.0;
  if (c < nc) {
    double v = (rp[c] - rp2[c]) * ixn;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k)
      if (k < m0) v = rt_fma(-I.mhQ[(size_t)k * ld + c], M->ac[k], v);
    v *= inu;
    const double zh = (y[c] - yp[c]) * ixn;
    I.mhQ[(size_t)m0 * ld + c] = v;
    I.mhZ[(size_t)m0 * ld + c] = zh;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k)
      if (k < m0) p[k] = v * I.mhZ[(size_t)k * ld + c];
    p[RT_RMAX] = v * zh;
  }
  __shared__ double red[(BLK / 64) * (RT_RMAX + 1)], out[RT_RMAX + 1];
  wg_sum_fast<RT_RMAX + 1>(p, red, out);
  if (threadIdx.x <= RT_RMAX) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
__global__ void __launch_bounds__(256) k_mh_small3(int nblk, const double *part, MhGrid *M) {
  if (M->skip) return;
  __shared__ double vec[RT_RMAX + 1], scratch[256];
  sum_partials<false>(part, nblk, RT_RMAX + 1, vec, scratch);
  const int m0 = M->m0;
  if ((int)threadIdx.x < m0) M->B[m0 * RT_RMAX + threadIdx.x] = vec[threadIdx.x];
  if (threadIdx.x == 0) {
    M->B[m0 * RT_RMAX + m0] = vec[RT_RMAX];
    M->m = m0 + 1;
  }
}
// the correction: partials of Q^T r, r = y - rho
__global__ void __launch_bounds__(BLK) k_mh_cpass(Inst I, int nc, const double *y, const double *rp,
                                                  const MhGrid *M, double *part) {
  const int m = M->m, ld = I.ld;
  if (m == 0) return;
  const int c = blockIdx.x * BLK + threadIdx.x;
  double p[RT_RMAX];
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) p[k] = 0.0;
  if (c < nc) {
    const double r = y[c] - rp[c];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k)
      if (k < m) p[k] = I.mhQ[(size_t)k * ld + c] * r;
  }
  __shared__ double red[(BLK / 64) * RT_RMAX], out[RT_RMAX];
  wg_sum_fast<RT_RMAX>(p, red, out);
  if (threadIdx.x < RT_RMAX) part[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}
// A~ = B R^{-1}, g = A~ Q^T r, and (I - A~) c = g on wave 0 (mh_solve_wave);
// c = 0 for an empty model or a singular system
__global__ void __launch_bounds__(256) k_mh_csolve(int nblk, const double *part, MhGrid *M) {
  __shared__ MhLds S;
  __shared__ double vec[RT_RMAX], scratch[256];
  const int m = M->m;
  if (m == 0) {
    if ((int)threadIdx.x < RT_RMAX) M->c[threadIdx.x] = 0.0;
    return;
  }
  sum_partials<false>(part, nblk, RT_RMAX, vec, scratch);
  if (threadIdx.x < 64) {
    const int i = threadIdx.x;
    if (i < m) {
      double at[RT_RMAX];
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j) {
        if (j < m) {
          double v = M->B[i * RT_RMAX + j];
#pragma unroll
          for (int k = 0; k < RT_RMAX; ++k)
            if (k < j) v = rt_fma(-at[k], M->R[k * RT_RMAX + j], v);
          at[j] = v / M->R[j * RT_RMAX + j];
        } else {
          at[j] = 0.0;
        }
      }
      double g = 0.0;
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j)
        if (j < m) g = rt_fma(at[j], vec[j], g);
      S.vec[i] = g;
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j)
        if (j < m) S.A[i * RT_KC + j] = (i == j ? 1.0 : 0.0) - at[j];
    }
  }
  __syncthreads();
  const int bad = mh_solve_wave(S, m);
  if ((int)threadIdx.x < RT_RMAX) M->c[threadIdx.x] = (!bad && (int)threadIdx.x < m) ? S.vec[threadIdx.x] : 0.0;
}
// d = Q c
__global__ void __launch_bounds__(BLK) k_mh_expand(Inst I, int nc, const MhGrid *M, double *d) {
  const int m = M->m, ld = I.ld;
  const int c = blockIdx.x * BLK + threadIdx.x;
  if (c >= nc) return;
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k)
    if (k < m) v = rt_fma(I.mhQ[(size_t)k * ld + c], M->c[k], v);
  d[c] = v;
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
  std::vector<int> quad;          // folded index -> quadrant
  char *mem = nullptr;            // one allocation for everything below
  double *y = nullptr, *rp = nullptr, *dvec = nullptr;
  float *src32 = nullptr;
  double *cr = nullptr, *cx = nullptr, *cd0 = nullptr, *cd1 = nullptr;
  double *diag = nullptr, *ax = nullptr, *ay = nullptr;
  double *blkmax = nullptr;
  // the stop test's two norms, written by the reduce kernel straight into
  // coherent pinned host memory (res_hd: its device address), and a pinned
  // copy of the step state: a round trip per SI iteration without a copy
  double *res_h = nullptr, *res_hd = nullptr;
  RtState *st_h = nullptr;
  double *rpart = nullptr, *rcoef = nullptr;
  double *yp = nullptr, *rp2 = nullptr;  // McClarren-Haut: y_{l-1}, rho^{(l-2)}
  MhGrid *mh = nullptr;                  // McClarren-Haut model state
  int cheb_iters = 0;
  int pd32 = 8, pd64 = 8;  // prefetch depth of the SI sweeps (FP32 / FP64), tuned per grid shape
  int dsa_tile = 32;       // tile edge of the Chebyshev DSA kernels (32 or 16), tuned per grid shape
  double cheb_theta = 1.0, cheb_delta = 0.0;
  double *cheb_c = nullptr;                 // device: c1[K], c2[K]
  size_t bytes = 0;
};

namespace {
struct PlaneGeom {
  int ndf, nbands, TT, SQ;
};
PlaneGeom plane_geom(const rtrom_problem_desc *d) {
  PlaneGeom g;
  g.ndf = d->n_polar * d->n_azim / 2;
  g.nbands = (d->ny + BAND - 1) / BAND;
  // steps per band incl. the unroll round-up and the prefetch run-out
  g.TT = ((d->nx + BAND - 1 + CH - 1) / CH) * CH + CH;
  g.SQ = g.nbands * g.TT * BAND;
  return g;
}
}  // namespace

static size_t plane_bytes_for(const rtrom_problem_desc *d) {
  const PlaneGeom g = plane_geom(d);
  const size_t nc = (size_t)d->nx * d->ny, SQ = (size_t)g.SQ;
  const size_t nblk = (nc + BLK - 1) / BLK;
  size_t b = 0;
  auto take = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  take((size_t)g.ndf * SQ * 8);     // per-ordinate partials
  take((size_t)g.ndf * SQ * 8);     // folded f
  if (d->time_scheme == RTROM_BDF2) take((size_t)g.ndf * SQ * 8);  // BDF2: the older level
  take(4 * SQ * 8 * 5);             // ctq, Gq, s1q, srcq, quadsum
  take(4 * SQ * 4);                 // ctf
  take(nc * 8 * 7);                 // y rp dvec cr cx cd0 cd1
  take(nc * 4);                     // src32
  take(nc * 8 * 3);                 // diag ax ay
  take(nblk * 2 * 8 + 64);          // blkmax
  take(2 * (size_t)RT_CHEB_MAX * 8);               // Chebyshev coefficients
  take(nblk * RT_NPART * 8 + RT_RMAX * 8);  // DMD solve partials, coefficients
  take((size_t)g.ndf * 3 * 8);      // mx my w
  if (d->precond == RTROM_PC_MH) {  // McClarren-Haut: y_{l-1}, rho^{(l-2)}, model state
    take(nc * 8 * 2);
    take(sizeof(MhGrid));
  }
  return b;
}

size_t rt_plane_extra_bytes(const rtrom_problem_desc *d) { return plane_bytes_for(d); }

// Largest nx for grids with more bands than waves: the bands then cycle
// through the waves, and the band-to-band rings (RING columns, moved CH at a
// time) must drain before a wave moves to its next band.
int rt_plane_max_nx_cyclic() { return MAXW * (RING - CH); }
int rt_plane_needs_cyclic(int ny) { return (ny + BAND - 1) / BAND > MAXW; }

#define PH(call)                                                            \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      rt_set_error(std::string("plane: ") + hipGetErrorString(e_));         \
      return RTROM_EDEVICE;                                                 \
    }                                                                       \
  } while (0)

// The SI sweep (MODE 0) with prefetch depth pd (2, 4, 8 or 16 steps of cell
// data loaded ahead).  The depth changes only how far ahead the loads are
// issued, never the arithmetic, so every depth gives bitwise the same result.
template <typename R>
static void launch_si_sweep(int pd, dim3 grid, dim3 block, hipStream_t s, const PlaneArgs &A) {
  switch (pd) {
    case 2: hipLaunchKernelGGL((k_plane_sweep<R, 0, 2>), grid, block, 0, s, A); break;
    case 4: hipLaunchKernelGGL((k_plane_sweep<R, 0, 4>), grid, block, 0, s, A); break;
    case 16: hipLaunchKernelGGL((k_plane_sweep<R, 0, 16>), grid, block, 0, s, A); break;
    default: hipLaunchKernelGGL((k_plane_sweep<R, 0, 8>), grid, block, 0, s, A); break;
  }
}

static int dsa_solve(rtrom_problem *p, PlaneHost *H, const double *y, const double *rp);

// Autotuner of the X-Y shapes: the SI sweep's prefetch depth and the tile
// edge of the Chebyshev DSA kernels.  For each grid shape (nx, ny, folded
// ordinates) the first problem created times the FP32 and FP64 SI sweeps at
// every depth and the DSA solve at both tile edges (one warm-up and three
// timed launches each, HIP events on the problem's stream; the sweeps write
// only their scratch partials and the DSA only its scratch vectors, so the
// state is untouched) and keeps the fastest; later problems of the same
// shape reuse the choice.  Neither choice changes the arithmetic of any cell,
// so results are bitwise the same whatever is chosen.  RTROM_TUNE_CACHE
// names a text file that keeps the choices across processes (one line per
// shape, "plane_tune nx ny ndf pd32 pd64 dsa_tile", read at the first tuning,
// appended after each new one; lines that do not parse are ignored).
// RTROM_TUNE=0 keeps depth 8 and tile 32; RTROM_PLANE_PD="<fp32>,<fp64>" and
// RTROM_DSA_TILE=<16|32> fix them; RTROM_TUNE_LOG=1 prints the timings.
namespace {
struct PlaneTune {
  int pd32, pd64, tile;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, PlaneTune> g_tune;
bool g_tune_file_read = false;
bool valid_depth(int v) { return v == 2 || v == 4 || v == 8 || v == 16; }
bool valid_tile(int v) { return v == 16 || v == 32; }
// with g_tune_mu held
void tune_cache_load() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char *path = std::getenv("RTROM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    int nx, ny, ndf, a, b, t;
    if (std::sscanf(line, "plane_tune %d %d %d %d %d %d", &nx, &ny, &ndf, &a, &b, &t) == 6 && valid_depth(a) &&
        valid_depth(b) && valid_tile(t))
      g_tune[std::make_tuple(nx, ny, ndf)] = {a, b, t};
  }
  std::fclose(f);
}
void tune_cache_append(int nx, int ny, int ndf, const PlaneTune &c) {
  const char *path = std::getenv("RTROM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "plane_tune %d %d %d %d %d %d\n", nx, ny, ndf, c.pd32, c.pd64, c.tile);
  std::fclose(f);
}
}  // namespace

static int tune_plane(rtrom_problem *p, PlaneHost *H) {
  const char *ftile = std::getenv("RTROM_DSA_TILE");
  const int fixed_tile = ftile && valid_tile(std::atoi(ftile)) ? std::atoi(ftile) : 0;
  H->dsa_tile = fixed_tile ? fixed_tile : 32;
  const char *fixed = std::getenv("RTROM_PLANE_PD");
  if (fixed) {
    int a = 8, b = 8;
    if (std::sscanf(fixed, "%d,%d", &a, &b) == 2) {
      H->pd32 = valid_depth(a) ? a : 8;
      H->pd64 = valid_depth(b) ? b : 8;
    }
    return RTROM_OK;
  }
  const char *tune = std::getenv("RTROM_TUNE");
  if (tune && std::atoi(tune) == 0) return RTROM_OK;
  const PlaneArgs &A = H->A;
  const auto key = std::make_tuple(A.nx, A.ny, A.ndf);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      H->pd32 = it->second.pd32;
      H->pd64 = it->second.pd64;
      H->dsa_tile = fixed_tile ? fixed_tile : it->second.tile;
      rt_log(2, "plane %dx%d, %d folded ordinates: SI sweep prefetch depths %d (FP32) / %d (FP64), DSA tile %d, cached",
             A.nx, A.ny, A.ndf, H->pd32, H->pd64, H->dsa_tile);
      return RTROM_OK;
    }
  }
  hipStream_t s = p->stream;
  const dim3 grid(A.ndf), block(64 * A.nw);
  hipEvent_t e0, e1;
  PH(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    rt_set_error("plane: tuning event");
    return RTROM_EDEVICE;
  }
  const bool log = std::getenv("RTROM_TUNE_LOG") && std::atoi(std::getenv("RTROM_TUNE_LOG"));
  int rc = RTROM_OK;
  // one warm-up and three timed runs of f; the average in ms, or -1 on error
  auto timed = [&](auto &&f) -> float {
    f();
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess) return -1.0f;
    for (int r = 0; r < 3; ++r) f();
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
      return -1.0f;
    return ms / 3.0f;
  };
  const int depths[4] = {2, 4, 8, 16};
  PlaneTune best{8, 8, 32};
  for (int prec = 0; prec < 2 && rc == RTROM_OK; ++prec) {
    float tbest = 1e30f;
    for (int pd : depths) {
      const float ms = timed([&] {
        if (prec == 0) launch_si_sweep<float>(pd, grid, block, s, A);
        else launch_si_sweep<double>(pd, grid, block, s, A);
      });
      if (ms < 0.0f) {
        rc = RTROM_EDEVICE;
        break;
      }
      if (log)
        std::fprintf(stderr, "rtrom tune: plane %dx%d, %d folded ordinates, %s SI sweep, depth %2d: %.1f us\n", A.nx,
                     A.ny, A.ndf, prec ? "FP64" : "FP32", pd, 1e3f * ms);
      if (ms < tbest) {
        tbest = ms;
        (prec ? best.pd64 : best.pd32) = pd;
      }
    }
  }
  float tbest = 1e30f;
  for (int te : {32, 16}) {
    if (rc != RTROM_OK) break;
    H->dsa_tile = te;
    const float ms = timed([&] { (void)dsa_solve(p, H, H->y, H->rp); });
    if (ms < 0.0f) {
      rc = RTROM_EDEVICE;
      break;
    }
    if (log)
      std::fprintf(stderr, "rtrom tune: plane %dx%d, DSA (%d Chebyshev iterations), tile %d: %.1f us\n", A.nx, A.ny,
                   H->cheb_iters, te, 1e3f * ms);
    if (ms < tbest) {
      tbest = ms;
      best.tile = te;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != RTROM_OK) {
    rt_set_error("plane: tuning failed");
    return rc;
  }
  H->pd32 = best.pd32;
  H->pd64 = best.pd64;
  H->dsa_tile = fixed_tile ? fixed_tile : best.tile;
  rt_log(2, "plane %dx%d, %d folded ordinates: SI sweep prefetch depths %d (FP32) / %d (FP64), DSA tile %d, tuned",
         A.nx, A.ny, A.ndf, H->pd32, H->pd64, best.tile);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune.emplace(key, best).second) tune_cache_append(A.nx, A.ny, A.ndf, best);
  return RTROM_OK;
}

// sweep + per-quadrant sums + un-skew into out
static int sweep_moment(rtrom_problem *p, PlaneHost *H, int mode, int fp32, double *out, const double *add,
                        int accumulate, const double *rp, double *blkmax) {
  PlaneArgs &A = H->A;
  hipStream_t s = p->stream;
  const dim3 grid(A.ndf), block(64 * A.nw), qgrid(A.nsblk, 4);
  const int kind = mode == 0 ? RT_K_PLANE_SWEEP : RT_K_PLANE_FPASS;
  rt_prof_begin(kind, s);
  if (mode == 0 && fp32) launch_si_sweep<float>(H->pd32, grid, block, s, A);
  else if (mode == 0) launch_si_sweep<double>(H->pd64, grid, block, s, A);
  else if (mode == 1) hipLaunchKernelGGL((k_plane_sweep<double, 1, 4>), grid, block, 0, s, A);
  else if (mode == 2) hipLaunchKernelGGL((k_plane_sweep<double, 2, 4>), grid, block, 0, s, A);
  else if (mode == 3) hipLaunchKernelGGL((k_plane_sweep<double, 3, 4>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_plane_sweep<double, 4, 4>), grid, block, 0, s, A);
  rt_prof_end(kind, s);
  rt_prof_begin(RT_K_PLANE_OTHER, s);
  if (mode == 0 && fp32) hipLaunchKernelGGL(k_quad_sum<float>, qgrid, dim3(BLK), 0, s, A);
  else hipLaunchKernelGGL(k_quad_sum<double>, qgrid, dim3(BLK), 0, s, A);
  hipLaunchKernelGGL(k_unskew, dim3(A.nblk), dim3(BLK), 0, s, A, out, add, accumulate, rp, blkmax);
  rt_prof_end(RT_K_PLANE_OTHER, s);
  PH(hipGetLastError());
  return RTROM_OK;
}

int rt_plane_create(rtrom_problem *p) {
  const rtrom_problem_desc *d = &p->d;
  PlaneHost *H = new PlaneHost();
  p->plane = H;
  const PlaneGeom g = plane_geom(d);
  const int ndf = g.ndf;
  H->bytes = plane_bytes_for(d);
  H->ndf = ndf;
  const int nx = d->nx, ny = d->ny, nc = nx * ny;
  const int nblk = (nc + BLK - 1) / BLK;
  if (g.nbands > MAXW && nx > rt_plane_max_nx_cyclic()) {
    rt_set_error("plane: grids with more than 1024 rows are limited to nx <= 3840");
    return RTROM_EINVAL;
  }
  // folded ordinates: the upper hemisphere (Omega_z > 0) grouped by upwind
  // quadrant, ordinate order within a quadrant; Omega_z < 0 ordinates map to
  // their mirror at the same azimuth
  const int nphi = d->n_azim, nz = d->n_polar;
  const double hx = d->lx / nx, hy = d->ly / ny;
  std::vector<double> hm(3 * (size_t)ndf, 0.0);
  H->fold_of.assign((size_t)nphi * nz, -1);
  H->quad.assign(ndf, 0);
  int nf = 0, qstart[5] = {0, 0, 0, 0, 0};
  for (int q = 0; q < 4; ++q) {
    qstart[q] = nf;
    for (int j2 = 0; j2 < nz; ++j2)
      for (int j1 = 0; j1 < nphi; ++j1) {
        const int j = j2 * nphi + j1;
        const int qj = (p->ox[j] > 0 ? 0 : 1) + (p->oy[j] > 0 ? 0 : 2);
        if (p->oz[j] > 0 && qj == q) {
          if (nf >= ndf) {
            rt_set_error("plane: quadrature is not symmetric in Omega_z");
            return RTROM_EINVAL;
          }
          const int idx = nf++;
          hm[idx] = std::fabs(p->ox[j]) / hx;
          hm[ndf + idx] = std::fabs(p->oy[j]) / hy;
          hm[2 * (size_t)ndf + idx] = 2.0 * p->w[j];
          H->fold_of[j] = idx;
          H->quad[idx] = q;
        }
      }
  }
  qstart[4] = nf;
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
  PH(hipMalloc(&H->mem, H->bytes));
  PH(hipMemsetAsync(H->mem, 0, H->bytes, p->stream));
  size_t off = 0;
  auto take = [&](size_t x) {
    char *q = H->mem + off;
    off += (x + 255) & ~size_t(255);
    return q;
  };
  const size_t SQ = (size_t)g.SQ;
  PlaneArgs &A = H->A;
  memset(&A, 0, sizeof(A));
  A.partial = take((size_t)ndf * SQ * 8);
  A.f = (double *)take((size_t)ndf * SQ * 8);
  A.fo = d->time_scheme == RTROM_BDF2 ? (double *)take((size_t)ndf * SQ * 8) : nullptr;
  double *q5 = (double *)take(4 * SQ * 8 * 5);
  A.ctq = q5;
  A.Gq = q5 + 4 * SQ;
  A.s1q = q5 + 8 * SQ;
  A.srcq = q5 + 12 * SQ;
  A.quadsum = q5 + 16 * SQ;
  A.ctf = (const float *)take(4 * SQ * 4);
  double *vecs = (double *)take((size_t)nc * 8 * 7);
  H->y = vecs;
  H->rp = H->y + nc;
  H->dvec = H->rp + nc;
  H->cr = H->dvec + nc;
  H->cx = H->cr + nc;
  H->cd0 = H->cx + nc;
  H->cd1 = H->cd0 + nc;
  H->src32 = (float *)take((size_t)nc * 4);
  H->diag = (double *)take((size_t)nc * 8 * 3);
  H->ax = H->diag + nc;
  H->ay = H->ax + nc;
  H->blkmax = (double *)take((size_t)nblk * 2 * 8 + 64);
  H->cheb_c = (double *)take(2 * (size_t)RT_CHEB_MAX * 8);
  H->rpart = (double *)take((size_t)nblk * RT_NPART * 8 + RT_RMAX * 8);
  H->rcoef = H->rpart + (size_t)nblk * RT_NPART;
  double *dmx = (double *)take((size_t)ndf * 3 * 8);
  if (d->precond == RTROM_PC_MH) {
    H->yp = (double *)take((size_t)nc * 8 * 2);
    H->rp2 = H->yp + nc;
    H->mh = (MhGrid *)take(sizeof(MhGrid));
  }
  Inst &I = p->hinst;
  PH(hipMemcpyAsync(dmx, hm.data(), hm.size() * 8, hipMemcpyHostToDevice, p->stream));
  PH(hipHostMalloc((void **)&H->res_h, 64, hipHostMallocCoherent | hipHostMallocMapped));
  PH(hipHostGetDevicePointer((void **)&H->res_hd, H->res_h, 0));
  PH(hipHostMalloc((void **)&H->st_h, sizeof(RtState), hipHostMallocDefault));
  A.nx = nx;
  A.ny = ny;
  A.nc = nc;
  A.ndf = ndf;
  A.nbands = g.nbands;
  A.nw = std::min(g.nbands, MAXW);
  A.nblk = nblk;
  A.TT = g.TT;
  A.SQ = g.SQ;
  A.nsblk = (g.SQ + BLK - 1) / BLK;
  for (int k = 0; k < 5; ++k) A.qstart[k] = qstart[k];
  A.inv_dt = 1.0 / d->dt;
  for (int k = 0; k < 4; ++k) A.g[k] = d->inflow[k];
  A.mx = dmx;
  A.my = dmx + ndf;
  A.w = dmx + 2 * (size_t)ndf;
  // static skewed inputs and f^0 (isotropic, from rho^0)
  const dim3 qgrid(A.nsblk, 4);
  hipLaunchKernelGGL((k_skew<double, 0>), qgrid, dim3(BLK), 0, p->stream, A, (const double *)nullptr, I.ct,
                     (const double *)nullptr, (double *)A.ctq);
  hipLaunchKernelGGL((k_skew<double, 0>), qgrid, dim3(BLK), 0, p->stream, A, (const double *)nullptr, I.G,
                     (const double *)nullptr, (double *)A.Gq);
  hipLaunchKernelGGL((k_skew<float, 0>), qgrid, dim3(BLK), 0, p->stream, A, (const double *)nullptr, I.ct,
                     (const double *)nullptr, (float *)A.ctf);
  hipLaunchKernelGGL(k_skew_f, dim3(A.nsblk, ndf), dim3(BLK), 0, p->stream, A, (const double *)I.rho);
  PH(hipGetLastError());
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
  // eigenvalues of diag^{-1} A lie in [1 - g, 1 + g] (Gershgorin; strictly
  // diagonally dominant because sigma_a + 1/dt > 0)
  const double lmin = std::max(1e-12, 1.0 - gmax), lmax = 1.0 + gmax;
  H->cheb_theta = 0.5 * (lmax + lmin);
  H->cheb_delta = 0.5 * (lmax - lmin);
  const double sigma1 = H->cheb_theta / std::max(H->cheb_delta, 1e-300);
  int K = 1;
  if (H->cheb_delta > 0.0) {
    // error bound 2 / T_K(sigma1) <= 1e-14
    const double kk = std::ceil(std::acosh(2e14) / std::acosh(sigma1));
    if (!(kk <= RT_CHEB_MAX)) {
      rt_set_error("2D DSA: the diffusion operator needs " + std::to_string(kk) +
                   " Chebyshev iterations for a 1e-14 error bound, more than the " + std::to_string(RT_CHEB_MAX) +
                   " this library runs (time step or mesh too fine for its diagonal dominance)");
      return RTROM_EINVAL;
    }
    K = std::max(1, (int)kk);
  }
  H->cheb_iters = K;
  // d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) diag^{-1} r_{k+1}
  std::vector<double> cc(2 * (size_t)K, 0.0);
  double rho_k = 1.0 / sigma1;
  for (int k = 0; k < K; ++k) {
    const double rho_n = 1.0 / (2.0 * sigma1 - rho_k);
    cc[k] = rho_n * rho_k;
    cc[K + k] = H->cheb_delta > 0.0 ? 2.0 * rho_n / H->cheb_delta : 0.0;
    rho_k = rho_n;
  }
  PH(hipMemcpyAsync(H->cheb_c, cc.data(), cc.size() * 8, hipMemcpyHostToDevice, p->stream));
  // the SI sweep's prefetch depth for this grid shape (the source is zero
  // until the first step writes it)
  PH(hipMemsetAsync(H->A.srcq, 0, 4 * (size_t)H->A.SQ * 8, p->stream));
  const int tr = tune_plane(p, H);
  if (tr != RTROM_OK) return tr;
  // b~^0 from f^0
  return rt_plane_rhs(p);
}

void rt_plane_destroy(rtrom_problem *p) {
  PlaneHost *H = (PlaneHost *)p->plane;
  if (!H) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (H->mem) (void)hipFree(H->mem);
  if (H->res_h) (void)hipHostFree(H->res_h);
  if (H->st_h) (void)hipHostFree(H->st_h);
  delete H;
  p->plane = nullptr;
}

// BDF2 after its backward-Euler start step: sigma~_t = sigma_t + 3/(2 dt)
// in the sweeps and the DSA coefficients with the same weight.  The
// Chebyshev interval taken at creation still holds: a larger time weight
// only strengthens the diagonal dominance it was derived from.
static int plane_bdf2_operator(rtrom_problem *p, PlaneHost *H) {
  const Inst &I = p->hinst;
  PlaneArgs &A = H->A;
  hipStream_t s = p->stream;
  const dim3 qgrid(A.nsblk, 4);
  hipLaunchKernelGGL((k_skew<double, 0>), qgrid, dim3(BLK), 0, s, A, (const double *)nullptr, I.ct_b,
                     (const double *)nullptr, (double *)A.ctq);
  hipLaunchKernelGGL((k_skew<float, 0>), qgrid, dim3(BLK), 0, s, A, (const double *)nullptr, I.ct_b,
                     (const double *)nullptr, (float *)A.ctf);
  hipLaunchKernelGGL(k_plane_setup, dim3(A.nblk), dim3(BLK), 0, s, H->D, I.ct_b, I.sa, 1.5 / p->d.dt,
                     p->d.lx / A.nx, p->d.ly / A.ny, H->diag, H->ax, H->ay, H->blkmax);
  PH(hipGetLastError());
  return RTROM_OK;
}

int rt_plane_rhs(rtrom_problem *p) {
  PlaneHost *H = (PlaneHost *)p->plane;
  for (int k = 0; k < 4; ++k) H->A.g[k] = p->d.inflow[k];
  // BDF2 after its start step: the history (4 f^n - f^{n-1}) / (2 dt)
  const int mode = p->hinst.bdf2 && p->steps >= 1 ? 4 : 2;
  return sweep_moment(p, H, mode, 0, p->hinst.bt2[p->steps & 1], nullptr, 0, nullptr, nullptr);
}

static int dsa_solve(rtrom_problem *p, PlaneHost *H, const double *y, const double *rp) {
  DsaSolve S;
  memset(&S, 0, sizeof(S));
  S.D = H->D;
  S.ss = p->hinst.ss;
  S.y = y;
  S.rp = rp;
  S.x = H->cx;
  S.r0 = H->cr;
  S.r1 = H->dvec;
  S.d0 = H->cd0;
  S.d1 = H->cd1;
  S.K = H->cheb_iters;
  S.c1 = H->cheb_c;
  S.c2 = H->cheb_c + S.K;
  const int te = H->dsa_tile;
  S.ntx = (H->A.nx + te - 1) / te;
  S.ntiles = S.ntx * ((H->A.ny + te - 1) / te);
  S.inv_theta = 1.0 / H->cheb_theta;
  hipStream_t s = p->stream;
  if (te == 16) hipLaunchKernelGGL(k_dsa_init<16>, dim3(S.ntiles), dim3(256), 0, s, S);
  else hipLaunchKernelGGL(k_dsa_init<32>, dim3(S.ntiles), dim3(1024), 0, s, S);
  int cur = 0;
  for (int done = 0; done < S.K; done += DS) {
    const int nit = std::min(DS, S.K - done);
    const int last = done + nit >= S.K;
    if (te == 16) hipLaunchKernelGGL(k_dsa_block<16>, dim3(S.ntiles), dim3(DTHR), 0, s, S, done, nit, last, cur);
    else hipLaunchKernelGGL(k_dsa_block<32>, dim3(S.ntiles), dim3(DTHR), 0, s, S, done, nit, last, cur);
    cur ^= 1;
  }
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

// residual of the current y against rp: ||y - rp||_inf, ||y||_inf
static int read_residual(rtrom_problem *p, PlaneHost *H, double *dn, double *yn) {
  hipLaunchKernelGGL(k_plane_maxreduce, dim3(1), dim3(256), 0, p->stream, (const double *)H->blkmax, H->A.nblk,
                     H->res_hd);
  PH(hipGetLastError());
  PH(hipStreamSynchronize(p->stream));
  const volatile double *r = H->res_h;
  *dn = r[0];
  *yn = r[1];
  return RTROM_OK;
}

// One backward-Euler step: Alg. 1 with the ROM hooks of Alg. 2 (initial guess
// and first correction), the loop driven from the host on the residual norms.
static int plane_one_step(rtrom_problem *p, PlaneHost *H) {
  Inst &I = p->hinst;
  PlaneArgs &A = H->A;
  const int nc = A.nc, nblk = A.nblk;
  const dim3 qgrid(A.nsblk, 4);
  hipStream_t s = p->stream;
  PH(hipMemcpyAsync(H->st_h, I.st, sizeof(RtState), hipMemcpyDeviceToHost, s));
  PH(hipStreamSynchronize(s));
  const RtState st = *H->st_h;
  const int rom = (I.method == RT_ROM);
  const int mixed = (I.precision == RT_MIXED);
  const int cur = (int)(st.steps & 1);
  const double *bt = I.bt2[cur];
  static const char *const phase_names[] = {"rtrom_step phase 0", "rtrom_step phase 1", "rtrom_step phase 2",
                                            "rtrom_step phase 3", "rtrom_step phase 4", "rtrom_step phase 5",
                                            "rtrom_step phase 6"};
  const RtRange range(phase_names[std::min(6, std::max(0, st.phase))]);
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
  if (H->mh) hipLaunchKernelGGL(k_mh_reset, dim3(1), dim3(64), 0, s, H->mh);  // a model per step
  int nsweep = 0, n32 = 0, conv = 0, used_pc = 0, pc_fb = 0, exact = 0, first_corr = 1, need64 = 1;
  int ncorr = 0, used_mask = 0, lv_fb = 0;  // corrections so far; levels applied (bit l - 1)
  int last_exact = 0;                       // whether the previous checked iterate came from an FP64 sweep
  double resid = 0.0;
  for (;;) {
    if (need64) {  // y = T (sigma_s rp) + b~ in FP64
      hipLaunchKernelGGL((k_skew<double, 1>), qgrid, dim3(BLK), 0, s, A, I.ss, (const double *)H->rp,
                         (const double *)nullptr, (double *)A.srcq);
      int e = sweep_moment(p, H, 0, 0, H->y, bt, 0, H->rp, H->blkmax);
      if (e) return e;
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
    const double tt = exact ? I.tol_cert : I.tol32;
    const bool pass = yn > 0.0 ? (dn < tt * yn) : (dn < tt);
    if (pass) {
      if (exact) {
        conv = 1;
        break;
      }
      if (nsweep >= I.max_iter) break;
      need64 = 1;  // certify the FP32-refined iterate with an FP64 sweep
      continue;
    }
    if (nsweep >= I.max_iter) break;
    if (H->mh) {
      // McClarren-Haut: the pair of this iteration, (rho^{(l-1)} - rho^{(l-2)},
      // y_l - y_{l-1}); in mixed precision an iterate recomputed by an FP64
      // sweep after FP32 increments starts a new chain instead (its
      // difference to the accumulated y_{l-1} would carry that chain's drift)
      if (nsweep >= 2 && !(mixed && exact && !last_exact)) {
        const double *rp_ = H->rp, *y_ = H->y;
        hipLaunchKernelGGL(k_mh_pass1, dim3(nblk), dim3(BLK), 0, s, I, nc, rp_, (const double *)H->rp2, y_,
                           (const double *)H->yp, H->mh, H->rpart);
        hipLaunchKernelGGL(k_mh_small1, dim3(1), dim3(256), 0, s, I, nblk, (const double *)H->rpart, H->mh);
        hipLaunchKernelGGL(k_mh_pass2, dim3(nblk), dim3(BLK), 0, s, I, nc, rp_, (const double *)H->rp2,
                           (const MhGrid *)H->mh, H->rpart);
        hipLaunchKernelGGL(k_mh_small2, dim3(1), dim3(256), 0, s, nblk, (const double *)H->rpart, H->mh);
        hipLaunchKernelGGL(k_mh_pass3, dim3(nblk), dim3(BLK), 0, s, I, nc, rp_, (const double *)H->rp2, y_,
                           (const double *)H->yp, (const MhGrid *)H->mh, H->rpart);
        hipLaunchKernelGGL(k_mh_small3, dim3(1), dim3(256), 0, s, nblk, (const double *)H->rpart, H->mh);
      }
      hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, H->yp);
      hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->rp, H->rp2);
      PH(hipGetLastError());
    }
    last_exact = exact;
    const double *dcorr = nullptr;
    // correction l = ncorr + 1 of the step.  Level l of the correction ROMs
    // (Sec. 3.2, key feature 1) keeps y_l = rho^{(l-1/2)} and rho^{(l-1)}
    // for its pair, and applies when complete and level l - 1 applied
    // before it.
    const int lc = ncorr + 1;
    bool lev_apply = false;
    if (rom && lc >= 2 && lc <= I.nlev) {
      const int k = lc - 2;
      hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, I.ylev[k]);
      hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->rp, I.rlev[k]);
      // mixed precision: a level ROM is built from and applied to FP64-swept
      // iterates only (an FP32-refined one carries its increments' rounding)
      if (exact) used_mask |= 1 << (8 + k);
      const bool due = st.flag_pl[k] && ((used_mask >> (lc - 2)) & 1) && (!mixed || exact);
      if (due && !st.lu_ok_pl[k]) lv_fb++;
      lev_apply = due && st.lu_ok_pl[k];
    }
    if (lev_apply) {
      // ROM-enhanced correction of iteration lc (eq. dmd-sa at iteration lc)
      const int k = lc - 2;
      rt_prof_begin(RT_K_PLANE_OTHER, s);
      hipLaunchKernelGGL(k_plane_sub, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y,
                         (const double *)H->rp, I.wlev[k]);
      e = rom_apply_grid(p, H, I.pl[k], &I.st->rank_pl[k], I.wlev[k], I.dlev[k]);
      rt_prof_end(RT_K_PLANE_OTHER, s);
      if (e) return e;
      dcorr = I.dlev[k];
      used_mask |= 1 << (lc - 1);
    } else if (rom && first_corr && st.flag_pc && st.lu_ok_pc) {
      rt_prof_begin(RT_K_PLANE_OTHER, s);
      hipLaunchKernelGGL(k_plane_sub, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y,
                         (const double *)I.rho0, I.work);
      e = rom_apply_grid(p, H, I.pc, &I.st->rank_pc, I.work, I.dpc);
      rt_prof_end(RT_K_PLANE_OTHER, s);
      if (e) return e;
      dcorr = I.dpc;
      used_pc = 1;
      used_mask |= 1;
    } else if (I.method != RT_SI_PLAIN) {
      if (rom && first_corr && st.flag_pc) pc_fb = 1;
      if (H->mh) {
        // McClarren-Haut correction from the step's pairs (Sec. 3.3)
        rt_prof_begin(RT_K_PLANE_OTHER, s);
        hipLaunchKernelGGL(k_mh_cpass, dim3(nblk), dim3(BLK), 0, s, I, nc, (const double *)H->y,
                           (const double *)H->rp, (const MhGrid *)H->mh, H->rpart);
        hipLaunchKernelGGL(k_mh_csolve, dim3(1), dim3(256), 0, s, nblk, (const double *)H->rpart, H->mh);
        hipLaunchKernelGGL(k_mh_expand, dim3(nblk), dim3(BLK), 0, s, I, nc, (const MhGrid *)H->mh, H->cx);
        rt_prof_end(RT_K_PLANE_OTHER, s);
        PH(hipGetLastError());
      } else {
        rt_prof_begin(RT_K_PLANE_DSA, s);
        e = dsa_solve(p, H, H->y, H->rp);
        rt_prof_end(RT_K_PLANE_DSA, s);
        if (e) return e;
      }
      dcorr = H->cx;
    }
    first_corr = 0;
    ncorr++;
    if (mixed && !(exact && resid < RT_FP64_BAND * I.tol)) {  // y += T (sigma_s (rp_new - rp)), increment in FP32
      hipLaunchKernelGGL(k_plane_increment, dim3(nblk), dim3(BLK), 0, s, nc, I.ss, (const double *)H->y, dcorr,
                         H->rp, H->src32);
      hipLaunchKernelGGL((k_skew<float, 0, float>), qgrid, dim3(BLK), 0, s, A, (const double *)nullptr,
                         (const float *)H->src32, (const double *)nullptr, (float *)A.srcq);
      e = sweep_moment(p, H, 0, 1, H->y, nullptr, 1, H->rp, H->blkmax);
      if (e) return e;
      exact = 0;
      n32++;
      nsweep++;
    } else {
      hipLaunchKernelGGL(k_plane_correct, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, dcorr, H->rp);
      need64 = 1;
    }
  }
  hipLaunchKernelGGL(k_plane_copy, dim3(nblk), dim3(BLK), 0, s, nc, (const double *)H->y, I.rho);
  hipLaunchKernelGGL(k_plane_status, dim3(1), dim3(1), 0, s, I.st, nsweep, conv, used_pc, ig_fb, pc_fb, resid, n32,
                     used_mask, lv_fb);
  PH(hipGetLastError());
  // ROM bookkeeping on the auxiliary stream, concurrent with the f-pass
  hipStream_t s2 = rom ? p->aux_stream : s;
  if (s2 != s) {
    PH(hipEventRecord(p->ev_si, s));
    PH(hipStreamWaitEvent(s2, p->ev_si, 0));
  }
  rt_prof_begin(RT_K_POST, s2);
  PH(rt_launch_rom(p->dinst, 1, nc, rom, 1 + I.nlev, s2));
  rt_prof_end(RT_K_POST, s2);
  if (rom) {
    rt_prof_begin(RT_K_ROM_UPDATE, s2);
    PH(rt_launch_rom_update(p->dinst, 1, nc, 1 + I.nlev, s2));
    rt_prof_end(RT_K_ROM_UPDATE, s2);
  }
  hipLaunchKernelGGL((k_skew<double, 2>), qgrid, dim3(BLK), 0, s, A, I.ss, (const double *)I.rho, I.G, A.s1q);
  int e;
  if (I.bdf2 && st.steps == 0) {
    // BDF2's backward-Euler start: f^1 over f with f^0 kept as the older
    // level, then the BDF2 operator and the right-hand side of step 2
    PH(hipMemcpyAsync(A.fo, A.f, (size_t)A.ndf * A.SQ * 8, hipMemcpyDeviceToDevice, s));
    e = sweep_moment(p, H, 1, 0, I.bt2[cur ^ 1], nullptr, 0, nullptr, nullptr);
    if (!e) e = plane_bdf2_operator(p, H);
    if (!e) e = sweep_moment(p, H, 4, 0, I.bt2[cur ^ 1], nullptr, 0, nullptr, nullptr);
  } else if (I.bdf2) {
    e = sweep_moment(p, H, 3, 0, I.bt2[cur ^ 1], nullptr, 0, nullptr, nullptr);
    std::swap(A.f, A.fo);  // f^n was written over f^{n-2}
  } else {
    e = sweep_moment(p, H, 1, 0, I.bt2[cur ^ 1], nullptr, 0, nullptr, nullptr);
  }
  if (e) return e;
  if (s2 != s) {
    PH(hipEventRecord(p->ev_rom, s2));
    PH(hipStreamWaitEvent(s, p->ev_rom, 0));
  }
  return RTROM_OK;
}

int rt_plane_dsa_iters(const rtrom_problem *p) {
  const PlaneHost *H = (const PlaneHost *)p->plane;
  return H ? H->cheb_iters : 0;
}

int rt_plane_step(rtrom_problem *p, int nsteps) {
  PlaneHost *H = (PlaneHost *)p->plane;
  for (int k = 0; k < nsteps; ++k) {
    int e = plane_one_step(p, H);
    if (e) return e;
  }
  return RTROM_OK;
}

// folded, skewed f -> full ordinate order, cell layout (host)
int rt_plane_unfold(const rtrom_problem *p, double *f_host) {
  const PlaneHost *H = (const PlaneHost *)p->plane;
  const PlaneArgs &A = H->A;
  const size_t nc = (size_t)p->nc, SQ = (size_t)A.SQ;
  std::vector<double> tmp((size_t)H->ndf * SQ);
  PH(hipMemcpyAsync(tmp.data(), A.f, tmp.size() * 8, hipMemcpyDeviceToHost, p->stream));
  PH(hipStreamSynchronize(p->stream));
  for (int j = 0; j < p->nv; ++j) {
    const int dir = H->fold_of[j], q = H->quad[dir];
    const double *src = tmp.data() + (size_t)dir * SQ;
    for (int iy = 0; iy < A.ny; ++iy)
      for (int ix = 0; ix < A.nx; ++ix) {
        const int u = (q & 2) ? A.ny - 1 - iy : iy;
        const int a = (q & 1) ? A.nx - 1 - ix : ix;
        const size_t slot = ((size_t)(u / BAND) * A.TT + a + (u % BAND)) * BAND + (u % BAND);
        f_host[(size_t)j * nc + (size_t)iy * A.nx + ix] = src[slot];
      }
  }
  return RTROM_OK;
}
