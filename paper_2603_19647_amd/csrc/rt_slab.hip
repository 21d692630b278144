// rt_slab.hip -- slab (1D) kernels of librtrom for gfx950.
//
// One workgroup owns one problem instance; thread t owns the contiguous cells
// [t*C, t*C + C) for the whole step, so every per-cell vector of the source
// iteration (rho, y, b~, sigma's) lives in registers.  Each upwind sweep
// (Sec. 2.3: one pass of block Gauss-Seidel in upwind order) is the affine
// recurrence f_i = a_i f_{i-1} + b_i of first-order upwind finite volumes,
// evaluated as a workgroup-wide affine prefix scan (wg_scan2).  The two
// ordinates of a mirror pair (mu, -mu) share a_i and the reciprocal of
// (sigma_t + 1/dt + |mu|/h) and are scanned together in opposite directions.
//
// A problem marched on its own may instead run its SI loop cooperatively on
// ng workgroups (k_si_slab<..., true>): workgroup g sweeps ordinate-pair group
// g and every workgroup keeps the full per-cell state, so after each sweep
// the groups' moments are exchanged (agent-scope atomic stores and loads,
// coherent across the L2 slices, then a grid barrier) and every workgroup
// continues with the same data and takes the same decisions.  DMD guesses
// are computed by cell slices and exchanged the same way.
#include <algorithm>

#include "rt_common.h"
#include "rt_dsa.h"
#include "rt_rom.h"

namespace {

// Threads per workgroup of the cooperative step tail (k_tail_coop); its ROM
// passes use one partial row per TAIL_NT cells.
constexpr int TAIL_NT = 512;

template <typename R>
__device__ __forceinline__ R *coop_part(const Inst &I);
template <>
__device__ __forceinline__ double *coop_part<double>(const Inst &I) { return I.sip; }
template <>
__device__ __forceinline__ float *coop_part<float>(const Inst &I) { return I.sip32; }
template <typename R>
__device__ __forceinline__ R *coop_sums(const Inst &I);
template <>
__device__ __forceinline__ double *coop_sums<double>(const Inst &I) { return I.sips; }
template <>
__device__ __forceinline__ float *coop_sums<float>(const Inst &I) { return I.sips32; }

// ---------------------------------------------------------------------------
// Sweep with an ordinate-independent source s and zero inflow, returning the
// angular moment acc = sum_j w_j f_j (the operator T of Sec. 2.3 applied to s).
// COOP: this workgroup sweeps its pair group only, then the groups' moments
// are summed in group order (the same sum in every workgroup).
// ---------------------------------------------------------------------------
template <int CMAX, typename R, bool COOP>
__device__ __forceinline__ void sweep_moment(const Inst &I, const R (&ct)[CMAX], const R (&s)[CMAX], int n, int c0,
                                             R (&acc)[CMAX], R *slots, int &parity, CoopSync &cs) {
#pragma unroll
  for (int t = 0; t < CMAX; ++t) acc[t] = R(0);
  int p0 = 0, p1 = I.npair;
  if constexpr (COOP) {
    p0 = blockIdx.x * I.pg;
    p1 = min(I.npair, p0 + I.pg);
  }
  for (int p = p0; p < p1; ++p) {
    const R m = (R)ldg(&I.pm[p]);
    const R w = (R)ldg(&I.pw[p]);
    R a[CMAX], b[CMAX];
    R Af = R(1), Bf = R(0);
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      if (t < n) {
        R inv = rt_rcp(ct[t] + m);
        a[t] = m * inv;
        b[t] = s[t] * inv;
        Bf = rt_fma(a[t], Bf, b[t]);
        Af = a[t] * Af;
      }
    }
    R Ab = R(1), Bb = R(0);
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t) {
      if (t < n) {
        Bb = rt_fma(a[t], Bb, b[t]);
        Ab = a[t] * Ab;
      }
    }
    R inF, inB;
    wg_scan2<R>(Af, Bf, Ab, Bb, R(0), R(0), inF, inB, slots, parity);
    parity ^= 1;
    R f = inF;
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      if (t < n) {
        f = rt_fma(a[t], f, b[t]);
        acc[t] = rt_fma(w, f, acc[t]);
      }
    }
    f = inB;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t) {
      if (t < n) {
        f = rt_fma(a[t], f, b[t]);
        acc[t] = rt_fma(w, f, acc[t]);
      }
    }
  }
  if constexpr (COOP) {
    // the groups' moments are added in group order by a reduce-scatter
    // (workgroup g adds the cells [g*S, g*S + S)) and an all-gather of the
    // sums: each workgroup reads 2 nc values instead of ng * nc
    const int nc = I.nc, ng = I.ng;
    R *part = coop_part<R>(I) + (size_t)cs.buf * ng * nc;
    R *sums = coop_sums<R>(I) + (size_t)cs.buf * nc;
    cs.buf ^= 1;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
      if (t < n) xstore(&part[(size_t)blockIdx.x * nc + c0 + t], acc[t]);
    grid_sync(cs);
    const int S = (nc + ng - 1) / ng, lo = blockIdx.x * S, hi = min(nc, lo + S);
    for (int c = lo + (int)threadIdx.x; c < hi; c += blockDim.x) {
      // every group's partial in flight together (past ng clamped, masked)
      R v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = xload(&part[(size_t)min(q, ng - 1) * nc + c]);
      R sv = R(0);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < ng) sv += v[q];
      xstore(&sums[c], sv);
    }
    grid_sync(cs);
#pragma unroll
    for (int t = 0; t < CMAX; ++t) acc[t] = (t < n) ? xload(&sums[c0 + t]) : R(0);
  }
}

// DMD application (eq. dmd-ig, eq. dmd-sa) by cell slices: workgroup g
// projects and expands the cells [g*cs, g*cs + cs); the coefficient partials
// and the expanded vector are exchanged like the sweep moments.  out is
// written with agent-scope stores; read it with xload.
__device__ inline void rom_apply_coop(const Inst &I, const RomDev &R, int rank, const double *rhs, double *out,
                                      double *red, double *vec, double *luS, int *permS, CoopSync &cs) {
  // the LU factors go to LDS first: their loads overlap the projection
  for (int e = threadIdx.x; e < RT_RMAX * RT_RMAX; e += blockDim.x) luS[e] = ldg(&R.LU[e]);
  if ((int)threadIdx.x < RT_RMAX) permS[threadIdx.x] = ldg(&R.perm[threadIdx.x]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nc = I.nc, ng = I.ng, ld = I.ld, NT = blockDim.x;
  const int csz = (nc + ng - 1) / ng;
  const int lo = blockIdx.x * csz, hi = min(nc, lo + csz);
  double *apx = I.apx + (size_t)cs.buf * ng * RT_RMAX;
  cs.buf ^= 1;
  static_assert(RT_RMAX == 20, "four column groups of five");
  if (nw % 4 == 0) {
    // the waves split into four column groups of five columns: every thread
    // has its five loads in flight at once (columns past the rank hold finite
    // values; their sums are not used)
    const int cg = wave & 3, sub = wave >> 2, nsub = nw >> 2;
    double sacc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = lo + sub * 64 + lane; c < hi; c += nsub * 64) {
      const double v = ldg(&rhs[c]);
      double u[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) u[q] = ldg(&R.U[(size_t)(cg * 5 + q) * ld + c]);
#pragma unroll
      for (int q = 0; q < 5; ++q) sacc[q] = rt_fma(u[q], v, sacc[q]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const double t = wave_sum_fast(sacc[q]);
      if (lane == 0) red[wave * 5 + q] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < rank) {
      const int k = threadIdx.x, kg = k / 5, kq = k % 5;
      double sv = 0.0;
      for (int sb = 0; sb < nsub; ++sb) sv += red[(sb * 4 + kg) * 5 + kq];
      xstore(&apx[(size_t)blockIdx.x * RT_RMAX + k], sv);
    }
  } else {
    for (int k0 = 0; k0 < rank; k0 += 4) {
      double sacc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int c = lo + (int)threadIdx.x; c < hi; c += NT) {
        const double v = ldg(&rhs[c]);
        double u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = ldg(&R.U[(size_t)(k0 + q) * ld + c]);
#pragma unroll
        for (int q = 0; q < 4; ++q) sacc[q] = rt_fma(u[q], v, sacc[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double t = wave_sum_fast(sacc[q]);
        if (lane == 0) red[wave * RT_RMAX + k0 + q] = t;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < rank) {
      double sv = 0.0;
      for (int w = 0; w < nw; ++w) sv += red[w * RT_RMAX + threadIdx.x];
      xstore(&apx[(size_t)blockIdx.x * RT_RMAX + threadIdx.x], sv);
    }
  }
  grid_sync(cs);
  if ((int)threadIdx.x < RT_RMAX) {
    double sv = 0.0;
    if ((int)threadIdx.x < rank) {
      // groups in order, sixteen loads in flight per batch (clamped, masked)
      for (int g0 = 0; g0 < ng; g0 += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = xload(&apx[(size_t)min(g0 + q, ng - 1) * RT_RMAX + threadIdx.x]);
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (g0 + q < ng) sv += v[q];
      }
    }
    vec[threadIdx.x] = sv;  // zero past the rank
  }
  __syncthreads();
  lu_solve_wave(luS, permS, rank, vec);
  // expansion: four lanes of a quad per cell, five columns each (all loads
  // in flight at once), the quad's partial sums added in a fixed order
  static_assert(RT_RMAX == 20, "four quarters of five columns");
  {
    const int q4 = threadIdx.x & 3, k0 = 5 * q4;
    double y5[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) y5[q] = vec[k0 + q];
    for (int cb = lo; cb < hi; cb += NT / 4) {
      const int c = cb + (int)(threadIdx.x >> 2);
      const int cc = min(c, hi - 1);
      double u[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) u[q] = ldg(&R.U[(size_t)(k0 + q) * ld + cc]);
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < 5; ++q) v = rt_fma(u[q], y5[q], v);
      v = QuadSum()(v);
      if (q4 == 0 && c < hi) xstore(&out[c], v);
    }
  }
  grid_sync(cs);
}

// ---------------------------------------------------------------------------
// The incremental SVD's two projection passes (App. B: classical
// Gram-Schmidt applied twice; the rotation applies the second step's
// correction) run at the end of the cooperative SI kernel, so the step tail
// starts with the small dense cores.  Unit (z, blk): ROM z over the cells
// [blk*H, blk*H + H), H = 64*hw cells with hw = nw/2 waves per half; the
// units are dealt over the ng workgroups.  The first hw waves take basis
// columns 0..9 of the block's cells, the next hw waves columns 10..19 (a
// wave past 2*hw idles), so a thread keeps 22 partial sums: the 1024-thread
// kernel's register budget.  A one-wave workgroup (hw = 0, H = 64) takes the
// two halves in turn.  Row blk of part1 / part2 gets the same sums as
// rom_pass1 / rom_pass2 (layout [U^T x | U^T b | x.x | x.b] and
// [U^T v | W^T v | v.v | v.b]), stored with agent-scope atomics.
// ---------------------------------------------------------------------------
constexpr int PASS_COLS = RT_RMAX / 2;
constexpr int PASS_NACC = 2 * PASS_COLS + 2;

struct PassGeom {
  int hw;   // waves per half (0: one wave takes both halves)
  int H;    // cells per block
  int h;    // this thread's half (2: idle), when hw > 0
  int cl;   // this thread's cell in the block
  int nit;  // halves per thread: 1, or 2 when hw = 0
};
__device__ __forceinline__ PassGeom pass_geom() {
  const int hw = (int)(blockDim.x >> 7), wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (hw == 0) return {0, 64, 0, lane, 2};
  const int h = min(2, wave / hw);
  return {hw, 64 * hw, h, (wave - h * hw) * 64 + lane, 1};
}
__host__ __device__ inline int coop_pass_blocks(int nc, int nthr) {
  const int H = 64 * (nthr >= 128 ? nthr / 128 : 1);
  return (nc + H - 1) / H;
}

// one half's accumulators: the four 16-lane row sums of each (DPP) into slot
// vw of red (4 * PASS_NACC doubles per slot)
__device__ __forceinline__ void pass_wave_sums(const double (&acc)[PASS_NACC], int vw, double *red) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < PASS_NACC; ++k) {
    const double t = row16_sum(acc[k]);
    if ((lane & 15) == 0) red[(vw * 4 + (lane >> 4)) * PASS_NACC + k] = t;
  }
}
// Row blk of part: entry k of the 2R+2 sums is the sum over its half's slots
// and their rows (in order) of that half's accumulator.
__device__ __forceinline__ void pass_rows(int hw, double *red, double *part, int blk) {
  __syncthreads();
  const int k = threadIdx.x, nv = 4 * max(hw, 1);
  if (k < 2 * RT_RMAX + 2) {
    int hh, ai;
    if (k < 2 * RT_RMAX) {
      const int j = k % RT_RMAX;  // column
      hh = j / PASS_COLS;
      ai = (k < RT_RMAX ? 0 : PASS_COLS) + j % PASS_COLS;
    } else {
      hh = 0;
      ai = 2 * PASS_COLS + (k - 2 * RT_RMAX);
    }
    double s = 0.0;
    for (int w = hh * nv; w < hh * nv + nv; ++w) s += red[w * PASS_NACC + ai];
    xstore(&part[blk * RT_NPART + k], s);
  }
  __syncthreads();
}
// columns k0..k0+9 of X at cell cc, zero past the rank or outside the block
__device__ __forceinline__ void pass_cols(const double *X, int ld, int cc, int k0, bool in, int rank,
                                          double (&u)[PASS_COLS]) {
#pragma unroll
  for (int q = 0; q < PASS_COLS; ++q) {
    const double v = ldg(&X[(size_t)(k0 + q) * ld + cc]);
    u[q] = (in && k0 + q < rank) ? v : 0.0;
  }
}

// Pass 1 of unit (z, blk): U^T x, U^T b, x.x, x.b of ROM z's snapshot pair
// (IG: x = rho^n, b = b~^{n-1}; PC: x = rho^n - rho^(1/2), b = rho^(1/2) -
// rho^(0), eq. correction_snapshot, also stored for pass 2 and the rotation).
// rho^n and rho^(1/2) were written by this workgroup; rho^(0) by any.
__device__ inline void coop_pass1(const Inst &I, int z, int blk, int rank, const double *bt, double *red) {
  const PassGeom G = pass_geom();
  const int nc = I.nc, ld = I.ld;
  const int c = blk * G.H + G.cl;
  const bool in = G.h < 2 && c < nc;
  const int cc = min(c, nc - 1);
  const RomDev &R = z ? I.pc : I.ig;
  double xv, bv;
  if (z == 0) {
    xv = ldg(&I.rho[cc]);
    bv = ldg(&bt[cc]);
  } else {
    const double rh = ldg(&I.rhalf[cc]);
    xv = ldg(&I.rho[cc]) - rh;
    bv = rh - xload(&I.rho0[cc]);
    if (in && G.h == 0) {
      xstore(I.work + 2 * (size_t)nc + c, xv);
      xstore(I.work + 3 * (size_t)nc + c, bv);
    }
  }
  if (!in) xv = bv = 0.0;
  for (int i = 0; i < G.nit; ++i) {
    const int hh = G.hw ? min(G.h, 1) : i;
    double u[PASS_COLS], acc[PASS_NACC];
    pass_cols(R.U, ld, cc, hh * PASS_COLS, in, rank, u);
#pragma unroll
    for (int q = 0; q < PASS_COLS; ++q) {
      acc[q] = u[q] * xv;
      acc[PASS_COLS + q] = u[q] * bv;
    }
    acc[2 * PASS_COLS] = xv * xv;
    acc[2 * PASS_COLS + 1] = xv * bv;
    pass_wave_sums(acc, G.hw ? (int)(threadIdx.x >> 6) : i, red);
  }
  pass_rows(G.hw, red, R.work->part1, blk);
}

// Pass 2 of unit (z, blk): v = x - U a1 (a1 = U^T x from pass 1's rows,
// columns in order), stored as the ROM's projected residual, and U^T v,
// W^T v, v.v, v.b.  The loads are issued before a1 is summed.  scr:
// blockDim doubles of LDS.
__device__ inline void coop_pass2(const Inst &I, int z, int blk, int nb, int rank, const double *bt, double *red,
                                  double *av, double *scr) {
  const PassGeom G = pass_geom();
  const int nc = I.nc, ld = I.ld;
  const RomDev &R = z ? I.pc : I.ig;
  const int c = blk * G.H + G.cl;
  const bool in = G.h < 2 && c < nc;
  const int cc = min(c, nc - 1);
  double xv = z ? xload(I.work + 2 * (size_t)nc + cc) : ldg(&I.rho[cc]);
  double bv = z ? xload(I.work + 3 * (size_t)nc + cc) : ldg(&bt[cc]);
  if (!in) xv = bv = 0.0;
  const int kh = min(G.h, 1) * PASS_COLS;
  double u[PASS_COLS], w[PASS_COLS];
  if (G.hw) {
    pass_cols(R.U, ld, cc, kh, in, rank, u);
    pass_cols(R.W, ld, cc, kh, in, rank, w);
  }
  sum_partials<true>(R.work->part1, nb, RT_RMAX, av, scr);  // zero past the rank
  // v = x - sum_k u_k a1_k, columns in order (the second half continues
  // from the first half's value)
  double v = xv;
  if (G.hw) {
    if (G.h == 0) {
#pragma unroll
      for (int q = 0; q < PASS_COLS; ++q) v = rt_fma(-u[q], av[q], v);
      scr[G.cl] = v;
    }
    __syncthreads();
    if (G.h == 1) {
      v = scr[G.cl];
#pragma unroll
      for (int q = 0; q < PASS_COLS; ++q) v = rt_fma(-u[q], av[PASS_COLS + q], v);
      scr[G.cl] = v;
    }
    __syncthreads();
    v = G.h < 2 ? scr[G.cl] : 0.0;
  } else {
    for (int hh = 0; hh < 2; ++hh) {
      pass_cols(R.U, ld, cc, hh * PASS_COLS, in, rank, u);
#pragma unroll
      for (int q = 0; q < PASS_COLS; ++q) v = rt_fma(-u[q], av[hh * PASS_COLS + q], v);
    }
  }
  const double *p = I.work + (size_t)(z ? 1 : 4) * nc;  // as rom_decide sets RomWork.p
  if (in && G.h == 0) xstore(const_cast<double *>(p) + c, v);  // first Gram-Schmidt residual
  for (int i = 0; i < G.nit; ++i) {
    if (!G.hw) {
      pass_cols(R.U, ld, cc, i * PASS_COLS, in, rank, u);
      pass_cols(R.W, ld, cc, i * PASS_COLS, in, rank, w);
    }
    double acc[PASS_NACC];
#pragma unroll
    for (int q = 0; q < PASS_COLS; ++q) {
      acc[q] = u[q] * v;
      acc[PASS_COLS + q] = w[q] * v;
    }
    acc[2 * PASS_COLS] = v * v;
    acc[2 * PASS_COLS + 1] = v * bv;
    pass_wave_sums(acc, G.hw ? (int)(threadIdx.x >> 6) : i, red);
  }
  pass_rows(G.hw, red, R.work->part2, blk);
}

}  // namespace

// ---------------------------------------------------------------------------
// k_si_slab: initial guess + Alg. 1 (SI with DSA, or the hybrid ROM/DSA
// preconditioner of Sec. 3.2 phase 3) for every instance of the launch, then
// the step's error indicators and Alg. 2's decisions (rom_decide).  Writes
// rho^n, rho^{(0)}, rho^{(1/2)}, the PC correction and per-step status.
// COOP: one instance on gridDim.x = ng workgroups (see the file comment);
// workgroup 0 writes the state and results.
// ---------------------------------------------------------------------------
template <int CMAX, int MAXT, bool COOP>
__global__ void __launch_bounds__(MAXT) k_si_slab(const Inst *__restrict__ insts) {
  const Inst &I = insts[COOP ? 0 : blockIdx.x];
  __shared__ double slots[8 * RT_MAXWAVES];
  __shared__ float slotsf[8 * RT_MAXWAVES];
  __shared__ double red[2 * RT_MAXWAVES];
  __shared__ double rred[RT_MAXWAVES * RT_RMAX];
  __shared__ double rvec[RT_RMAX + 4];
  __shared__ double luS[COOP ? RT_RMAX * RT_RMAX : 1];
  __shared__ int permS[COOP ? RT_RMAX : 1];
  const int NT = I.nthr, tid = threadIdx.x;
  const int nc = I.nc;
  const int C = (nc + NT - 1) / NT;
  const int c0 = tid * C;
  const int n = max(0, min(C, nc - c0));
  const bool leader = !COOP || blockIdx.x == 0;
  RtState *st = I.st;
  const int rom = (I.method == RT_ROM);
  const int flag_ig = st->flag_ig, flag_pc = st->flag_pc;
  const int lu_ig = st->lu_ok_ig, lu_pc = st->lu_ok_pc;
  const int rank_ig = st->rank_ig, rank_pc = st->rank_pc;
  const int mixed = (I.precision == RT_MIXED);
  // counters as the step starts (the end-of-step bookkeeping adds to them
  // without reading back what this launch writes)
  const long long steps0 = st->steps, si0 = st->si_total, sw0 = st->sweeps_total, f32_0 = st->fp32_sweeps;
  const int nonconv0 = st->nonconv, fb0 = st->fallbacks;
  const int cur = (int)(steps0 & 1);
  const double *__restrict__ bt = I.bt2[cur];
  CoopSync cs{nullptr, 0ull, nullptr, 0};
  if constexpr (COOP) {
    // a barrier that gave up left the counters out of step: the state is
    // invalid (the host reports it) and later launches do nothing
    // (plain loads: both were written by earlier launches)
    if (st->fault) return;
    cs.bar = I.bar;
    cs.gen = I.bar[2];
    cs.fault = &st->fault;
  }
  // a vector the cooperative DMD apply wrote (other workgroups' slices)
  auto rd = [&](const double *p) { return COOP ? xload(p) : *p; };

  // initial guess: DMD when the IG ROM is available (eq. dmd-ig), else rho^{n-1}
  int ig_fb = 0;
  if (rom && flag_ig && lu_ig) {
    if constexpr (COOP) rom_apply_coop(I, I.ig, rank_ig, bt, I.rho0, rred, rvec, luS, permS, cs);
    else rom_apply(I.ig, rank_ig, I.ld, nc, NT, bt, I.rho0, rred, rvec);
  } else {
    ig_fb = rom && flag_ig;
    // every workgroup copies (the same values; agent-scope stores, like the
    // cooperative DMD output, so later reads see them wherever they land)
    for (int c = c0; c < c0 + n; ++c) {
      if constexpr (COOP) xstore(&I.rho0[c], ldg(&I.rho[c]));
      else stg(&I.rho0[c], ldg(&I.rho[c]));
    }
  }
  double ct[CMAX], ss[CMAX], rp[CMAX], y[CMAX];
#pragma unroll
  for (int t = 0; t < CMAX; ++t) {
    const bool in = t < n;
    ct[t] = in ? ldg(&I.ct[c0 + t]) : 1.0;
    ss[t] = in ? ldg(&I.ss[c0 + t]) : 0.0;
    rp[t] = in ? rd(&I.rho0[c0 + t]) : 0.0;
    y[t] = 0.0;
  }
  int parity = 0, parityf = 0;
  int nsweep = 0, n32 = 0, conv = 0, used_pc = 0, pc_fb = 0, exact = 0, first_corr = 1;
  int need64 = 1;
  double resid = 0.0;
  for (;;) {
    if (need64) {
      // rho^{(l-1/2)} = T Sigma_s rho^{(l-1)} + b~ (eq. SI_rho) in FP64
      double s[CMAX], acc[CMAX];
#pragma unroll
      for (int t = 0; t < CMAX; ++t) s[t] = ss[t] * rp[t];
      sweep_moment<CMAX, double, COOP>(I, ct, s, n, c0, acc, slots, parity, cs);
#pragma unroll
      for (int t = 0; t < CMAX; ++t) y[t] = acc[t] + ((t < n) ? ldg(&bt[c0 + t]) : 0.0);
      if (nsweep == 0) {  // COOP: every workgroup (the same values), for its passes
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
          if (t < n) stg(&I.rhalf[c0 + t], y[t]);
      }
      nsweep++;
      exact = 1;
      need64 = 0;
    }
    double dl = 0.0, yl = 0.0;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
      if (t < n) {
        dl = fmax(dl, fabs(y[t] - rp[t]));
        yl = fmax(yl, fabs(y[t]));
      }
    double dn, yn;
    wg_max2(dl, yl, red, dn, yn);
    resid = yn > 0.0 ? dn / yn : dn;
    if (stop_test(dn, yn, exact ? I.tol_cert : I.tol32)) {
      if (exact) {
        conv = 1;
        break;
      }
      // mixed precision: the FP32-accumulated iterate passed; re-check it on
      // an FP64 sweep before accepting
      if (nsweep >= I.max_iter) break;
      need64 = 1;
      continue;
    }
    if (nsweep >= I.max_iter) break;
    // synthetic acceleration
    double d[CMAX];
    if (rom && first_corr && flag_pc && lu_pc) {
      // ROM-enhanced correction of the first iteration (eq. dmd-sa); every
      // workgroup writes the same right-hand side and reads its own copy
#pragma unroll
      for (int t = 0; t < CMAX; ++t)
        if (t < n) stg(&I.work[c0 + t], y[t] - rd(&I.rho0[c0 + t]));
      __syncthreads();
      if constexpr (COOP) rom_apply_coop(I, I.pc, rank_pc, I.work, I.dpc, rred, rvec, luS, permS, cs);
      else rom_apply(I.pc, rank_pc, I.ld, nc, NT, I.work, I.dpc, rred, rvec);
#pragma unroll
      for (int t = 0; t < CMAX; ++t) d[t] = (t < n) ? rd(&I.dpc[c0 + t]) : 0.0;
      used_pc = 1;
    } else if (I.method == RT_SI_PLAIN) {
#pragma unroll
      for (int t = 0; t < CMAX; ++t) d[t] = 0.0;
    } else {
      if (rom && first_corr && flag_pc) pc_fb = 1;
      double rhs[CMAX];
#pragma unroll
      for (int t = 0; t < CMAX; ++t) rhs[t] = ss[t] * (y[t] - rp[t]);
      dsa_solve_slab<CMAX>(I, c0, n, rhs, d, slots, parity);
    }
    first_corr = 0;
    if (mixed && !(exact && resid < RT_FP64_BAND * I.tol)) {
      // y <- y + T32 Sigma_s (rho^{(l)} - rho^{(l-1)}): increment swept in FP32
      float s32[CMAX], acc32[CMAX], ctf[CMAX];
#pragma unroll
      for (int t = 0; t < CMAX; ++t) {
        const double rn = y[t] + d[t];
        s32[t] = (float)(ss[t] * (rn - rp[t]));
        ctf[t] = (float)ct[t];
        rp[t] = rn;
      }
      sweep_moment<CMAX, float, COOP>(I, ctf, s32, n, c0, acc32, slotsf, parityf, cs);
#pragma unroll
      for (int t = 0; t < CMAX; ++t) y[t] += (double)acc32[t];
      exact = 0;
      n32++;
      nsweep++;
    } else {
#pragma unroll
      for (int t = 0; t < CMAX; ++t) rp[t] = y[t] + d[t];
      need64 = 1;
    }
  }
  // rho^n = rho^{(l-1/2)} (Alg. 1 returns the un-corrected iterate); COOP:
  // every workgroup writes it (the same values), for its passes
#pragma unroll
  for (int t = 0; t < CMAX; ++t)
    if (t < n) stg(&I.rho[c0 + t], y[t]);
  if (leader && tid == 0) {
    st->iters = nsweep;
    st->conv = conv;
    st->used_pc = used_pc;
    st->ig_fb = ig_fb;
    st->pc_fb = pc_fb;
    st->residual = resid;
    st->phase = !flag_ig ? 1 : (!flag_pc ? 2 : 3);
    st->cur = cur;
    st->fp32_sweeps = f32_0 + n32;
  }
  __syncthreads();
  // end of step: error indicators from the final iterate and Alg. 2's
  // decisions, so the ROM work that follows needs no launch of its own
  // (COOP: every workgroup computes the same sums and decisions)
  if (rom && flag_ig) {
    double part[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
      if (t < n) {
        const double r = y[t];
        part[0] = rt_fma(r, r, part[0]);
        const double e1 = rd(&I.rho0[c0 + t]) - r;
        part[1] = rt_fma(e1, e1, part[1]);
        const double e2 = rd(&I.dpc[c0 + t]) - (r - ldg(&I.rhalf[c0 + t]));
        part[2] = rt_fma(e2, e2, part[2]);
      }
    wg_sum_fast<3>(part, rred, rvec);
  }
  const int nbp = COOP ? coop_pass_blocks(nc, NT) : I.post_nb;
  if (leader)
    rom_decide(I, rvec, nbp,
               StepIn{nsweep, conv, used_pc, ig_fb, pc_fb, !flag_ig ? 1 : (!flag_pc ? 2 : 3), cur, flag_ig, flag_pc,
                      rank_ig, rank_pc, nonconv0, fb0, resid, steps0, si0, sw0});
  if constexpr (COOP) {
    // the snapshot projections of the ROMs that take one (units dealt over
    // the workgroups), so the step tail starts with the cores
    const RomPlan P = rom ? rom_plan(I, flag_ig, flag_pc, used_pc, nsweep, rvec) : RomPlan{0, 0, 0, 0, -1.0, -1.0};
    if (P.ig_on || P.pc_on) {
      __shared__ double pred[4 * RT_MAXWAVES * PASS_NACC], pav[RT_RMAX], pscr[MAXT];
      for (int it = blockIdx.x; it < 2 * nbp; it += gridDim.x) {
        const int z = it / nbp;
        if (z ? P.pc_on : P.ig_on) coop_pass1(I, z, it - z * nbp, z ? rank_pc : rank_ig, bt, pred);
      }
      grid_sync(cs);
      for (int it = blockIdx.x; it < 2 * nbp; it += gridDim.x) {
        const int z = it / nbp;
        if (z ? P.pc_on : P.ig_on) coop_pass2(I, z, it - z * nbp, nbp, z ? rank_pc : rank_ig, bt, pred, pav, pscr);
      }
    }
    if (leader && tid == 0) xstore(&I.bar[2], cs.gen);
  }
}

// ---------------------------------------------------------------------------
// k_fpass_pair: f^n from rho^n (eq. sweep_to_obtain_f) and the ordinate
// pairs' shares of the right-hand side b~^n = sum_j w_j sweep_j(f^n_j / dt +
// G, g) of the next step (Sec. 2.3).  The pairs are independent, so a launch
// spreads them over workgroups: workgroup (x, i) takes pairs [x*gp, x*gp + gp)
// of instance i.  Each pair's moment goes to fpart[p]; k_fpass_sum adds the
// pairs in a fixed order, so the result does not depend on gp.
// rhs_only: skip the first sweep and rebuild b~ from the stored f (creation,
// or a new inflow).
// ---------------------------------------------------------------------------
// One ordinate pair of the f-pass for the calling workgroup's cells: ct, G
// and srcc = sigma_s rho^n + G are the thread's cells; the pair's moment goes
// to fpart[p] (COH: agent-scope stores, for a cooperative launch).
template <int CMAX, bool COH>
__device__ __forceinline__ void fpass_one_pair(const Inst &I, int p, int c0, int n, const double (&ct)[CMAX],
                                               const double (&G)[CMAX], const double (&srcc)[CMAX], int rhs_only,
                                               double *slots, int &parity) {
  const int nc = I.nc;
  const double idt = I.inv_dt;
  const double m = ldg(&I.pm[p]), w = ldg(&I.pw[p]);
  double *fneg = I.f + (size_t)p * nc + c0;               // mu < 0
  double *fpos = I.f + (size_t)(I.nv - 1 - p) * nc + c0;  // mu > 0
  double inv[CMAX], bp[CMAX], bn[CMAX];
#pragma unroll
  for (int t = 0; t < CMAX; ++t) {
    const bool in = t < n;
    inv[t] = rt_rcp(ct[t] + m);
    bp[t] = in ? ldg(&fpos[t]) : 0.0;
    bn[t] = in ? ldg(&fneg[t]) : 0.0;
  }
  if (!rhs_only) {
    double Af = 1.0, Bf = 0.0, Ab = 1.0, Bb = 0.0;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
      if (t < n) {
        bp[t] = rt_fma(bp[t], idt, srcc[t]) * inv[t];
        const double a = m * inv[t];
        Bf = rt_fma(a, Bf, bp[t]);
        Af *= a;
      }
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
      if (t < n) {
        bn[t] = rt_fma(bn[t], idt, srcc[t]) * inv[t];
        const double a = m * inv[t];
        Bb = rt_fma(a, Bb, bn[t]);
        Ab *= a;
      }
    double inF, inB;
    wg_scan2<double>(Af, Bf, Ab, Bb, I.g[0], I.g[1], inF, inB, slots, parity);
    parity ^= 1;
    double f = inF;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
      if (t < n) {
        f = rt_fma(m * inv[t], f, bp[t]);
        bp[t] = f;
        stg(&fpos[t], f);
      }
    f = inB;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
      if (t < n) {
        f = rt_fma(m * inv[t], f, bn[t]);
        bn[t] = f;
        stg(&fneg[t], f);
      }
  }
  // right-hand-side sweep with source f^n_j / dt + G and inflow g
  double Af = 1.0, Bf = 0.0, Ab = 1.0, Bb = 0.0;
#pragma unroll
  for (int t = 0; t < CMAX; ++t)
    if (t < n) {
      bp[t] = rt_fma(bp[t], idt, G[t]) * inv[t];
      const double a = m * inv[t];
      Bf = rt_fma(a, Bf, bp[t]);
      Af *= a;
    }
#pragma unroll
  for (int t = CMAX - 1; t >= 0; --t)
    if (t < n) {
      bn[t] = rt_fma(bn[t], idt, G[t]) * inv[t];
      const double a = m * inv[t];
      Bb = rt_fma(a, Bb, bn[t]);
      Ab *= a;
    }
  double inF, inB;
  wg_scan2<double>(Af, Bf, Ab, Bb, I.g[0], I.g[1], inF, inB, slots, parity);
  parity ^= 1;
  double fw[CMAX];
  double f = inF;
#pragma unroll
  for (int t = 0; t < CMAX; ++t)
    if (t < n) {
      f = rt_fma(m * inv[t], f, bp[t]);
      fw[t] = f;
    }
  f = inB;
#pragma unroll
  for (int t = CMAX - 1; t >= 0; --t)
    if (t < n) {
      f = rt_fma(m * inv[t], f, bn[t]);
      fw[t] = w * (fw[t] + f);
    }
  double *part = I.fpart + (size_t)p * nc + c0;
#pragma unroll
  for (int t = 0; t < CMAX; ++t)
    if (t < n) {
      if constexpr (COH) xstore(&part[t], fw[t]);
      else stg(&part[t], fw[t]);
    }
}

// The thread's cells (the instance's cells split over NT threads) and the
// f-pass inputs ct, G, srcc = sigma_s rho^n + G.
template <int CMAX>
__device__ __forceinline__ void fpass_inputs(const Inst &I, int NT, int rhs_only, int &c0, int &n,
                                             double (&ct)[CMAX], double (&G)[CMAX], double (&srcc)[CMAX]) {
  const int nc = I.nc;
  const int C = (nc + NT - 1) / NT;
  c0 = threadIdx.x * C;
  n = max(0, min(C, nc - c0));
#pragma unroll
  for (int t = 0; t < CMAX; ++t) {
    const bool in = t < n;
    ct[t] = in ? ldg(&I.ct[c0 + t]) : 1.0;
    G[t] = in ? ldg(&I.G[c0 + t]) : 0.0;
    srcc[t] = (in && !rhs_only) ? rt_fma(ldg(&I.ss[c0 + t]), ldg(&I.rho[c0 + t]), G[t]) : 0.0;
  }
}

template <int CMAX, int MAXT>
__global__ void __launch_bounds__(MAXT) k_fpass_pair(const Inst *__restrict__ insts, int rhs_only, int gp) {
  const Inst &I = insts[blockIdx.y];
  const int p0 = blockIdx.x * gp;
  const int p1 = min(I.npair, p0 + gp);
  if (p0 >= p1) return;
  __shared__ double slots[8 * RT_MAXWAVES];
  int c0, n;
  double ct[CMAX], G[CMAX], srcc[CMAX];
  fpass_inputs<CMAX>(I, I.nthr, rhs_only, c0, n, ct, G, srcc);
  int parity = 0;
  for (int p = p0; p < p1; ++p) fpass_one_pair<CMAX, false>(I, p, c0, n, ct, G, srcc, rhs_only, slots, parity);
}

// ---------------------------------------------------------------------------
// k_tail_coop: everything after the SI solve of a problem marched on its own,
// in one launch of 2 + max(min(npair, 32), 4 nbp) workgroups of TAIL_NT
// threads, nbp = nc / TAIL_NT rounded up (up to eight cells per thread for
// the f-pass scans: no register spills), waiting for each other at one grid
// barrier:
//   1. workgroups 0 and 1 run the IG and PC cores (App. B) while the others
//      run the f-pass, ordinate pairs dealt round-robin;
//   2. workgroups 0 and 1 factorise the reduced operators while the others
//      rotate the bases (U and W of each ROM on their own nbp workgroups) and
//      form b~ (the pairs' sum), by cells.
// The SI kernel took the decisions and ran the projection passes (their
// partial rows and the projected residuals are read coherently).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void publish_pend(RomPend *P) {
  // the rotation is read by workgroups on other XCDs: store it again with
  // agent-scope atomics (same values) once the core has written it
  __syncthreads();
  for (int e = threadIdx.x; e < RT_KC * RT_KC; e += blockDim.x) {
    xstore(&P->Uc[e], ldg(&P->Uc[e]));
    xstore(&P->Vc[e], ldg(&P->Vc[e]));
  }
  if (threadIdx.x < RT_RMAX) xstore(&P->a2[threadIdx.x], ldg(&P->a2[threadIdx.x]));
  if (threadIdx.x == 0) {
    xstore(&P->r_old, ldg(&P->r_old));
    xstore(&P->k, ldg(&P->k));
    xstore(&P->inv_nu, ldg(&P->inv_nu));
    xstore(&P->pending, ldg(&P->pending));
  }
}

template <int CMAX, int MAXT>
__global__ void __launch_bounds__(MAXT) k_tail_coop(const Inst *__restrict__ insts) {
  static_assert(MAXT == TAIL_NT && CMAX * TAIL_NT >= RT_SLAB_MAX_CELLS, "tail layout");
  const Inst &I = insts[0];
  RtState *st = I.st;
  if (st->fault) return;  // written by an earlier launch
  __shared__ double slots[8 * RT_MAXWAVES];
  __shared__ double cc[RT_KC * RT_KC + 4], a2s[RT_RMAX];
  __shared__ RomSmem sm;
  // the tail's own barrier counters (the SI kernel's use another grid size)
  unsigned long long *bar = I.bar + 4;
  CoopSync cs{bar, bar[2], &st->fault, 0};
  const int g = blockIdx.x, G = gridDim.x, NT = blockDim.x;
  const int nc = I.nc;
  const int nbp = (nc + NT - 1) / NT;
  const int rom = I.method == RT_ROM;
  const RomWork &Wi = *I.ig.work, &Wp = *I.pc.work;
  const int act0 = rom && Wi.active, act1 = rom && Wp.active;
  // 1. cores on workgroups 0 and 1 (all but the LU of A_r), f-pass on the
  // others
  if (g < 2) {
    if (g == 0 && act0) {
      rom_core<true, true>(I, I.ig, Wi, 0, sm);
      publish_pend(I.ig.pend);
    }
    if (g == 1 && act1) {
      rom_core<true, true>(I, I.pc, Wp, 1, sm);
      publish_pend(I.pc.pend);
    }
  } else {
    int c0, n, parity = 0;
    double ct[CMAX], Gs[CMAX], srcc[CMAX];
    fpass_inputs<CMAX>(I, NT, 0, c0, n, ct, Gs, srcc);
    for (int p = g - 2; p < I.npair; p += G - 2)
      fpass_one_pair<CMAX, true>(I, p, c0, n, ct, Gs, srcc, 0, slots, parity);
  }
  grid_sync(cs);
  // 2. workgroups 0 and 1 factorise A_r; the others rotate the bases (matrix
  // mat of ROM z on workgroups 2 + [s*nbp, s*nbp + nbp), s = 2*mat + z) and
  // form b~
  if (g == 0 && act0) rom_core_lu(I, I.ig, 0, sm);
  if (g == 1 && act1) rom_core_lu(I, I.pc, 1, sm);
  const int zr = g >= 2 ? (g - 2) / nbp : 4, gr = g >= 2 ? g - 2 - zr * nbp : 0;
  if (rom && zr < 4) {
    const int z = zr & 1, mat = zr >> 1;
    const RomDev &R = z ? I.pc : I.ig;
    RomPend *P = R.pend;
    if (xload(&P->pending)) {  // uniform
      const double *src = mat ? P->Vc : P->Uc;
      for (int e = threadIdx.x; e < RT_KC * RT_KC; e += NT) cc[e] = xload(&src[e]);
      if (threadIdx.x < RT_RMAX) a2s[threadIdx.x] = xload(&P->a2[threadIdx.x]);
      __syncthreads();
      const int r = xload(&P->r_old), k = xload(&P->k);
      const int c = gr * NT + threadIdx.x;
      if (c < nc) {
        const RomWork &W = z ? Wp : Wi;
        double *X = mat ? R.W : R.U;
        double old[1][RT_RMAX], e[1];
        int cv[1] = {c};
        bool ok[1] = {true};
#pragma unroll
        for (int q = 0; q < RT_RMAX; ++q) {
          const double v = ldg(&X[(size_t)q * I.ld + c]);
          old[0][q] = q < r ? v : 0.0;
        }
        // the new direction (v - U a2) / nu for U, b for W (both written by
        // other workgroups: coherent loads)
        e[0] = mat ? xload(W.b + c) : second_residual(xload(W.p + c), old[0], a2s) * xload(&P->inv_nu);
        rotate_block<1>(old, e, cc, r, k, X, I.ld, cv, ok);
      }
    }
  }
  // b~: the pairs' moments in pair order, by cells c = (g - 2)*NT + t
  const int c = (g - 2) * NT + threadIdx.x;
  if (g >= 2 && c < nc) {
    // eight loads in flight per batch (clamped, masked)
    double acc = 0.0;
    const double *part = I.fpart + c;
    const int np = I.npair;
    for (int p0 = 0; p0 < np; p0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = xload(&part[(size_t)min(p0 + q, np - 1) * nc]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (p0 + q < np) acc += v[q];
    }
    stg(&I.bt2[st->cur ^ 1][c], acc);
  }
  if (g == 0 && threadIdx.x == 0) xstore(&bar[2], cs.gen);
}

// b~ = sum over pairs of fpart[p], in pair order, into the b~ buffer the step
// did not read (or, for rhs_only, the one the next step reads).
__global__ void __launch_bounds__(256) k_fpass_sum(const Inst *__restrict__ insts, int rhs_only) {
  const Inst &I = insts[blockIdx.y];
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= I.nc) return;
  const int nc = I.nc, np = I.npair;
  const double *part = I.fpart + c;
  double acc = 0.0;
#pragma unroll 8
  for (int p = 0; p < np; ++p) acc += ldg(&part[(size_t)p * nc]);
  double *bt_out = rhs_only ? I.bt2[I.st->steps & 1] : I.bt2[I.st->cur ^ 1];
  stg(&bt_out[c], acc);
}

// ---------------------------------------------------------------------------
// Setup: cell-centred DSA operator for finite volumes and its Thomas factors
// in affine form (serial over cells, once per problem).
// Reading of eq. rho_residual for FV: diffusion coefficient
// D = 1/(3 sigma~_t) + h/4, harmonic face coupling, Marshak vacuum faces.
// alt: the factors of the BDF2 operator (time weight 3 / (2 dt)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_setup_dsa_slab(const Inst *__restrict__ insts, int alt) {
  const Inst &I = insts[blockIdx.x];
  extern __shared__ double lds[];
  const int nc = I.nc;
  const double h = I.hx;
  double *diag = lds;       // [nc] diagonal, then the Thomas pivots d'_i
  double *q = lds + nc;     // [nc] lo_i * up_{i-1}
  double *fe = const_cast<double *>(alt ? I.dsa_fe_b : I.dsa_fe);
  double *bg = const_cast<double *>(alt ? I.dsa_bg_b : I.dsa_bg);
  double *invd = const_cast<double *>(alt ? I.dsa_invd_b : I.dsa_invd);
  const double *ct = alt ? I.ct_b : I.ct;
  const double adt = alt ? I.adt_b : I.inv_dt;
  auto Dof = [&](int i) { return 1.0 / (3.0 * ct[i]) + 0.25 * h; };
  auto face = [&](double Dp, double Dq) { return 2.0 * Dp * Dq / (h * (Dp + Dq)); };
  auto bdry = [&](double Dp) { return 2.0 * Dp / (h + 4.0 * Dp); };
  // entries of row i: lo_i = -k_{i-1/2}/h, up_i = -k_{i+1/2}/h, in parallel
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const double Di = Dof(i);
    const double kl = (i > 0) ? face(Di, Dof(i - 1)) : bdry(Di);
    const double kr = (i < nc - 1) ? face(Di, Dof(i + 1)) : bdry(Di);
    diag[i] = I.sa[i] + adt + (kl + kr) / h;
    // lo_i * up_{i-1}: both equal -k_{i-1/2}/h
    q[i] = (i > 0) ? (kl / h) * (kl / h) : 0.0;
    bg[i] = (i < nc - 1) ? -kr / h : 0.0;  // up_i for now
  }
  __syncthreads();
  // pivots d'_i = diag_i - lo_i up_{i-1} / d'_{i-1} (sequential recurrence;
  // the reciprocal of rt_rcp keeps the chain short: a prefix-product form of
  // the recurrence loses accuracy where the matrix is barely dominant)
  if (threadIdx.x == 0) {
    double dp = diag[0];
    for (int i = 1; i < nc; ++i) {
      dp = rt_fma(-q[i], rt_rcp(dp), diag[i]);
      diag[i] = dp;
    }
  }
  __syncthreads();
  // affine form: z_i = fe_i z_{i-1} + rhs_i, d_i = bg_i d_{i+1} + invd_i z_i
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const double Di = Dof(i);
    const double kl = (i > 0) ? face(Di, Dof(i - 1)) : bdry(Di);
    const double lo = (i > 0) ? -kl / h : 0.0;
    fe[i] = (i > 0) ? -lo / diag[i - 1] : 0.0;
    const double id = 1.0 / diag[i];
    invd[i] = id;
    bg[i] = -bg[i] * id;
  }
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (C linkage inside the library only)
// ---------------------------------------------------------------------------
// The SI kernel's instantiation for a launch.  The thread bound sets the
// register budget (1024 threads: 128 VGPRs, 512: 256): a launch of one
// instance with at most 512 threads takes the 512-thread build, whose state
// stays in registers (no spills); batches keep the 1024-thread build, whose
// smaller register file lets two 512-thread workgroups share a compute unit.
template <bool COOP>
static const void *si_kernel(int nthreads, int cmax, bool single) {
  if (cmax <= 4 && nthreads <= 512 && single) return reinterpret_cast<const void *>(&k_si_slab<4, 512, COOP>);
  if (cmax <= 4) return reinterpret_cast<const void *>(&k_si_slab<4, 1024, COOP>);
  return reinterpret_cast<const void *>(&k_si_slab<8, 512, COOP>);
}

extern "C" hipError_t rt_launch_slab_si(const Inst *dinsts, int ninst, int nthreads, int cmax,
                                        hipStream_t stream) {
  void *args[] = {const_cast<Inst **>(&dinsts)};
  return hipLaunchKernel(si_kernel<false>(nthreads, cmax, ninst == 1), dim3(ninst), dim3(nthreads), args, 0, stream);
}

// One instance on ng workgroups that wait for each other at grid barriers.
// They are launched as an ordinary grid: a cooperative launch guarantees
// co-residency but costs ~17 us more per launch here.  Co-residency holds
// because rt_slab_coop_fits checked at creation that the device holds every
// workgroup of both cooperative kernels at once (with ng <= 16 and tails of
// <= 34 workgroups, a small fraction of the device); should other work keep
// some of them from starting for ~2 s, the barrier waits give up, the state
// is flagged and the march reports an error instead of hanging.
extern "C" hipError_t rt_launch_slab_si_coop(const Inst *dinst, int ng, int nthreads, int cmax, hipStream_t stream) {
  void *args[] = {const_cast<Inst **>(&dinst)};
  return hipLaunchKernel(si_kernel<true>(nthreads, cmax, true), dim3(ng), dim3(nthreads), args, 0, stream);
}

static int tail_grid(int npair, int nc) {
  return 2 + std::max(std::min(npair, 32), 4 * ((nc + TAIL_NT - 1) / TAIL_NT));
}

// Whether the device holds all workgroups of the SI kernel (ng x nthreads)
// and of the step tail at once.
extern "C" int rt_slab_coop_fits(int device, int ng, int nthreads, int cmax, int npair, int nc) {
  int cus = 0, a = 0, b = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  const void *si = si_kernel<true>(nthreads, cmax, true);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, si, nthreads, 0) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void *>(&k_tail_coop<8, TAIL_NT>),
                                                   TAIL_NT, 0) != hipSuccess)
    return 0;
  return (long long)a * cus >= ng && (long long)b * cus >= tail_grid(npair, nc);
}

// gp pairs per workgroup: one when the launch has few pairs in total (every
// pair on its own compute unit), more for large batches so that each
// workgroup amortises its set-up over several pairs.
static hipError_t launch_fpass(const Inst *dinsts, int ninst, int nthreads, int cmax, int npair_max, int nc_max,
                               int rhs_only, int pairs_total, hipStream_t stream) {
  // large launches: one workgroup per instance, which computes the isotropic
  // source once for all its pairs
  const int gp = pairs_total > 4096 ? npair_max : std::max(1, std::min(npair_max, (pairs_total + 1023) / 1024));
  dim3 grid((npair_max + gp - 1) / gp, ninst), blk(nthreads);
  if (cmax <= 4)
    hipLaunchKernelGGL((k_fpass_pair<4, 1024>), grid, blk, 0, stream, dinsts, rhs_only, gp);
  else
    hipLaunchKernelGGL((k_fpass_pair<8, 512>), grid, blk, 0, stream, dinsts, rhs_only, gp);
  hipLaunchKernelGGL(k_fpass_sum, dim3((nc_max + 255) / 256, ninst), dim3(256), 0, stream, dinsts, rhs_only);
  return hipGetLastError();
}

extern "C" hipError_t rt_launch_slab_fpass(const Inst *dinsts, int ninst, int nthreads, int cmax, int npair_max,
                                           int nc_max, int pairs_total, hipStream_t stream) {
  return launch_fpass(dinsts, ninst, nthreads, cmax, npair_max, nc_max, 0, pairs_total, stream);
}

extern "C" hipError_t rt_launch_slab_rhs(const Inst *dinsts, int ninst, int nthreads, int cmax, int npair_max,
                                         int nc_max, hipStream_t stream) {
  return launch_fpass(dinsts, ninst, nthreads, cmax, npair_max, nc_max, 1, npair_max * ninst, stream);
}

// The step's tail for a problem marched on its own.
extern "C" hipError_t rt_launch_slab_tail_coop(const Inst *dinst, int npair, int nc, int nthreads, int cmax,
                                               hipStream_t stream) {
  (void)nthreads;
  (void)cmax;
  // two core workgroups + the f-pass ones, and four sets of one workgroup per
  // TAIL_NT cells (the passes of the two ROMs, the rotation of U and W of
  // each: one cell per thread); an ordinary grid, as for the SI kernel
  hipLaunchKernelGGL((k_tail_coop<8, TAIL_NT>), dim3(tail_grid(npair, nc)), dim3(TAIL_NT), 0, stream, dinst);
  return hipGetLastError();
}

extern "C" hipError_t rt_launch_slab_setup(const Inst *dinsts, int ninst, int nc_max, int alt, hipStream_t stream) {
  hipLaunchKernelGGL(k_setup_dsa_slab, dim3(ninst), dim3(1024), 2 * sizeof(double) * nc_max, stream, dinsts, alt);
  return hipGetLastError();
}
