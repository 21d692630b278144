// rt_wave.hip -- slab (1D) SI solve for instances of up to 2048 cells: one
// workgroup of eight waves per instance, the ordinate pairs spread over the
// waves.
//
// A transport sweep of one ordinate pair (Sec. 2.3: one upwind pass of block
// Gauss-Seidel per ordinate) is the affine recurrence f_i = a_i f_{i-1} + b_i
// of first-order upwind finite volumes, run forwards for mu > 0 and backwards
// for -mu; both directions share a_i = m / (sigma_t + 1/dt + m) and b_i =
// s_i / (sigma_t + 1/dt + m), m = |mu| / h.  Here one wave sweeps a whole pair
// on its own: lane l takes the C = ceil(nc / 64) consecutive cells [l C,
// l C + C), composes their maps serially, and a wave-wide affine prefix scan
// (DPP inside the 16-lane rows, lane reads across them) gives every lane the
// value entering its run -- no barrier between pairs, so the eight waves
// sweep eight pairs at once.  The moment sum_j w_j f_j accumulates in the
// wave's registers over its pairs; after the sweep the waves' partial moments
// are added through LDS in a fixed order.
//
// The per-cell data the sweeps read (sigma_t + 1/dt and the source) sit in
// LDS in the sweep layout: lane l's run at row l, padded to an odd row length
// so that a wave reading cell t of every run hits distinct banks.  Everything
// else (stop test, DSA solve, ROM corrections, Alg. 2's decisions) works on
// the cells split over the 512 threads in contiguous runs of up to four, as
// in the other slab SI kernel.
#include "rt_common.h"
#include "rt_dsa.h"
#include "rt_mh.h"
#include "rt_rom.h"

namespace {

constexpr int WNT = 512;              // threads per workgroup
constexpr int WNW = WNT / 64;         // waves
constexpr int WCM = RT_WAVE_MAX_CELLS / 64;  // cells per lane of a sweep run
constexpr int WPM = WCM + 1;          // padded LDS row (odd)
constexpr int WOWN = RT_WAVE_MAX_CELLS / WNT;  // cells per thread outside the sweeps
constexpr int WPAIRS = 128;           // ordinate pairs held in LDS (S_256)

// Exclusive affine scans of per-lane maps (A, B): x -> A x + B across one
// wave, forwards (lane 0 receives gF) and backwards (lane 63 receives gB).
template <typename R>
__device__ __forceinline__ void wave_scan2(R Af, R Bf, R Ab, R Bb, R gF, R gB, R &inF, R &inB) {
  const int lane = threadIdx.x & 63, row = lane >> 4;
  row_scan_fwd(Af, Bf);
  row_scan_bwd(Ab, Bb);
  {
    const R a0 = lane_value(Af, 15), b0 = lane_value(Bf, 15);
    const R a1 = lane_value(Af, 31), b1 = lane_value(Bf, 31);
    const R a2 = lane_value(Af, 47), b2 = lane_value(Bf, 47);
    R pA1 = a0, pB1 = b0;
    R pA2 = a1, pB2 = b1;
    compose_after(pA2, pB2, pA1, pB1);
    R pA3 = a2, pB3 = b2;
    compose_after(pA3, pB3, pA2, pB2);
    const R pA = row == 1 ? pA1 : (row == 2 ? pA2 : (row == 3 ? pA3 : R(1)));
    const R pB = row == 1 ? pB1 : (row == 2 ? pB2 : (row == 3 ? pB3 : R(0)));
    compose_after(Af, Bf, pA, pB);
  }
  {
    const R a3 = lane_value(Ab, 48), b3 = lane_value(Bb, 48);
    const R a2 = lane_value(Ab, 32), b2 = lane_value(Bb, 32);
    const R a1 = lane_value(Ab, 16), b1 = lane_value(Bb, 16);
    R qA2 = a3, qB2 = b3;
    R qA1 = a2, qB1 = b2;
    compose_after(qA1, qB1, qA2, qB2);
    R qA0 = a1, qB0 = b1;
    compose_after(qA0, qB0, qA1, qB1);
    const R qA = row == 0 ? qA0 : (row == 1 ? qA1 : (row == 2 ? qA2 : R(1)));
    const R qB = row == 0 ? qB0 : (row == 1 ? qB1 : (row == 2 ? qB2 : R(0)));
    compose_after(Ab, Bb, qA, qB);
  }
  const R eAf = dpp_fill<0x138>(R(1), Af), eBf = dpp_fill<0x138>(R(0), Bf);  // wave_shr:1
  const R eAb = dpp_fill<0x130>(R(1), Ab), eBb = dpp_fill<0x130>(R(0), Bb);  // wave_shl:1
  inF = rt_fma(eAf, gF, eBf);
  inB = rt_fma(eAb, gB, eBb);
}

// The calling wave's pairs (p = wave, wave + 8, ...): zero-inflow sweeps of
// the source s (LDS, sweep layout, rows of CM + 1) with the moments summed
// into acc.  A lane's run holds C <= CM cells; the row slots past them, and
// cells past nc, have sigma_t = 0 and s = 0, so their maps are the identity
// (a = 1 to rounding, b = 0) and the loops run over all CM slots without
// branches (their loads can be issued ahead).  Registers hold a_t and the
// moments only: b_t = (s_t a_t) / m is formed again from the source wherever
// it is needed (the same expression each time, so the scan and the
// application use identical maps), and one ascending pass composes both
// directions, the backward map as B_b = sum_t b_t prod_{k<t} a_k.
template <typename R, int CM>
__device__ __forceinline__ void wave_sweep(int npair, const R *ctL, const R *sL, const double *pmS,
                                           const double *pwS, R (&acc)[WCM]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = lane * (CM + 1);
#pragma unroll
  for (int t = 0; t < WCM; ++t) acc[t] = R(0);
  for (int p = wave; p < npair; p += WNW) {
    const R m = (R)pmS[p], w = (R)pwS[p];
    const R rm = R(1) / m;
    R a[CM];
    R pi = R(1), Bf = R(0), Bb = R(0);
    // chunks of eight cells: the scheduler may issue a chunk's LDS loads
    // ahead of its arithmetic but not the whole run's (register budget)
#pragma unroll
    for (int t = 0; t < CM; ++t) {
      if (t % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      a[t] = m * rt_rcp(ctL[base + t] + m);
      const R b = (sL[base + t] * a[t]) * rm;
      Bf = rt_fma(a[t], Bf, b);
      Bb = rt_fma(b, pi, Bb);
      pi *= a[t];
    }
    R inF, inB;
    wave_scan2<R>(pi, Bf, pi, Bb, R(0), R(0), inF, inB);
    R f = inF;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
      if (t % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      f = rt_fma(a[t], f, (sL[base + t] * a[t]) * rm);
      acc[t] = rt_fma(w, f, acc[t]);
    }
    f = inB;
#pragma unroll
    for (int t = CM - 1; t >= 0; --t) {
      if (t % 8 == 7) __builtin_amdgcn_sched_barrier(0);
      f = rt_fma(a[t], f, (sL[base + t] * a[t]) * rm);
      acc[t] = rt_fma(w, f, acc[t]);
    }
  }
}

// the sweep for the instance's row class CM (a multiple of four slots)
template <typename R>
__device__ __forceinline__ void wave_sweep_cls(int CM, int npair, const R *ctL, const R *sL, const double *pmS,
                                               const double *pwS, R (&acc)[WCM]) {
  static_assert(WCM == 32, "row classes 4..32");
  switch (CM) {
    case 4: wave_sweep<R, 4>(npair, ctL, sL, pmS, pwS, acc); break;
    case 8: wave_sweep<R, 8>(npair, ctL, sL, pmS, pwS, acc); break;
    case 12: wave_sweep<R, 12>(npair, ctL, sL, pmS, pwS, acc); break;
    case 16: wave_sweep<R, 16>(npair, ctL, sL, pmS, pwS, acc); break;
    case 20: wave_sweep<R, 20>(npair, ctL, sL, pmS, pwS, acc); break;
    case 24: wave_sweep<R, 24>(npair, ctL, sL, pmS, pwS, acc); break;
    case 28: wave_sweep<R, 28>(npair, ctL, sL, pmS, pwS, acc); break;
    default: wave_sweep<R, 32>(npair, ctL, sL, pmS, pwS, acc); break;
  }
}

// Sum of the eight waves' moments at the calling thread's cells (sweep-layout
// indices oidx[k], k < n), in a fixed order: waves 4..7 store theirs, waves
// 0..3 add their own to wave w + 4's, and the four rows are added in order.
// red: 4 rows of 64 * WPM elements.
template <typename R>
__device__ __forceinline__ void wave_reduce(const R (&acc)[WCM], int C, int P, R *red, const int (&oidx)[WOWN], int n,
                                            R (&out)[WOWN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = lane * P, row = 64 * WPM;
  __syncthreads();  // every wave is done reading the previous contents
  if (wave >= WNW / 2) {
    R *r = red + (wave - WNW / 2) * row + base;
#pragma unroll
    for (int t = 0; t < WCM; ++t)
      if (t < C) r[t] = acc[t];
  }
  __syncthreads();
  if (wave < WNW / 2) {
    R *r = red + wave * row + base;
#pragma unroll
    for (int t = 0; t < WCM; ++t)
      if (t < C) r[t] = acc[t] + r[t];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < WOWN; ++k) {
    R v = R(0);
    if (k < n) {
      const int i = oidx[k];
      v = ((red[i] + red[row + i]) + red[2 * row + i]) + red[3 * row + i];
    }
    out[k] = v;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// k_si_wave: initial guess + Alg. 1 (SI with DSA, or the hybrid ROM/DSA
// preconditioner of Sec. 3.2 phase 3) for every instance of the launch (one
// workgroup each, nc <= RT_WAVE_MAX_CELLS), then the step's error indicators
// and Alg. 2's decisions (rom_decide).  Writes rho^n, rho^{(0)}, rho^{(1/2)},
// the PC correction and the per-step status, as k_si_slab does.
// MH: the instantiation for instances whose correction is McClarren-Haut
// instead of DSA (rt_mh.h); each instantiation skips the other instances.
// BDF2 instances take the BDF2 operator (transport and DSA) from their second
// step on.
// ---------------------------------------------------------------------------
template <bool MH>
struct MhSlot {
  MhLds s;
};
template <>
struct MhSlot<false> {};

template <bool MH>
__global__ void __launch_bounds__(WNT) k_si_wave(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if ((I.precond == RT_PC_MH) != MH) return;
  __shared__ MhSlot<MH> mhslot;
  __shared__ double ct64[64 * WPM];
  __shared__ float ct32[64 * WPM];
  __shared__ double src[64 * WPM];   // the sweep source: FP64 sweeps
  __shared__ float src32[64 * WPM];  // FP32 increment sweeps
  __shared__ double redd[4 * 64 * WPM];
  __shared__ double pmS[WPAIRS], pwS[WPAIRS];
  __shared__ double slots[8 * RT_MAXWAVES];
  __shared__ double red[2 * RT_MAXWAVES];
  __shared__ double rred[RT_MAXWAVES * RT_RMAX];
  __shared__ double rvec[RT_RMAX + 4];
  float *redf = reinterpret_cast<float *>(redd);
  const int tid = threadIdx.x;
  const int nc = I.nc, npair = I.npair;
  // sweep layout: lane l's run is cells [l C, l C + C), row l of P = CM + 1
  // slots (odd), CM = C rounded up to a multiple of four
  const int C = (nc + 63) / 64;
  const int CM = (C + 3) & ~3, P = CM + 1;
  const int CW = (nc + WNT - 1) / WNT;
  const int c0 = tid * CW;
  const int n = max(0, min(CW, nc - c0));
  int oidx[WOWN];
#pragma unroll
  for (int k = 0; k < WOWN; ++k) {
    const int c = c0 + min(k, max(n - 1, 0));
    oidx[k] = min((c / C) * P + c % C, 64 * WPM - 1);  // used only for k < n
  }
  RtState *st = I.st;
  const int rom = (I.method == RT_ROM);
  const int flag_ig = st->flag_ig, flag_pc = st->flag_pc;
  const int lu_ig = st->lu_ok_ig, lu_pc = st->lu_ok_pc;
  const int rank_ig = st->rank_ig, rank_pc = st->rank_pc;
  // correction ROMs of iterations 2..nlev (Sec. 3.2, key feature 1); their
  // state is read where it is used (it does not change during the solve)
  const int nlev = I.nlev;
  int phase0 = !flag_ig ? 1 : (!flag_pc ? 2 : 3);
  for (int k = 0; k + 2 <= nlev; ++k) phase0 += (phase0 == k + 3 && st->flag_pl[k]) ? 1 : 0;
  const int mixed = (I.precision == RT_MIXED);
  const long long steps0 = st->steps, si0 = st->si_total, sw0 = st->sweeps_total, f32_0 = st->fp32_sweeps;
  const int nonconv0 = st->nonconv, fb0 = st->fallbacks;
  const int cur = (int)(steps0 & 1);
  const double *__restrict__ bt = I.bt2[cur];
  const bool alt = I.bdf2 && steps0 >= 1;  // BDF2 operator after the backward-Euler start
  const double *__restrict__ ctp = alt ? I.ct_b : I.ct;

  // per-cell constants of the sweeps in LDS (cells past nc: sigma_t = 0 and a
  // zero source, i.e. identity maps), the pairs' |mu|/h and weights
  for (int i = tid; i < 64 * P; i += WNT) {
    const int l = i / P, t = i - l * P, c = l * C + t;
    const double v = (t < C && c < nc) ? ldg(&ctp[c]) : 0.0;
    ct64[i] = v;
    ct32[i] = (float)v;
    src[i] = 0.0;
    src32[i] = 0.0f;
  }
  for (int p = tid; p < npair && p < WPAIRS; p += WNT) {
    pmS[p] = ldg(&I.pm[p]);
    pwS[p] = ldg(&I.pw[p]);
  }

  // initial guess: DMD when the IG ROM is available (eq. dmd-ig), else rho^{n-1}
  int ig_fb = 0;
  if (rom && flag_ig && lu_ig) {
    rom_apply<WOWN, 10, 10>(I.ig, rank_ig, I.ld, nc, WNT, bt, I.rho0, rred, rvec, redd);
  } else {
    ig_fb = rom && flag_ig;
    for (int c = c0; c < c0 + n; ++c) stg(&I.rho0[c], ldg(&I.rho[c]));
  }
  double ss[WOWN], rp[WOWN], y[WOWN], b0[WOWN];
#pragma unroll
  for (int t = 0; t < WOWN; ++t) {
    const bool in = t < n;
    ss[t] = in ? ldg(&I.ss[c0 + t]) : 0.0;
    rp[t] = in ? ldg(&I.rho0[c0 + t]) : 0.0;
    b0[t] = in ? ldg(&bt[c0 + t]) : 0.0;
    y[t] = 0.0;
  }
  int parity = 0;
  int nsweep = 0, n32 = 0, conv = 0, used_pc = 0, pc_fb = 0, exact = 0, first_corr = 1;
  int ncorr = 0, used_mask = 0, lv_fb = 0;  // corrections so far; levels applied (bit l - 1)
  int need64 = 1;
  double resid = 0.0;
  // McClarren-Haut: y_{l-1} and rho^{(l-2)}; the model lives within the step
  double yp[WOWN], rp2[WOWN];
  if constexpr (MH) {
#pragma unroll
    for (int t = 0; t < WOWN; ++t) yp[t] = rp2[t] = 0.0;
    if (tid == 0) mhslot.s.m = 0;
    __syncthreads();
  }
  for (;;) {
    if (need64) {
      // rho^{(l-1/2)} = T Sigma_s rho^{(l-1)} + b~ (eq. SI_rho) in FP64
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) src[oidx[t]] = ss[t] * rp[t];
      __syncthreads();
      double acc[WCM], mom[WOWN];
      wave_sweep_cls<double>(CM, npair, ct64, src, pmS, pwS, acc);
      wave_reduce<double>(acc, C, P, redd, oidx, n, mom);
#pragma unroll
      for (int t = 0; t < WOWN; ++t) y[t] = mom[t] + b0[t];
      if (nsweep == 0) {
#pragma unroll
        for (int t = 0; t < WOWN; ++t)
          if (t < n) stg(&I.rhalf[c0 + t], y[t]);
      }
      nsweep++;
      exact = 1;
      need64 = 0;
    }
    double dl = 0.0, yl = 0.0;
#pragma unroll
    for (int t = 0; t < WOWN; ++t)
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
    if constexpr (MH) {
      // the pair of this iteration: (rho^{(l-1)} - rho^{(l-2)}, y_l - y_{l-1})
      if (nsweep >= 2) {
        double x[WOWN], z[WOWN];
#pragma unroll
        for (int t = 0; t < WOWN; ++t) {
          x[t] = rp[t] - rp2[t];
          z[t] = y[t] - yp[t];
        }
        mh_push<WOWN>(I, c0, n, x, z, mhslot.s);
      }
#pragma unroll
      for (int t = 0; t < WOWN; ++t) {
        yp[t] = y[t];
        rp2[t] = rp[t];
      }
    }
    // synthetic acceleration; correction l = ncorr + 1 of the step.  Level l
    // of the correction ROMs keeps y_l = rho^{(l-1/2)} and rho^{(l-1)} for its
    // pair, and applies when complete and level l - 1 applied before it.
    const int lc = ncorr + 1;
    const bool lev_here = rom && lc >= 2 && lc <= nlev;
    bool lev_apply = false;
    if (lev_here) {
      const int k = lc - 2;
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) {
          stg(&I.ylev[k][c0 + t], y[t]);
          stg(&I.rlev[k][c0 + t], rp[t]);
        }
      const bool due = st->flag_pl[k] && ((used_mask >> (lc - 2)) & 1);
      const int luok = st->lu_ok_pl[k];
      if (due && !luok) lv_fb++;
      lev_apply = due && luok;
    }
    double d[WOWN];
    if (lev_apply) {
      // ROM-enhanced correction of iteration lc (eq. dmd-sa at iteration lc)
      const int k = lc - 2;
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) stg(&I.wlev[k][c0 + t], y[t] - rp[t]);
      __syncthreads();
      rom_apply<WOWN, 10, 10>(I.pl[k], st->rank_pl[k], I.ld, nc, WNT, I.wlev[k], I.dlev[k], rred, rvec, redd);
#pragma unroll
      for (int t = 0; t < WOWN; ++t) d[t] = (t < n) ? ldg(&I.dlev[k][c0 + t]) : 0.0;
      used_mask |= 1 << (lc - 1);
    } else if (rom && first_corr && flag_pc && lu_pc) {
      // ROM-enhanced correction of the first iteration (eq. dmd-sa)
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) stg(&I.work[c0 + t], y[t] - ldg(&I.rho0[c0 + t]));
      __syncthreads();
      rom_apply<WOWN, 10, 10>(I.pc, rank_pc, I.ld, nc, WNT, I.work, I.dpc, rred, rvec, redd);
#pragma unroll
      for (int t = 0; t < WOWN; ++t) d[t] = (t < n) ? ldg(&I.dpc[c0 + t]) : 0.0;
      used_pc = 1;
      used_mask |= 1;
    } else if (I.method == RT_SI_PLAIN) {
#pragma unroll
      for (int t = 0; t < WOWN; ++t) d[t] = 0.0;
    } else if constexpr (MH) {
      // McClarren-Haut correction from the step's pairs (Sec. 3.3)
      if (rom && first_corr && flag_pc) pc_fb = 1;
      double r[WOWN];
#pragma unroll
      for (int t = 0; t < WOWN; ++t) r[t] = y[t] - rp[t];
      mh_correct<WOWN>(I, c0, n, r, d, mhslot.s);
    } else {
      if (rom && first_corr && flag_pc) pc_fb = 1;
      double rhs[WOWN];
#pragma unroll
      for (int t = 0; t < WOWN; ++t) rhs[t] = ss[t] * (y[t] - rp[t]);
      dsa_solve_slab<WOWN>(I, c0, n, rhs, d, slots, parity, alt);
    }
    first_corr = 0;
    ncorr++;
    if (mixed) {
      // y <- y + T32 Sigma_s (rho^{(l)} - rho^{(l-1)}): increment swept in FP32
#pragma unroll
      for (int t = 0; t < WOWN; ++t) {
        const double rn = y[t] + d[t];
        if (t < n) src32[oidx[t]] = (float)(ss[t] * (rn - rp[t]));
        rp[t] = rn;
      }
      __syncthreads();
      float acc[WCM], mom[WOWN];
      wave_sweep_cls<float>(CM, npair, ct32, src32, pmS, pwS, acc);
      wave_reduce<float>(acc, C, P, redf, oidx, n, mom);
#pragma unroll
      for (int t = 0; t < WOWN; ++t) y[t] += (double)mom[t];
      exact = 0;
      n32++;
      nsweep++;
    } else {
#pragma unroll
      for (int t = 0; t < WOWN; ++t) rp[t] = y[t] + d[t];
      need64 = 1;
    }
  }
  // rho^n = rho^{(l-1/2)} (Alg. 1 returns the un-corrected iterate)
#pragma unroll
  for (int t = 0; t < WOWN; ++t)
    if (t < n) stg(&I.rho[c0 + t], y[t]);
  if (tid == 0) {
    st->iters = nsweep;
    st->conv = conv;
    st->used_pc = used_pc;
    st->ig_fb = ig_fb;
    st->pc_fb = pc_fb;
    st->residual = resid;
    st->phase = phase0;
    st->cur = cur;
    st->fp32_sweeps = f32_0 + n32;
    st->used_mask = used_mask;
  }
  __syncthreads();
  // end of step: error indicators from the final iterate and Alg. 2's
  // decisions, so the ROM work that follows needs no launch of its own
  if (rom && flag_ig) {
    if (nlev > 1) {
      // also ||dlev - (rho^n - y_l)||^2 of the levels that applied
      double part[3 + RT_XLEV];
#pragma unroll
      for (int k = 0; k < 3 + RT_XLEV; ++k) part[k] = 0.0;
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) {
          const double r = y[t];
          part[0] = rt_fma(r, r, part[0]);
          const double e1 = ldg(&I.rho0[c0 + t]) - r;
          part[1] = rt_fma(e1, e1, part[1]);
          const double e2 = ldg(&I.dpc[c0 + t]) - (r - ldg(&I.rhalf[c0 + t]));
          part[2] = rt_fma(e2, e2, part[2]);
#pragma unroll
          for (int k = 0; k < RT_XLEV; ++k)
            if ((used_mask >> (k + 1)) & 1) {
              const double e = ldg(&I.dlev[k][c0 + t]) - (r - ldg(&I.ylev[k][c0 + t]));
              part[3 + k] = rt_fma(e, e, part[3 + k]);
            }
        }
      wg_sum_fast<3 + RT_XLEV>(part, rred, rvec);
    } else {
      double part[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < WOWN; ++t)
        if (t < n) {
          const double r = y[t];
          part[0] = rt_fma(r, r, part[0]);
          const double e1 = ldg(&I.rho0[c0 + t]) - r;
          part[1] = rt_fma(e1, e1, part[1]);
          const double e2 = ldg(&I.dpc[c0 + t]) - (r - ldg(&I.rhalf[c0 + t]));
          part[2] = rt_fma(e2, e2, part[2]);
        }
      wg_sum_fast<3>(part, rred, rvec);
    }
  }
  StepIn S{nsweep, conv, used_pc, ig_fb, pc_fb, phase0, cur, flag_ig, flag_pc,
           rank_ig, rank_pc, nonconv0, fb0, resid, steps0, si0, sw0};
  S.used_mask = used_mask;
  S.lv_fb = lv_fb;
  rom_decide(I, rvec, I.post_nb, S);
}

extern "C" hipError_t rt_launch_slab_si_wave(const Inst *dinsts, int ninst, int kinds, hipStream_t stream) {
  if (kinds & 1) hipLaunchKernelGGL(k_si_wave<false>, dim3(ninst), dim3(WNT), 0, stream, dinsts);
  if (kinds & 2) hipLaunchKernelGGL(k_si_wave<true>, dim3(ninst), dim3(WNT), 0, stream, dinsts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_fpass_wave: the f-pass of instances of up to 2048 cells, one workgroup of
// eight waves per instance, wave w taking the ordinate pairs w, w + 8, ...:
// f^n_j from rho^n (eq. sweep_to_obtain_f: source sigma_s rho^n + f^{n-1}_j /
// dt + G, inflow g) and the right-hand side of the next step, b~^n = sum_j
// w_j sweep_j(f^n_j / dt + G; g) (Sec. 2.3), in one traversal.
//
// The cells go in blocks of 256: in block b lane l takes the four cells
// 256 b + 4 l + k, so a wave's four loads of f cover 2 KB of one ordinate's
// row.  Each block is an affine scan across the wave (its per-lane maps
// composed serially) fed by the value leaving the previous block; the
// positive ordinate runs its blocks upwards, the negative one downwards, and
// a wave scans one block of each at once.  Both sweeps of an ordinate advance
// block by block, the second consuming the first one's f^n of the block.  The
// moments accumulate in registers; at the end the waves' moments are added
// through LDS in a fixed order and b~^n is written.  f is read and written
// once (16 B per cell-angle); there is no per-pair moment array.
// rhs_only: skip the first sweep and rebuild b~ from the stored f (creation,
// or a new inflow).
// ---------------------------------------------------------------------------
namespace {
constexpr int FK = 4;                         // cells per lane and block
constexpr int FB = 64 * FK;                   // cells per block
constexpr int FNB = RT_WAVE_MAX_CELLS / FB;   // blocks at most
constexpr int FROW = RT_WAVE_MAX_CELLS + RT_WAVE_MAX_CELLS / FK;  // padded LDS row
__device__ __forceinline__ int fidx(int c) { return c + (c >> 2); }  // one pad per four cells
}  // namespace

__global__ void __launch_bounds__(WNT) k_fpass_wave(const Inst *__restrict__ insts, int rhs_only) {
  const Inst &I = insts[blockIdx.x];
  if (I.bdf2) return;  // k_fpass_wave_bdf2
  __shared__ double big[4 * FROW];  // ct, srcc, G during the sweeps; then the moment rows
  double *ctS = big, *srcS = big + FROW, *gS = big + 2 * FROW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = I.nc, npair = I.npair, nv = I.nv;
  const int NB = (nc + FB - 1) / FB;
  const double idt = I.inv_dt;
  // per-cell inputs; cells past nc (up to the last block) are identity maps
  for (int c = tid; c < NB * FB; c += WNT) {
    const bool in = c < nc;
    const double g = in ? ldg(&I.G[c]) : 0.0;
    ctS[fidx(c)] = in ? ldg(&I.ct[c]) : 0.0;
    gS[fidx(c)] = g;
    srcS[fidx(c)] = (in && !rhs_only) ? rt_fma(ldg(&I.ss[c]), ldg(&I.rho[c]), g) : 0.0;
  }
  __syncthreads();
  double acc[FNB][FK];
#pragma unroll
  for (int b = 0; b < FNB; ++b)
#pragma unroll
    for (int k = 0; k < FK; ++k) acc[b][k] = 0.0;
  const double g0 = I.g[0], g1 = I.g[1];
  for (int p = wave; p < npair; p += WNW) {
    const double m = ldg(&I.pm[p]), w = ldg(&I.pw[p]);
    double *fneg = I.f + (size_t)p * nc;               // mu < 0: swept downwards
    double *fpos = I.f + (size_t)(nv - 1 - p) * nc;    // mu > 0: swept upwards
    double cp1 = g0, cp2 = g0, cn1 = g1, cn2 = g1;     // values entering the next block
#pragma unroll
    for (int s = 0; s < FNB; ++s) {
      if (s < NB) {
        const int bp = s, bn = NB - 1 - s;
        const int cpb = bp * FB + lane * FK, cnb = bn * FB + lane * FK;
        double fp[FK], fn[FK], ip[FK], in_[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          fp[k] = cpb + k < nc ? ldg(&fpos[cpb + k]) : 0.0;
          fn[k] = cnb + k < nc ? ldg(&fneg[cnb + k]) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          ip[k] = rt_rcp(ctS[fidx(cpb + k)] + m);
          in_[k] = rt_rcp(ctS[fidx(cnb + k)] + m);
        }
        // a_k = m / (ct_k + m) is formed from the stored reciprocal wherever
        // it is needed (the same expression each time)
        if (!rhs_only) {
          // first sweep: f^n with source sigma_s rho^n + f^{n-1} / dt + G
          double Bf = 0.0, pf = 1.0, Bb = 0.0, pb = 1.0;
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            const double bk = rt_fma(fp[k], idt, srcS[fidx(cpb + k)]) * ip[k];
            Bf = rt_fma(m * ip[k], Bf, bk);
            pf *= m * ip[k];
            const double bkn = rt_fma(fn[k], idt, srcS[fidx(cnb + k)]) * in_[k];
            Bb = rt_fma(bkn, pb, Bb);
            pb *= m * in_[k];
          }
          double inF, inB;
          wave_scan2<double>(pf, Bf, pb, Bb, cp1, cn1, inF, inB);
          double f = inF;
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            f = rt_fma(m * ip[k], f, rt_fma(fp[k], idt, srcS[fidx(cpb + k)]) * ip[k]);
            fp[k] = f;
            if (cpb + k < nc) stg(&fpos[cpb + k], f);
          }
          cp1 = lane_value(f, 63);
          f = inB;
#pragma unroll
          for (int k = FK - 1; k >= 0; --k) {
            f = rt_fma(m * in_[k], f, rt_fma(fn[k], idt, srcS[fidx(cnb + k)]) * in_[k]);
            fn[k] = f;
            if (cnb + k < nc) stg(&fneg[cnb + k], f);
          }
          cn1 = lane_value(f, 0);
          // cells past nc carried the inflow through; as sources of the
          // second sweep they are zero (the identity map again)
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            if (cpb + k >= nc) fp[k] = 0.0;
            if (cnb + k >= nc) fn[k] = 0.0;
          }
        }
        // second sweep: source f^n / dt + G, the moment of b~^n
        double Bf = 0.0, pf = 1.0, Bb = 0.0, pb = 1.0;
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          const double bk = rt_fma(fp[k], idt, gS[fidx(cpb + k)]) * ip[k];
          Bf = rt_fma(m * ip[k], Bf, bk);
          pf *= m * ip[k];
          const double bkn = rt_fma(fn[k], idt, gS[fidx(cnb + k)]) * in_[k];
          Bb = rt_fma(bkn, pb, Bb);
          pb *= m * in_[k];
        }
        double inF, inB;
        wave_scan2<double>(pf, Bf, pb, Bb, cp2, cn2, inF, inB);
        double f = inF;
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          f = rt_fma(m * ip[k], f, rt_fma(fp[k], idt, gS[fidx(cpb + k)]) * ip[k]);
          fp[k] = f;
        }
        cp2 = lane_value(f, 63);
        f = inB;
#pragma unroll
        for (int k = FK - 1; k >= 0; --k) {
          f = rt_fma(m * in_[k], f, rt_fma(fn[k], idt, gS[fidx(cnb + k)]) * in_[k]);
          fn[k] = f;
        }
        cn2 = lane_value(f, 0);
#pragma unroll
        for (int b = 0; b < FNB; ++b) {
          if (b == bp) {
#pragma unroll
            for (int k = 0; k < FK; ++k) acc[b][k] = rt_fma(w, fp[k], acc[b][k]);
          }
          if (b == bn) {
#pragma unroll
            for (int k = 0; k < FK; ++k) acc[b][k] = rt_fma(w, fn[k], acc[b][k]);
          }
        }
      }
    }
  }
  // the waves' moments in a fixed order: waves 4..7 store, waves 0..3 add
  // theirs, then the four rows are added in order
  __syncthreads();
  if (wave >= WNW / 2) {
    double *r = big + (wave - WNW / 2) * FROW;
#pragma unroll
    for (int b = 0; b < FNB; ++b)
      if (b < NB)
#pragma unroll
        for (int k = 0; k < FK; ++k) r[fidx(b * FB + lane * FK + k)] = acc[b][k];
  }
  __syncthreads();
  if (wave < WNW / 2) {
    double *r = big + wave * FROW;
#pragma unroll
    for (int b = 0; b < FNB; ++b)
      if (b < NB)
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          const int i = fidx(b * FB + lane * FK + k);
          r[i] = acc[b][k] + r[i];
        }
  }
  __syncthreads();
  double *bt_out = rhs_only ? I.bt2[I.st->steps & 1] : I.bt2[I.st->cur ^ 1];
  for (int c = tid; c < nc; c += WNT) {
    const int i = fidx(c);
    stg(&bt_out[c], ((big[i] + big[FROW + i]) + big[2 * FROW + i]) + big[3 * FROW + i]);
  }
}

// ---------------------------------------------------------------------------
// k_fpass_wave_bdf2: the f-pass of BDF2 instances, in k_fpass_wave's layout
// and order.  For the step n just solved (n = the state's step count): f^n
// from rho^n with the source sigma_s rho^n + (4 f^{n-1} - f^{n-2}) / (2 dt)
// + G and the BDF2 operator (at n = 1 the backward-Euler start: f^{n-1} / dt
// and the backward-Euler operator), written over f^{n-2}; then the
// right-hand side of step n + 1, b~^n = sum_j w_j sweep_j((4 f^n - f^{n-1})
// / (2 dt) + G; g), with the BDF2 operator.  rhs_only: b~ of step S + 1 from
// the stored f^S (and f^{S-1}), S the state's step count.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WNT) k_fpass_wave_bdf2(const Inst *__restrict__ insts, int rhs_only) {
  const Inst &I = insts[blockIdx.x];
  if (!I.bdf2) return;
  __shared__ double big[4 * FROW];  // ct (solve), ct (rhs), srcc, G; then the moment rows
  double *ctS = big, *srcS = big + FROW, *gS = big + 2 * FROW, *ct2S = big + 3 * FROW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = I.nc, npair = I.npair, nv = I.nv;
  const int NB = (nc + FB - 1) / FB;
  const double idt = I.inv_dt, hidt = 0.5 * I.inv_dt;
  const long long S = I.st->steps;
  const bool now_b = !rhs_only && S >= 2;        // f^n from the BDF2 formula
  const bool next_b = rhs_only ? S >= 1 : true;  // b~ of a BDF2 step
  const double *__restrict__ ct_now = now_b ? I.ct_b : I.ct;
  const double *__restrict__ ct_next = next_b ? I.ct_b : I.ct;
  // rhs_only: fA = f^{S-1}, fB = f^S.  Otherwise fA = f^{n-1}, fB = f^{n-2},
  // overwritten by f^n.
  double *fA = I.fb[(S + 1) & 1];
  double *fB = I.fb[S & 1];
  for (int c = tid; c < NB * FB; c += WNT) {
    const bool in = c < nc;
    const double g = in ? ldg(&I.G[c]) : 0.0;
    ctS[fidx(c)] = in ? ldg(&ct_now[c]) : 0.0;
    ct2S[fidx(c)] = in ? ldg(&ct_next[c]) : 0.0;
    gS[fidx(c)] = g;
    srcS[fidx(c)] = (in && !rhs_only) ? rt_fma(ldg(&I.ss[c]), ldg(&I.rho[c]), g) : 0.0;
  }
  __syncthreads();
  double acc[FNB][FK];
#pragma unroll
  for (int b = 0; b < FNB; ++b)
#pragma unroll
    for (int k = 0; k < FK; ++k) acc[b][k] = 0.0;
  const double g0 = I.g[0], g1 = I.g[1];
  for (int p = wave; p < npair; p += WNW) {
    const double m = ldg(&I.pm[p]), w = ldg(&I.pw[p]);
    const size_t on = (size_t)p * nc, op = (size_t)(nv - 1 - p) * nc;  // mu < 0, mu > 0
    double cp1 = g0, cp2 = g0, cn1 = g1, cn2 = g1;  // values entering the next block
#pragma unroll
    for (int s = 0; s < FNB; ++s) {
      if (s < NB) {
        const int bp = s, bn = NB - 1 - s;
        const int cpb = bp * FB + lane * FK, cnb = bn * FB + lane * FK;
        // fp, fn: f of the newest level (f^n once solved); ap, an: the level
        // before it, for the BDF2 source of the right-hand side
        double fp[FK], fn[FK], ap[FK], an[FK], ip[FK], in_[FK], jp[FK], jn[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          const bool okp = cpb + k < nc, okn = cnb + k < nc;
          if (rhs_only) {
            fp[k] = okp ? ldg(&fB[op + cpb + k]) : 0.0;
            fn[k] = okn ? ldg(&fB[on + cnb + k]) : 0.0;
            ap[k] = (okp && next_b) ? ldg(&fA[op + cpb + k]) : 0.0;
            an[k] = (okn && next_b) ? ldg(&fA[on + cnb + k]) : 0.0;
          } else {
            ap[k] = okp ? ldg(&fA[op + cpb + k]) : 0.0;
            an[k] = okn ? ldg(&fA[on + cnb + k]) : 0.0;
            fp[k] = (okp && now_b) ? ldg(&fB[op + cpb + k]) : 0.0;  // f^{n-2}
            fn[k] = (okn && now_b) ? ldg(&fB[on + cnb + k]) : 0.0;
          }
        }
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          ip[k] = rt_rcp(ctS[fidx(cpb + k)] + m);
          in_[k] = rt_rcp(ctS[fidx(cnb + k)] + m);
          jp[k] = rt_rcp(ct2S[fidx(cpb + k)] + m);
          jn[k] = rt_rcp(ct2S[fidx(cnb + k)] + m);
        }
        if (!rhs_only) {
          // f^n: source sigma_s rho^n + history + G, history from f^{n-1}
          // (ap, an) and f^{n-2} (fp, fn)
          double hp[FK], hn[FK];
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            hp[k] = now_b ? rt_fma(4.0, ap[k], -fp[k]) * hidt : ap[k] * idt;
            hn[k] = now_b ? rt_fma(4.0, an[k], -fn[k]) * hidt : an[k] * idt;
          }
          double Bf = 0.0, pf = 1.0, Bb = 0.0, pb = 1.0;
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            const double bk = (hp[k] + srcS[fidx(cpb + k)]) * ip[k];
            Bf = rt_fma(m * ip[k], Bf, bk);
            pf *= m * ip[k];
            const double bkn = (hn[k] + srcS[fidx(cnb + k)]) * in_[k];
            Bb = rt_fma(bkn, pb, Bb);
            pb *= m * in_[k];
          }
          double inF, inB;
          wave_scan2<double>(pf, Bf, pb, Bb, cp1, cn1, inF, inB);
          double f = inF;
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            f = rt_fma(m * ip[k], f, (hp[k] + srcS[fidx(cpb + k)]) * ip[k]);
            fp[k] = f;
            if (cpb + k < nc) stg(&fB[op + cpb + k], f);
          }
          cp1 = lane_value(f, 63);
          f = inB;
#pragma unroll
          for (int k = FK - 1; k >= 0; --k) {
            f = rt_fma(m * in_[k], f, (hn[k] + srcS[fidx(cnb + k)]) * in_[k]);
            fn[k] = f;
            if (cnb + k < nc) stg(&fB[on + cnb + k], f);
          }
          cn1 = lane_value(f, 0);
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            if (cpb + k >= nc) fp[k] = 0.0;
            if (cnb + k >= nc) fn[k] = 0.0;
          }
        }
        // right-hand side of the next step: source (4 f^n - f^{n-1}) / (2 dt)
        // + G (a backward-Euler step: f / dt + G), its operator
        double sp[FK], sn[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          sp[k] = (next_b ? rt_fma(4.0, fp[k], -ap[k]) * hidt : fp[k] * idt) + gS[fidx(cpb + k)];
          sn[k] = (next_b ? rt_fma(4.0, fn[k], -an[k]) * hidt : fn[k] * idt) + gS[fidx(cnb + k)];
        }
        double Bf = 0.0, pf = 1.0, Bb = 0.0, pb = 1.0;
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          Bf = rt_fma(m * jp[k], Bf, sp[k] * jp[k]);
          pf *= m * jp[k];
          Bb = rt_fma(sn[k] * jn[k], pb, Bb);
          pb *= m * jn[k];
        }
        double inF, inB;
        wave_scan2<double>(pf, Bf, pb, Bb, cp2, cn2, inF, inB);
        double f = inF;
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          f = rt_fma(m * jp[k], f, sp[k] * jp[k]);
          fp[k] = f;
        }
        cp2 = lane_value(f, 63);
        f = inB;
#pragma unroll
        for (int k = FK - 1; k >= 0; --k) {
          f = rt_fma(m * jn[k], f, sn[k] * jn[k]);
          fn[k] = f;
        }
        cn2 = lane_value(f, 0);
#pragma unroll
        for (int b = 0; b < FNB; ++b) {
          if (b == bp) {
#pragma unroll
            for (int k = 0; k < FK; ++k) acc[b][k] = rt_fma(w, fp[k], acc[b][k]);
          }
          if (b == bn) {
#pragma unroll
            for (int k = 0; k < FK; ++k) acc[b][k] = rt_fma(w, fn[k], acc[b][k]);
          }
        }
      }
    }
  }
  __syncthreads();
  if (wave >= WNW / 2) {
    double *r = big + (wave - WNW / 2) * FROW;
#pragma unroll
    for (int b = 0; b < FNB; ++b)
      if (b < NB)
#pragma unroll
        for (int k = 0; k < FK; ++k) r[fidx(b * FB + lane * FK + k)] = acc[b][k];
  }
  __syncthreads();
  if (wave < WNW / 2) {
    double *r = big + wave * FROW;
#pragma unroll
    for (int b = 0; b < FNB; ++b)
      if (b < NB)
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          const int i = fidx(b * FB + lane * FK + k);
          r[i] = acc[b][k] + r[i];
        }
  }
  __syncthreads();
  double *bt_out = rhs_only ? I.bt2[S & 1] : I.bt2[I.st->cur ^ 1];
  for (int c = tid; c < nc; c += WNT) {
    const int i = fidx(c);
    stg(&bt_out[c], ((big[i] + big[FROW + i]) + big[2 * FROW + i]) + big[3 * FROW + i]);
  }
}

extern "C" hipError_t rt_launch_slab_fpass_wave(const Inst *dinsts, int ninst, int rhs_only, int kinds,
                                                hipStream_t stream) {
  if (kinds & 1) hipLaunchKernelGGL(k_fpass_wave, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  if (kinds & 2) hipLaunchKernelGGL(k_fpass_wave_bdf2, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  return hipGetLastError();
}
