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

// Piecewise-linear DG (eq. DG with K = 1) on the slab: on a cell f = u0 +
// sqrt(3) u1 xi, xi in [-1, 1] across the cell, tested with 1 and sqrt(3) xi
// and upwinded at the faces.  With c = sigma_t + 1/dt, m = |mu| / h, the
// cell's source s0 + sqrt(3) s1 xi and f_in the value entering through the
// upwind face, the cell's 2x2 system for mu > 0 is
//   (c + m) u0 + sqrt(3) m u1 = s0 + m f_in
//   -sqrt(3) m u0 + (c + 3 m) u1 = s1 - sqrt(3) m f_in
// with determinant det = c (c + 4 m) + 6 m^2.  Solved:
//   u0 = [(c + 3 m) s0 - sqrt(3) m s1 + m (c + 6 m) f_in] / det
//   u1 = [(c + m) s1 + sqrt(3) m s0 - sqrt(3) m c f_in] / det
// and the value leaving through the downwind face, u0 + sqrt(3) u1, is
// affine in f_in:  f_out = a f_in + b,  a = 2 m (3 m - c) / det,  b = [(c +
// 6 m) s0 + sqrt(3) c s1] / det  (|a| < 1).  mu < 0 is the mirror image (xi
// -> -xi: s1 and u1 change sign), so both directions share a and det and
// differ in b.  The sweep is therefore the same affine recurrence as for
// finite volumes, on face values, and each cell's two unknowns follow from
// the value entering it.
constexpr double kR3 = 1.7320508075688772;  // sqrt(3)

template <typename R>
struct DgCell {
  R q, a, bf, bb;  // 1/det, face factor, forward and backward offsets
};
template <typename R>
__device__ __forceinline__ DgCell<R> dg_cell(R c, R m, R s0, R s1) {
  DgCell<R> z;
  z.q = rt_rcp(rt_fma(c, c + R(4) * m, R(6) * m * m));
  z.a = (R(2) * m * (R(3) * m - c)) * z.q;
  // the same expressions as where the sweep applies the maps
  const R v = (R(kR3) * c) * s1;
  z.bf = rt_fma(c + R(6) * m, s0, v) * z.q;
  z.bb = rt_fma(c + R(6) * m, s0, -v) * z.q;
  return z;
}
// the cell's unknowns from the entering face value (fwd: mu > 0)
template <typename R, bool FWD>
__device__ __forceinline__ void dg_unknowns(R c, R m, R s0, R s1, R q, R fin, R &u0, R &u1) {
  const R r3m = R(kR3) * m;
  if (FWD) {
    u0 = rt_fma(m * (c + R(6) * m), fin, rt_fma(c + R(3) * m, s0, -r3m * s1)) * q;
    u1 = rt_fma(-r3m * c, fin, rt_fma(c + m, s1, r3m * s0)) * q;
  } else {
    u0 = rt_fma(m * (c + R(6) * m), fin, rt_fma(c + R(3) * m, s0, r3m * s1)) * q;
    u1 = rt_fma(r3m * c, fin, rt_fma(c + m, s1, -r3m * s0)) * q;
  }
}

// wave_sweep for DG slabs: a lane's run holds C <= CM cells, two unknowns
// each, at slots 2 t, 2 t + 1 of its row (rows of 2 CM + 1); acc[2 t + k]
// takes the moments.  Padding slots (c = 0, s = 0) are identity maps.
template <typename R, int CM>
__device__ __forceinline__ void wave_sweep_dg(int npair, const R *ctL, const R *sL, const double *pmS,
                                              const double *pwS, R (&acc)[WCM]) {
  static_assert(2 * CM <= WCM, "two unknowns per cell");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = lane * (2 * CM + 1);
#pragma unroll
  for (int t = 0; t < WCM; ++t) acc[t] = R(0);
  for (int p = wave; p < npair; p += WNW) {
    const R m = (R)pmS[p], w = (R)pwS[p];
    R a[CM], q[CM];
    R pi = R(1), Bf = R(0), Bb = R(0);
#pragma unroll
    for (int t = 0; t < CM; ++t) {
      if (t % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      const DgCell<R> z = dg_cell<R>(ctL[base + 2 * t], m, sL[base + 2 * t], sL[base + 2 * t + 1]);
      a[t] = z.a;
      q[t] = z.q;
      Bf = rt_fma(z.a, Bf, z.bf);
      Bb = rt_fma(z.bb, pi, Bb);
      pi *= z.a;
    }
    R inF, inB;
    wave_scan2<R>(pi, Bf, pi, Bb, R(0), R(0), inF, inB);
    R f = inF;
#pragma unroll
    for (int t = 0; t < CM; ++t) {
      if (t % 8 == 0) __builtin_amdgcn_sched_barrier(0);
      const R c = ctL[base + 2 * t], s0 = sL[base + 2 * t], s1 = sL[base + 2 * t + 1];
      R u0, u1;
      dg_unknowns<R, true>(c, m, s0, s1, q[t], f, u0, u1);
      acc[2 * t] = rt_fma(w, u0, acc[2 * t]);
      acc[2 * t + 1] = rt_fma(w, u1, acc[2 * t + 1]);
      f = rt_fma(a[t], f, (rt_fma(c + R(6) * m, s0, (R(kR3) * c) * s1)) * q[t]);
    }
    f = inB;
#pragma unroll
    for (int t = CM - 1; t >= 0; --t) {
      if (t % 8 == 7) __builtin_amdgcn_sched_barrier(0);
      const R c = ctL[base + 2 * t], s0 = sL[base + 2 * t], s1 = sL[base + 2 * t + 1];
      R u0, u1;
      dg_unknowns<R, false>(c, m, s0, s1, q[t], f, u0, u1);
      acc[2 * t] = rt_fma(w, u0, acc[2 * t]);
      acc[2 * t + 1] = rt_fma(w, u1, acc[2 * t + 1]);
      f = rt_fma(a[t], f, (rt_fma(c + R(6) * m, s0, -(R(kR3) * c) * s1)) * q[t]);
    }
  }
}

template <typename R>
__device__ __forceinline__ void wave_sweep_dg_cls(int CM, int npair, const R *ctL, const R *sL, const double *pmS,
                                                  const double *pwS, R (&acc)[WCM]) {
  switch (CM) {
    case 4: wave_sweep_dg<R, 4>(npair, ctL, sL, pmS, pwS, acc); break;
    case 8: wave_sweep_dg<R, 8>(npair, ctL, sL, pmS, pwS, acc); break;
    case 12: wave_sweep_dg<R, 12>(npair, ctL, sL, pmS, pwS, acc); break;
    default: wave_sweep_dg<R, 16>(npair, ctL, sL, pmS, pwS, acc); break;
  }
}

// DSA of DG slabs: C d = rhs with C block tridiagonal (2x2 blocks L_i, D_i,
// L_{i+1}^T), by block elimination written as two recurrences of 2x2 affine
// maps over the cells: z_i = F_i z_{i-1} + rhs_i forward, then d_i = B_i
// d_{i+1} + S_i^{-1} z_i backward (F, S^{-1}, B from k_setup_dsa_dg).  Each
// thread composes the maps of its cells, a workgroup scan of the composites
// gives every thread the value entering its run, and the thread applies its
// maps.
struct Blk2 {
  double a00, a01, a10, a11, b0, b1;  // x -> A x + b
};
__device__ __forceinline__ Blk2 blk_id() { return {1.0, 0.0, 0.0, 1.0, 0.0, 0.0}; }
// X o Y: x -> X(Y(x))
__device__ __forceinline__ Blk2 blk_after(const Blk2 &X, const Blk2 &Y) {
  Blk2 r;
  r.a00 = rt_fma(X.a00, Y.a00, X.a01 * Y.a10);
  r.a01 = rt_fma(X.a00, Y.a01, X.a01 * Y.a11);
  r.a10 = rt_fma(X.a10, Y.a00, X.a11 * Y.a10);
  r.a11 = rt_fma(X.a10, Y.a01, X.a11 * Y.a11);
  r.b0 = rt_fma(X.a00, Y.b0, rt_fma(X.a01, Y.b1, X.b0));
  r.b1 = rt_fma(X.a10, Y.b0, rt_fma(X.a11, Y.b1, X.b1));
  return r;
}
__device__ __forceinline__ void blk_apply(const Blk2 &X, double &v0, double &v1) {
  const double t0 = rt_fma(X.a00, v0, rt_fma(X.a01, v1, X.b0));
  const double t1 = rt_fma(X.a10, v0, rt_fma(X.a11, v1, X.b1));
  v0 = t0;
  v1 = t1;
}
template <int CTRL>
__device__ __forceinline__ Blk2 blk_dpp(const Blk2 &v) {  // lanes without a source get the identity
  return {dpp_fill<CTRL>(1.0, v.a00), dpp_fill<CTRL>(0.0, v.a01), dpp_fill<CTRL>(0.0, v.a10),
          dpp_fill<CTRL>(1.0, v.a11), dpp_fill<CTRL>(0.0, v.b0),  dpp_fill<CTRL>(0.0, v.b1)};
}
__device__ __forceinline__ Blk2 blk_lane(const Blk2 &v, int l) {
  return {lane_value(v.a00, l), lane_value(v.a01, l), lane_value(v.a10, l),
          lane_value(v.a11, l), lane_value(v.b0, l),  lane_value(v.b1, l)};
}

// Exclusive scan of the threads' composite maps M over the workgroup (WNW
// waves), applied to a zero boundary value: FWD, the maps of the threads
// below in ascending order; otherwise those above in descending order.
// slots: 2 x 64 doubles (parity halves, as wg_scan2).
template <bool FWD>
__device__ __forceinline__ void wg_scan_blk(Blk2 M, double &in0, double &in1, double *slots, int parity) {
  const int lane = threadIdx.x & 63, row = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (FWD) {
    M = blk_after(M, blk_dpp<0x111>(M));  // row_shr:1
    M = blk_after(M, blk_dpp<0x112>(M));  // row_shr:2
    M = blk_after(M, blk_dpp<0x114>(M));  // row_shr:4
    M = blk_after(M, blk_dpp<0x118>(M));  // row_shr:8
    const Blk2 r0 = blk_lane(M, 15), r1 = blk_lane(M, 31), r2 = blk_lane(M, 47);
    const Blk2 p1 = r0, p2 = blk_after(r1, p1), p3 = blk_after(r2, p2);
    if (row == 1) M = blk_after(M, p1);
    if (row == 2) M = blk_after(M, p2);
    if (row == 3) M = blk_after(M, p3);
  } else {
    M = blk_after(M, blk_dpp<0x101>(M));  // row_shl:1
    M = blk_after(M, blk_dpp<0x102>(M));  // row_shl:2
    M = blk_after(M, blk_dpp<0x104>(M));  // row_shl:4
    M = blk_after(M, blk_dpp<0x108>(M));  // row_shl:8
    const Blk2 r3 = blk_lane(M, 48), r2 = blk_lane(M, 32), r1 = blk_lane(M, 16);
    const Blk2 q2 = r3, q1 = blk_after(r2, q2), q0 = blk_after(r1, q1);
    if (row == 0) M = blk_after(M, q0);
    if (row == 1) M = blk_after(M, q1);
    if (row == 2) M = blk_after(M, q2);
  }
  const Blk2 E = FWD ? blk_dpp<0x138>(M) : blk_dpp<0x130>(M);  // wave_shr:1 / wave_shl:1
  const Blk2 T = blk_lane(M, FWD ? 63 : 0);                    // the wave's composite
  double *sl = slots + parity * 64;
  if (lane == 0) {
    sl[6 * wave + 0] = T.a00;
    sl[6 * wave + 1] = T.a01;
    sl[6 * wave + 2] = T.a10;
    sl[6 * wave + 3] = T.a11;
    sl[6 * wave + 4] = T.b0;
    sl[6 * wave + 5] = T.b1;
  }
  __syncthreads();
  double v0 = 0.0, v1 = 0.0;  // the value entering the wave
  if (FWD) {
    for (int k = 0; k < wave; ++k)
      blk_apply({sl[6 * k], sl[6 * k + 1], sl[6 * k + 2], sl[6 * k + 3], sl[6 * k + 4], sl[6 * k + 5]}, v0, v1);
  } else {
    for (int k = WNW - 1; k > wave; --k)
      blk_apply({sl[6 * k], sl[6 * k + 1], sl[6 * k + 2], sl[6 * k + 3], sl[6 * k + 4], sl[6 * k + 5]}, v0, v1);
  }
  blk_apply(E, v0, v1);
  in0 = v0;
  in1 = v1;
}

// d = C^{-1} rhs for the thread's unknowns [c0, c0 + n) (whole cells, n even)
template <int CMAX>
__device__ __forceinline__ void dsa_solve_dg(const Inst &I, int c0, int n, const double (&rhs)[CMAX],
                                             double (&d)[CMAX], double *slots, int &parity, bool alt = false) {
  constexpr int NCL = CMAX / 2;
  const int N = I.ncell, i0 = c0 / 2, ncl = n / 2;
  const double *__restrict__ K = alt ? I.dsa_blk_b : I.dsa_blk;
#pragma unroll
  for (int k = 0; k < CMAX; ++k) d[k] = 0.0;
  Blk2 fw[NCL];
  Blk2 T = blk_id();
#pragma unroll
  for (int k = 0; k < NCL; ++k) {
    if (k < ncl) {
      const int i = i0 + k;
      fw[k] = {ldg(&K[i]), ldg(&K[N + i]), ldg(&K[2 * N + i]), ldg(&K[3 * N + i]), rhs[2 * k], rhs[2 * k + 1]};
      T = blk_after(fw[k], T);
    }
  }
  double z0, z1;
  wg_scan_blk<true>(T, z0, z1, slots, parity);
  parity ^= 1;
  double z[CMAX];
#pragma unroll
  for (int k = 0; k < NCL; ++k) {
    if (k < ncl) {
      blk_apply(fw[k], z0, z1);
      z[2 * k] = z0;
      z[2 * k + 1] = z1;
    }
  }
  Blk2 bw[NCL];
  T = blk_id();
#pragma unroll
  for (int k = NCL - 1; k >= 0; --k) {
    if (k < ncl) {
      const int i = i0 + k;
      const double s00 = ldg(&K[4 * N + i]), s01 = ldg(&K[5 * N + i]);
      const double s10 = ldg(&K[6 * N + i]), s11 = ldg(&K[7 * N + i]);
      bw[k] = {ldg(&K[8 * N + i]), ldg(&K[9 * N + i]), ldg(&K[10 * N + i]), ldg(&K[11 * N + i]),
               rt_fma(s00, z[2 * k], s01 * z[2 * k + 1]), rt_fma(s10, z[2 * k], s11 * z[2 * k + 1])};
      T = blk_after(bw[k], T);
    }
  }
  double x0, x1;
  wg_scan_blk<false>(T, x0, x1, slots, parity);
  parity ^= 1;
#pragma unroll
  for (int k = NCL - 1; k >= 0; --k) {
    if (k < ncl) {
      blk_apply(bw[k], x0, x1);
      d[2 * k] = x0;
      d[2 * k + 1] = x1;
    }
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
// step on.  DG: the instantiation for piecewise-linear DG instances (two
// unknowns per cell: the sweeps of wave_sweep_dg, the block DSA of
// dsa_solve_dg); everything else works on the unknowns as on cells.
// ---------------------------------------------------------------------------
template <bool MH>
struct MhSlot {
  MhLds s;
};
template <>
struct MhSlot<false> {};

template <bool MH, bool DG>
__global__ void __launch_bounds__(WNT) k_si_wave(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if ((I.precond == RT_PC_MH) != MH || (I.dg != 0) != DG) return;
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
  // slots (odd), CM = C rounded up to a multiple of four.  DG: the run's
  // cells hold two slots each (rows of P = 2 CM + 1), and the threads own
  // whole cells outside the sweeps.
  const int ncl = DG ? nc / 2 : nc;  // cells
  const int C = (ncl + 63) / 64;
  const int CM = (C + 3) & ~3, P = DG ? 2 * CM + 1 : CM + 1;
  const int CW = DG ? 2 * ((ncl + WNT - 1) / WNT) : (nc + WNT - 1) / WNT;
  const int c0 = tid * CW;
  const int n = max(0, min(CW, nc - c0));
  int oidx[WOWN];
#pragma unroll
  for (int k = 0; k < WOWN; ++k) {
    const int u = c0 + min(k, max(n - 1, 0));  // unknown
    const int c = DG ? u / 2 : u;
    const int slot = DG ? 2 * (c % C) + (u & 1) : c % C;
    oidx[k] = min((c / C) * P + slot, 64 * WPM - 1);  // used only for k < n
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
    const int l = i / P, t = i - l * P, tc = DG ? t / 2 : t, c = l * C + tc;
    const double v = (tc < C && c < ncl) ? ldg(&ctp[DG ? 2 * c : c]) : 0.0;
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
  int need64 = 1, last_exact = 0;  // last_exact: whether the previous checked iterate came from an FP64 sweep
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
      if constexpr (DG) wave_sweep_dg_cls<double>(CM, npair, ct64, src, pmS, pwS, acc);
      else wave_sweep_cls<double>(CM, npair, ct64, src, pmS, pwS, acc);
      wave_reduce<double>(acc, DG ? 2 * C : C, P, redd, oidx, n, mom);
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
      if (!exact) {
        // mixed precision: the FP32-accumulated iterate passed; re-check it
        // on an FP64 sweep before accepting
        if (nsweep >= I.max_iter) break;
        need64 = 1;
        continue;
      }
      // DG: an iterate refined by FP32 increments must also pass on an
      // estimate of its error.  The stop test sees an error e of
      // rho^{(l-1)} only through the residual (T Sigma_s - I) e, which is
      // small for the slowly converging (diffusive) modes that DSA exists to
      // remove, and the FP32 increments of DG sweeps leave errors in exactly
      // those modes (uncaught, they accumulate over the steps).  The step to
      // the next DSA-corrected iterate, y - rho + C^{-1} Sigma_s (y - rho),
      // measures them and must pass the same test.  Finite-volume runs were
      // not seen to fail this check, and skip its DSA solve.
      bool accept = n32 == 0 || !DG;
      if (!accept) {
        double rhs[WOWN], dd[WOWN];
#pragma unroll
        for (int t = 0; t < WOWN; ++t) rhs[t] = ss[t] * (y[t] - rp[t]);
        if constexpr (DG) dsa_solve_dg<WOWN>(I, c0, n, rhs, dd, slots, parity, alt);
        double el = 0.0;
#pragma unroll
        for (int t = 0; t < WOWN; ++t)
          if (t < n) el = fmax(el, fabs((y[t] - rp[t]) + dd[t]));
        double en, e2;
        wg_max2(el, 0.0, red, en, e2);
        accept = stop_test(en, yn, I.tol_cert);
      }
      if (accept) {
        conv = 1;
        break;
      }
    }
    if (nsweep >= I.max_iter) break;
    if constexpr (MH) {
      // the pair of this iteration: (rho^{(l-1)} - rho^{(l-2)}, y_l - y_{l-1}).
      // Mixed precision: y_l - y_{l-1} is the image of the input difference
      // only along one chain of FP32 increments; a y_l recomputed by an FP64
      // sweep (the certification) replaces the accumulated value, and its
      // difference to the accumulated y_{l-1} would carry that chain's
      // rounding drift, not T Sigma_s x.  Such an iteration starts a new
      // chain instead of adding a pair.
      if (nsweep >= 2 && !(mixed && exact && !last_exact)) {
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
    last_exact = exact;
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
      // mixed precision: a level ROM is built from and applied to FP64-swept
      // iterates only (an FP32-refined one carries its increments' rounding)
      if (exact) used_mask |= 1 << (8 + k);
      const bool due = st->flag_pl[k] && ((used_mask >> (lc - 2)) & 1) && (!mixed || exact);
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
      if constexpr (DG) dsa_solve_dg<WOWN>(I, c0, n, rhs, d, slots, parity, alt);
      else dsa_solve_slab<WOWN>(I, c0, n, rhs, d, slots, parity, alt);
    }
    first_corr = 0;
    ncorr++;
    if (mixed && !(exact && resid < RT_FP64_BAND * I.tol)) {
      // y <- y + T32 Sigma_s (rho^{(l)} - rho^{(l-1)}): increment swept in FP32
#pragma unroll
      for (int t = 0; t < WOWN; ++t) {
        const double rn = y[t] + d[t];
        if (t < n) src32[oidx[t]] = (float)(ss[t] * (rn - rp[t]));
        rp[t] = rn;
      }
      __syncthreads();
      float acc[WCM], mom[WOWN];
      if constexpr (DG) wave_sweep_dg_cls<float>(CM, npair, ct32, src32, pmS, pwS, acc);
      else wave_sweep_cls<float>(CM, npair, ct32, src32, pmS, pwS, acc);
      wave_reduce<float>(acc, DG ? 2 * C : C, P, redf, oidx, n, mom);
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
  if (kinds & 1) hipLaunchKernelGGL((k_si_wave<false, false>), dim3(ninst), dim3(WNT), 0, stream, dinsts);
  if (kinds & 2) hipLaunchKernelGGL((k_si_wave<true, false>), dim3(ninst), dim3(WNT), 0, stream, dinsts);
  if (kinds & 4) hipLaunchKernelGGL((k_si_wave<false, true>), dim3(ninst), dim3(WNT), 0, stream, dinsts);
  if (kinds & 8) hipLaunchKernelGGL((k_si_wave<true, true>), dim3(ninst), dim3(WNT), 0, stream, dinsts);
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
  if (I.bdf2 || I.dg) return;  // k_fpass_wave_bdf2, k_fpass_dg
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
    // one block at a time: unrolled, the blocks' live ranges overlap (248 VGPRs, spills)
#pragma unroll 1
    for (int s = 0; s < NB; ++s) {
      {
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
  if (!I.bdf2 || I.dg) return;
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
    // one block at a time: unrolled, the blocks' live ranges overlap (248 VGPRs, spills)
#pragma unroll 1
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

// ---------------------------------------------------------------------------
// k_fpass_dg: the f-pass of piecewise-linear DG slabs in k_fpass_wave's
// layout and order, on unknowns: in block b lane l takes the two cells 128 b
// + 2 l, 128 b + 2 l + 1, i.e. the four unknowns 256 b + 4 l + k, so the
// loads of f are those of k_fpass_wave.  A lane composes its two cells' face
// maps (wave_sweep_dg), the wave scans them, and each cell's unknowns follow
// from the face value entering it.  First sweep: f^n with source sigma_s
// rho^n + f^{n-1} / dt + G and inflow g; second: b~^n from f^n / dt + G.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WNT) k_fpass_dg(const Inst *__restrict__ insts, int rhs_only) {
  const Inst &I = insts[blockIdx.x];
  if (!I.dg || I.bdf2) return;  // DG with BDF2: k_fpass_dg_bdf2
  __shared__ double big[4 * FROW];  // ct, srcc, G during the sweeps; then the moment rows
  double *ctS = big, *srcS = big + FROW, *gS = big + 2 * FROW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = I.nc, npair = I.npair, nv = I.nv;  // nc: unknowns
  const int NB = (nc + FB - 1) / FB;
  const double idt = I.inv_dt;
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
    double *fneg = I.f + (size_t)p * nc;
    double *fpos = I.f + (size_t)(nv - 1 - p) * nc;
    double cp1 = g0, cp2 = g0, cn1 = g1, cn2 = g1;
    // one block at a time: unrolled, the blocks' live ranges overlap (248 VGPRs, spills)
#pragma unroll 1
    for (int s = 0; s < NB; ++s) {
      {
        const int bp = s, bn = NB - 1 - s;
        const int cpb = bp * FB + lane * FK, cnb = bn * FB + lane * FK;
        double fp[FK], fn[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          fp[k] = cpb + k < nc ? ldg(&fpos[cpb + k]) : 0.0;
          fn[k] = cnb + k < nc ? ldg(&fneg[cnb + k]) : 0.0;
        }
        double cP[2], cN[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          cP[h] = ctS[fidx(cpb + 2 * h)];
          cN[h] = ctS[fidx(cnb + 2 * h)];
        }
        if (!rhs_only) {
          double sP[FK], sN[FK];
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            sP[k] = rt_fma(fp[k], idt, srcS[fidx(cpb + k)]);
            sN[k] = rt_fma(fn[k], idt, srcS[fidx(cnb + k)]);
          }
          DgCell<double> zp[2], zn[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            zp[h] = dg_cell<double>(cP[h], m, sP[2 * h], sP[2 * h + 1]);
            zn[h] = dg_cell<double>(cN[h], m, sN[2 * h], sN[2 * h + 1]);
          }
          const double pf = zp[0].a * zp[1].a, Bf = rt_fma(zp[1].a, zp[0].bf, zp[1].bf);
          const double pb = zn[0].a * zn[1].a, Bb = rt_fma(zn[0].a, zn[1].bb, zn[0].bb);
          double inF, inB;
          wave_scan2<double>(pf, Bf, pb, Bb, cp1, cn1, inF, inB);
          double f = inF;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            dg_unknowns<double, true>(cP[h], m, sP[2 * h], sP[2 * h + 1], zp[h].q, f, fp[2 * h], fp[2 * h + 1]);
            f = rt_fma(zp[h].a, f, zp[h].bf);
          }
#pragma unroll
          for (int k = 0; k < FK; ++k)
            if (cpb + k < nc) stg(&fpos[cpb + k], fp[k]);
          cp1 = lane_value(f, 63);
          f = inB;
#pragma unroll
          for (int h = 1; h >= 0; --h) {
            dg_unknowns<double, false>(cN[h], m, sN[2 * h], sN[2 * h + 1], zn[h].q, f, fn[2 * h], fn[2 * h + 1]);
            f = rt_fma(zn[h].a, f, zn[h].bb);
          }
#pragma unroll
          for (int k = 0; k < FK; ++k)
            if (cnb + k < nc) stg(&fneg[cnb + k], fn[k]);
          cn1 = lane_value(f, 0);
          // cells past the last one: zero sources of the second sweep
#pragma unroll
          for (int k = 0; k < FK; ++k) {
            if (cpb + k >= nc) fp[k] = 0.0;
            if (cnb + k >= nc) fn[k] = 0.0;
          }
        }
        // second sweep: source f^n / dt + G, the moments of b~^n
        double sP[FK], sN[FK];
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          sP[k] = rt_fma(fp[k], idt, gS[fidx(cpb + k)]);
          sN[k] = rt_fma(fn[k], idt, gS[fidx(cnb + k)]);
        }
        DgCell<double> zp[2], zn[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          zp[h] = dg_cell<double>(cP[h], m, sP[2 * h], sP[2 * h + 1]);
          zn[h] = dg_cell<double>(cN[h], m, sN[2 * h], sN[2 * h + 1]);
        }
        const double pf = zp[0].a * zp[1].a, Bf = rt_fma(zp[1].a, zp[0].bf, zp[1].bf);
        const double pb = zn[0].a * zn[1].a, Bb = rt_fma(zn[0].a, zn[1].bb, zn[0].bb);
        double inF, inB;
        wave_scan2<double>(pf, Bf, pb, Bb, cp2, cn2, inF, inB);
        double f = inF;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          dg_unknowns<double, true>(cP[h], m, sP[2 * h], sP[2 * h + 1], zp[h].q, f, fp[2 * h], fp[2 * h + 1]);
          f = rt_fma(zp[h].a, f, zp[h].bf);
        }
        cp2 = lane_value(f, 63);
        f = inB;
#pragma unroll
        for (int h = 1; h >= 0; --h) {
          dg_unknowns<double, false>(cN[h], m, sN[2 * h], sN[2 * h + 1], zn[h].q, f, fn[2 * h], fn[2 * h + 1]);
          f = rt_fma(zn[h].a, f, zn[h].bb);
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
  double *bt_out = rhs_only ? I.bt2[I.st->steps & 1] : I.bt2[I.st->cur ^ 1];
  for (int c = tid; c < nc; c += WNT) {
    const int i = fidx(c);
    stg(&bt_out[c], ((big[i] + big[FROW + i]) + big[2 * FROW + i]) + big[3 * FROW + i]);
  }
}

// ---------------------------------------------------------------------------
// k_fpass_dg_bdf2: the f-pass of DG slabs with BDF2, k_fpass_dg's cell maps in
// k_fpass_wave_bdf2's order of levels: for the step n just solved, f^n from
// rho^n with the source sigma_s rho^n + (4 f^{n-1} - f^{n-2}) / (2 dt) + G
// and the BDF2 operator (n = 1: the backward-Euler start), written over
// f^{n-2}; then b~^n of step n + 1 from (4 f^n - f^{n-1}) / (2 dt) + G with the
// BDF2 operator.  rhs_only: b~ of step S + 1 from the stored f^S, f^{S-1}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WNT) k_fpass_dg_bdf2(const Inst *__restrict__ insts, int rhs_only) {
  const Inst &I = insts[blockIdx.x];
  if (!I.dg || !I.bdf2) return;
  __shared__ double big[4 * FROW];  // ct (solve), ct (rhs), srcc, G; then the moment rows
  double *ctS = big, *srcS = big + FROW, *gS = big + 2 * FROW, *ct2S = big + 3 * FROW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = I.nc, npair = I.npair, nv = I.nv;  // nc: unknowns
  const int NB = (nc + FB - 1) / FB;
  const double idt = I.inv_dt, hidt = 0.5 * I.inv_dt;
  const long long S = I.st->steps;
  const bool now_b = !rhs_only && S >= 2;
  const bool next_b = rhs_only ? S >= 1 : true;
  const double *__restrict__ ct_now = now_b ? I.ct_b : I.ct;
  const double *__restrict__ ct_next = next_b ? I.ct_b : I.ct;
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
    double cp1 = g0, cp2 = g0, cn1 = g1, cn2 = g1;
    // one block at a time: unrolled, the blocks' live ranges overlap
#pragma unroll 1
    for (int s = 0; s < NB; ++s) {
      const int bp = s, bn = NB - 1 - s;
      const int cpb = bp * FB + lane * FK, cnb = bn * FB + lane * FK;
      // fp, fn: the newest level (f^n once solved); ap, an: the level before
      double fp[FK], fn[FK], ap[FK], an[FK];
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
      if (!rhs_only) {
        double cP[2], cN[2], sP[FK], sN[FK];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          cP[h] = ctS[fidx(cpb + 2 * h)];
          cN[h] = ctS[fidx(cnb + 2 * h)];
        }
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          const double hp = now_b ? rt_fma(4.0, ap[k], -fp[k]) * hidt : ap[k] * idt;
          const double hn = now_b ? rt_fma(4.0, an[k], -fn[k]) * hidt : an[k] * idt;
          sP[k] = hp + srcS[fidx(cpb + k)];
          sN[k] = hn + srcS[fidx(cnb + k)];
        }
        DgCell<double> zp[2], zn[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          zp[h] = dg_cell<double>(cP[h], m, sP[2 * h], sP[2 * h + 1]);
          zn[h] = dg_cell<double>(cN[h], m, sN[2 * h], sN[2 * h + 1]);
        }
        const double pf = zp[0].a * zp[1].a, Bf = rt_fma(zp[1].a, zp[0].bf, zp[1].bf);
        const double pb = zn[0].a * zn[1].a, Bb = rt_fma(zn[0].a, zn[1].bb, zn[0].bb);
        double inF, inB;
        wave_scan2<double>(pf, Bf, pb, Bb, cp1, cn1, inF, inB);
        double f = inF;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          dg_unknowns<double, true>(cP[h], m, sP[2 * h], sP[2 * h + 1], zp[h].q, f, fp[2 * h], fp[2 * h + 1]);
          f = rt_fma(zp[h].a, f, zp[h].bf);
        }
#pragma unroll
        for (int k = 0; k < FK; ++k)
          if (cpb + k < nc) stg(&fB[op + cpb + k], fp[k]);
        cp1 = lane_value(f, 63);
        f = inB;
#pragma unroll
        for (int h = 1; h >= 0; --h) {
          dg_unknowns<double, false>(cN[h], m, sN[2 * h], sN[2 * h + 1], zn[h].q, f, fn[2 * h], fn[2 * h + 1]);
          f = rt_fma(zn[h].a, f, zn[h].bb);
        }
#pragma unroll
        for (int k = 0; k < FK; ++k)
          if (cnb + k < nc) stg(&fB[on + cnb + k], fn[k]);
        cn1 = lane_value(f, 0);
#pragma unroll
        for (int k = 0; k < FK; ++k) {
          if (cpb + k >= nc) fp[k] = 0.0;
          if (cnb + k >= nc) fn[k] = 0.0;
        }
      }
      // right-hand side of the next step: source (4 f^n - f^{n-1}) / (2 dt) + G
      // (a backward-Euler step: f / dt + G), its operator
      double cP[2], cN[2], sP[FK], sN[FK];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        cP[h] = ct2S[fidx(cpb + 2 * h)];
        cN[h] = ct2S[fidx(cnb + 2 * h)];
      }
#pragma unroll
      for (int k = 0; k < FK; ++k) {
        sP[k] = (next_b ? rt_fma(4.0, fp[k], -ap[k]) * hidt : fp[k] * idt) + gS[fidx(cpb + k)];
        sN[k] = (next_b ? rt_fma(4.0, fn[k], -an[k]) * hidt : fn[k] * idt) + gS[fidx(cnb + k)];
      }
      DgCell<double> zp[2], zn[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        zp[h] = dg_cell<double>(cP[h], m, sP[2 * h], sP[2 * h + 1]);
        zn[h] = dg_cell<double>(cN[h], m, sN[2 * h], sN[2 * h + 1]);
      }
      const double pf = zp[0].a * zp[1].a, Bf = rt_fma(zp[1].a, zp[0].bf, zp[1].bf);
      const double pb = zn[0].a * zn[1].a, Bb = rt_fma(zn[0].a, zn[1].bb, zn[0].bb);
      double inF, inB;
      wave_scan2<double>(pf, Bf, pb, Bb, cp2, cn2, inF, inB);
      double f = inF;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        dg_unknowns<double, true>(cP[h], m, sP[2 * h], sP[2 * h + 1], zp[h].q, f, fp[2 * h], fp[2 * h + 1]);
        f = rt_fma(zp[h].a, f, zp[h].bf);
      }
      cp2 = lane_value(f, 63);
      f = inB;
#pragma unroll
      for (int h = 1; h >= 0; --h) {
        dg_unknowns<double, false>(cN[h], m, sN[2 * h], sN[2 * h + 1], zn[h].q, f, fn[2 * h], fn[2 * h + 1]);
        f = rt_fma(zn[h].a, f, zn[h].bb);
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

// ---------------------------------------------------------------------------
// k_setup_dsa_dg: the DSA operator of DG slabs and its block elimination.
// The operator: the correction equation's diffusion limit -(D d')' +
// sigma~_a d (D = 1/(3 sigma~_t), sigma~_a = sigma_a + 1/dt) in the DG-P1
// space by the modified interior penalty method -- symmetric interior
// penalty with kappa = max((D_L + D_R) / h, 1/4) on interior faces and
// Marshak vacuum faces (1/2 u v) -- divided by h, so that its right-hand
// side is sigma_s times the unknown-wise residual (the orthonormal basis
// has mass matrix h I).  Per cell, with e+ = (1, sqrt 3), e- = (1, -sqrt 3)
// the basis at the right / left end and g = (0, 2 sqrt(3) / h) the
// derivatives (all terms / h):
//   D_i = h diag(sa~, sa~ + 12 D_i / h^2)
//         + [left face]  kappa e- e-^T + (D_i / 2)(g e-^T + e- g^T)   (Marshak: e- e-^T / 2)
//         + [right face] kappa e+ e+^T - (D_i / 2)(g e+^T + e+ g^T)   (Marshak: e+ e+^T / 2)
//   L_i = -kappa e- e+^T + (D_{i-1} / 2) e- g^T - (D_i / 2) g e+^T      (row i, column i - 1)
// Block elimination: S_0 = D_0, S_i = D_i - L_i S_{i-1}^{-1} L_i^T
// (sequential, one thread), then F_i = -L_i S_{i-1}^{-1} and B_i =
// -S_i^{-1} L_{i+1}^T.  One workgroup per instance; blocks in LDS.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_setup_dsa_dg(const Inst *__restrict__ insts, int alt) {
  const Inst &I = insts[blockIdx.x];
  if (!I.dg) return;
  __shared__ double Dl[4 * RT_DG_MAX_CELLS], Ll[4 * RT_DG_MAX_CELLS], Sl[4 * RT_DG_MAX_CELLS];
  const int N = I.ncell;
  const double h = I.hx, r3 = kR3, dd = 2.0 * kR3 / h;
  // alt: the BDF2 operator (time weight 3 / (2 dt))
  double *K = const_cast<double *>(alt ? I.dsa_blk_b : I.dsa_blk);
  const double *__restrict__ ctp = alt ? I.ct_b : I.ct;
  const double adt = alt ? I.adt_b : I.inv_dt;
  auto Dif = [&](int i) { return 1.0 / (3.0 * ldg(&ctp[2 * i])); };
  auto kap = [&](double a, double b) { return fmax((a + b) / h, 0.25); };
  const double ep[2] = {1.0, r3}, em[2] = {1.0, -r3}, gd[2] = {0.0, dd};
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double Di = Dif(i);
    const double sat = ldg(&I.sa[2 * i]) + adt;
    double A[2][2] = {{sat * h, 0.0}, {0.0, sat * h + 12.0 * Di / h}};
    const double kl = i > 0 ? kap(Dif(i - 1), Di) : 0.0;
    const double kr = i < N - 1 ? kap(Di, Dif(i + 1)) : 0.0;
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        A[r][c] += i > 0 ? kl * em[r] * em[c] + 0.5 * Di * (gd[r] * em[c] + em[r] * gd[c]) : 0.5 * em[r] * em[c];
        A[r][c] += i < N - 1 ? kr * ep[r] * ep[c] - 0.5 * Di * (gd[r] * ep[c] + ep[r] * gd[c]) : 0.5 * ep[r] * ep[c];
        Dl[4 * i + 2 * r + c] = A[r][c] / h;
        Ll[4 * i + 2 * r + c] =
            i > 0 ? (-kl * em[r] * ep[c] + 0.5 * Dif(i - 1) * em[r] * gd[c] - 0.5 * Di * gd[r] * ep[c]) / h : 0.0;
      }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // S_i^{-1}, i = 0..N-1
    double s00 = Dl[0], s01 = Dl[1], s10 = Dl[2], s11 = Dl[3];
    for (int i = 0;; ++i) {
      const double id = rt_rcp(s00 * s11 - s01 * s10);
      const double i00 = s11 * id, i01 = -s01 * id, i10 = -s10 * id, i11 = s00 * id;
      Sl[4 * i] = i00;
      Sl[4 * i + 1] = i01;
      Sl[4 * i + 2] = i10;
      Sl[4 * i + 3] = i11;
      if (i + 1 == N) break;
      const double *L = Ll + 4 * (i + 1), *D = Dl + 4 * (i + 1);
      // X = L S^{-1}; S' = D - X L^T
      const double x00 = L[0] * i00 + L[1] * i10, x01 = L[0] * i01 + L[1] * i11;
      const double x10 = L[2] * i00 + L[3] * i10, x11 = L[2] * i01 + L[3] * i11;
      s00 = D[0] - (x00 * L[0] + x01 * L[1]);
      s01 = D[1] - (x00 * L[2] + x01 * L[3]);
      s10 = D[2] - (x10 * L[0] + x11 * L[1]);
      s11 = D[3] - (x10 * L[2] + x11 * L[3]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double *S = Sl + 4 * i;
    double F[4] = {0.0, 0.0, 0.0, 0.0}, B[4] = {0.0, 0.0, 0.0, 0.0};
    if (i > 0) {  // F_i = -L_i S_{i-1}^{-1}
      const double *L = Ll + 4 * i, *P = Sl + 4 * (i - 1);
      F[0] = -(L[0] * P[0] + L[1] * P[2]);
      F[1] = -(L[0] * P[1] + L[1] * P[3]);
      F[2] = -(L[2] * P[0] + L[3] * P[2]);
      F[3] = -(L[2] * P[1] + L[3] * P[3]);
    }
    if (i + 1 < N) {  // B_i = -S_i^{-1} L_{i+1}^T
      const double *L = Ll + 4 * (i + 1);
      B[0] = -(S[0] * L[0] + S[1] * L[1]);
      B[1] = -(S[0] * L[2] + S[1] * L[3]);
      B[2] = -(S[2] * L[0] + S[3] * L[1]);
      B[3] = -(S[2] * L[2] + S[3] * L[3]);
    }
    for (int k = 0; k < 4; ++k) {
      K[k * N + i] = F[k];
      K[(4 + k) * N + i] = S[k];
      K[(8 + k) * N + i] = B[k];
    }
  }
}

extern "C" hipError_t rt_launch_setup_dsa_dg(const Inst *dinsts, int ninst, int alt, hipStream_t stream) {
  hipLaunchKernelGGL(k_setup_dsa_dg, dim3(ninst), dim3(256), 0, stream, dinsts, alt);
  return hipGetLastError();
}

extern "C" hipError_t rt_launch_slab_fpass_wave(const Inst *dinsts, int ninst, int rhs_only, int kinds,
                                                hipStream_t stream) {
  if (kinds & 1) hipLaunchKernelGGL(k_fpass_wave, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  if (kinds & 2) hipLaunchKernelGGL(k_fpass_wave_bdf2, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  if (kinds & 4) hipLaunchKernelGGL(k_fpass_dg, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  if (kinds & 16) hipLaunchKernelGGL(k_fpass_dg_bdf2, dim3(ninst), dim3(WNT), 0, stream, dinsts, rhs_only);
  return hipGetLastError();
}
