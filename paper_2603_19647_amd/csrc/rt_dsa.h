// rt_dsa.h -- the slab DSA solve and Alg. 1's stop test, shared by the slab
// SI kernels (one instance per workgroup, cells split over the threads in
// contiguous runs).
#pragma once
#include "rt_common.h"

// DSA correction (eq. rho_residual): solve C d = rhs with the precomputed
// Thomas factors written as two affine recurrences, z_i = fe_i z_{i-1} + rhs_i
// forward and d_i = bg_i d_{i+1} + invd_i z_i backward.  alt: the factors of
// the BDF2 operator.
template <int CMAX>
__device__ __forceinline__ void dsa_solve_slab(const Inst &I, int c0, int n, const double (&rhs)[CMAX],
                                               double (&d)[CMAX], double *slots, int &parity, bool alt = false) {
  const double *__restrict__ dfe = alt ? I.dsa_fe_b : I.dsa_fe;
  const double *__restrict__ dbg = alt ? I.dsa_bg_b : I.dsa_bg;
  const double *__restrict__ dinvd = alt ? I.dsa_invd_b : I.dsa_invd;
  double fe[CMAX], z[CMAX];
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int t = 0; t < CMAX; ++t) {
    if (t < n) {
      fe[t] = ldg(&dfe[c0 + t]);
      B = rt_fma(fe[t], B, rhs[t]);
      A *= fe[t];
    }
  }
  double inF, inB;
  wg_scan2<double>(A, B, 1.0, 0.0, 0.0, 0.0, inF, inB, slots, parity);
  parity ^= 1;
  double f = inF;
#pragma unroll
  for (int t = 0; t < CMAX; ++t) {
    if (t < n) {
      f = rt_fma(fe[t], f, rhs[t]);
      z[t] = f;
    }
  }
  double bg[CMAX];
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int t = CMAX - 1; t >= 0; --t) {
    if (t < n) {
      bg[t] = ldg(&dbg[c0 + t]);
      z[t] *= ldg(&dinvd[c0 + t]);
      B = rt_fma(bg[t], B, z[t]);
      A *= bg[t];
    }
  }
  wg_scan2<double>(1.0, 0.0, A, B, 0.0, 0.0, inF, inB, slots, parity);
  parity ^= 1;
  f = inB;
#pragma unroll
  for (int t = CMAX - 1; t >= 0; --t) {
    if (t < n) {
      f = rt_fma(bg[t], f, z[t]);
      d[t] = f;
    }
  }
}

__device__ __forceinline__ bool stop_test(double dn, double yn, double tol) {
  return yn > 0.0 ? (dn < tol * yn) : (dn < tol);
}
