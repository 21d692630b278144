// rt_mh.h -- McClarren-Haut correction (Sec. 3.3) inside the one-workgroup
// slab SI kernel: a DMD model of the sweep operator T Sigma_s built from the
// pairs of the current step's iterates.
//
// Pair l (iterations l >= 2): input x = rho^{(l-1)} - rho^{(l-2)}, image
// z = y_l - y_{l-1} = T Sigma_s x, both scaled by 1/||x||_2.  The inputs are
// orthonormalised as they arrive (classical Gram-Schmidt applied twice) into
// Q, so X = Q R; with B = Q^T Z the model's reduced operator is
// A~ = Q^T Z R^{-1} = B R^{-1} (the pairs' DMD, computed through the QR of the
// inputs instead of an SVD: the same operator without truncation).  The
// correction restricts the ideal correction equation (eq. ideal_correct),
// (I - T Sigma_s) d = T Sigma_s r with r = y_l - rho^{(l-1)}, to span(Q):
// d = Q (I - A~)^{-1} A~ Q^T r.  A pair whose scaled input keeps an
// orthogonal remainder of at most 1e-6 adds nothing and is skipped; a full
// model (mh_cap pairs) restarts from the newest pair.
//
// Q and Z live in global memory ([mh_cap][ld], column k contiguous, whole
// cache lines); every thread touches only its own cells, and a column is
// written once per step before any read of it, so no thread reads a line it
// has written since the kernel started.  R, B and the small system, which
// change every iteration, live in LDS only (a global copy rewritten and read
// back within the kernel could be served from a stale L1 line); the O(m^2)
// and O(m^3) work runs on wave 0.
#pragma once
#include "rt_common.h"
#include "rt_rom.h"

constexpr double RT_MH_DEP = 1e-6;
constexpr int RT_MH_NP = 2 * RT_RMAX + 1;  // partial sums of the first pass

struct MhLds {
  double R[RT_RMAX * RT_RMAX];  // R[i * RT_RMAX + j], upper triangular
  double B[RT_RMAX * RT_RMAX];  // B = Q^T Z
  double A[RT_RMAX * RT_KC];    // I - A~ for the LU (stride RT_KC)
  double red[RT_MAXWAVES * RT_MH_NP];
  double out[RT_MH_NP];
  double qz[RT_RMAX];  // Q^T z of the pair being added
  double vec[RT_RMAX];
  double P[RT_RMAX * RT_KC];  // pivot rows of the elimination, right-hand side in column RT_RMAX
  int m, flag;
};

// Solve (I - A~) c = g by Gaussian elimination with partial pivoting on wave
// 0, in LDS: S.A holds the matrix (stride RT_KC), S.vec the right-hand side
// and, on return, c.  Lane i keeps row i (and its right-hand side) in
// registers; step k picks the largest |a_ik| among the rows not yet used
// (lowest row on ties), publishes it in S.P and eliminates below it; the back
// substitution broadcasts one solved component per step.  A pivot below
// 1e-14 max|A| marks the system singular: returns 1 (every thread) and
// leaves S.vec undefined.  Every thread calls; ends with a barrier.
__device__ inline int mh_solve_wave(MhLds &S, int m) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const bool mine = lane < m;
    double row[RT_RMAX], rhs = mine ? S.vec[lane] : 0.0;
    double amax = 0.0;
#pragma unroll
    for (int j = 0; j < RT_RMAX; ++j) {
      row[j] = (mine && j < m) ? S.A[lane * RT_KC + j] : 0.0;
      amax = fmax(amax, fabs(row[j]));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    int bad = (amax == 0.0);
    bool active = mine;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      if (k < m) {
        double v = active ? fabs(row[k]) : -1.0;
        double vmax = v;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
        const unsigned long long cand = __ballot(active && v == vmax);
        const int p = cand ? __builtin_ctzll(cand) : __builtin_ctzll(__ballot(active) | (1ull << 63));
        if (!cand) bad = 1;
        if (lane == p) {
#pragma unroll
          for (int j = 0; j < RT_RMAX; ++j) S.P[k * RT_KC + j] = row[j];
          S.P[k * RT_KC + RT_RMAX] = rhs;
          active = false;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double akk = S.P[k * RT_KC + k];
        if (akk == 0.0 || fabs(akk) < 1e-14 * amax) {
          bad = 1;
          continue;
        }
        if (active) {
          const double l = row[k] / akk;
#pragma unroll
          for (int j = 0; j < RT_RMAX; ++j)
            if (j > k) row[j] = rt_fma(-l, S.P[k * RT_KC + j], row[j]);
          rhs = rt_fma(-l, S.P[k * RT_KC + RT_RMAX], rhs);
        }
      }
    }
    if (lane == 0) S.flag = bad;
    if (!bad) {
      // back substitution on the pivot rows: lane i holds component i
      double s = mine ? S.P[lane * RT_KC + RT_RMAX] : 0.0;
#pragma unroll
      for (int j = RT_RMAX - 1; j >= 0; --j) {
        if (j < m) {
          const double xj = __shfl(s, j, 64) / S.P[j * RT_KC + j];
          if (lane == j) s = xj;
          if (mine && lane < j) s = rt_fma(-S.P[lane * RT_KC + j], xj, s);
        }
      }
      if (mine) S.vec[lane] = s;
    }
  }
  __syncthreads();
  const int bad = S.flag;
  __syncthreads();
  return bad;
}

// Add the pair (x, z) given per thread on its cells [c0, c0 + n).  Every
// thread calls; S.m must be current in LDS.  Ends with a barrier.
template <int NW>
__device__ inline void mh_push(const Inst &I, int c0, int n, const double (&x)[NW], const double (&z)[NW],
                               MhLds &S) {
  const int ld = I.ld, cap = I.mh_cap;
  const int mold = S.m;
  const int m0 = mold == cap ? 0 : mold;  // a full model restarts
  double part[RT_MH_NP];
#pragma unroll
  for (int k = 0; k < RT_MH_NP; ++k) part[k] = 0.0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    if (t < n) {
      const int c = c0 + t;
      const double xv = x[t], zv = z[t];
      part[2 * RT_RMAX] = rt_fma(xv, xv, part[2 * RT_RMAX]);
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k) {
        if (k < m0) {
          const double q = ldg(&I.mhQ[(size_t)k * ld + c]);
          part[k] = rt_fma(q, xv, part[k]);
          part[RT_RMAX + k] = rt_fma(q, zv, part[RT_RMAX + k]);
        }
      }
    }
  }
  wg_sum_fast<RT_MH_NP>(part, S.red, S.out);
  const double xx = S.out[2 * RT_RMAX];
  if (!(xx > 0.0)) return;  // no input difference: nothing to learn
  const double xn = sqrt(xx), ixn = 1.0 / xn;
  double a1[RT_RMAX];
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) a1[k] = k < m0 ? S.out[k] * ixn : 0.0;
  if ((int)threadIdx.x < m0) S.qz[threadIdx.x] = S.out[RT_RMAX + threadIdx.x];
  // second Gram-Schmidt pass: a2 = Q^T p, p = x / ||x|| - Q a1
  double p[NW];
  double part2[RT_RMAX + 1];
#pragma unroll
  for (int k = 0; k <= RT_RMAX; ++k) part2[k] = 0.0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    p[t] = 0.0;
    if (t < n) {
      const int c = c0 + t;
      double q[RT_RMAX];
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k) q[k] = k < m0 ? ldg(&I.mhQ[(size_t)k * ld + c]) : 0.0;
      double pv = x[t] * ixn;
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k) pv = rt_fma(-q[k], a1[k], pv);
      p[t] = pv;
      part2[RT_RMAX] = rt_fma(pv, pv, part2[RT_RMAX]);
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k) part2[k] = rt_fma(q[k], pv, part2[k]);
    }
  }
  wg_sum_fast<RT_RMAX + 1>(part2, S.red, S.out);
  double ac[RT_RMAX], a2s = 0.0;
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) {
    const double a2 = k < m0 ? S.out[k] : 0.0;
    ac[k] = a1[k] + a2;
    a2s = rt_fma(a2, a2, a2s);
  }
  const double nu = sqrt(fmax(S.out[RT_RMAX] - a2s, 0.0));
  if (!(nu > RT_MH_DEP)) return;  // in span already (never at m0 = 0: nu = 1)
  const double inu = 1.0 / nu;
  // new column of R and of B = Q^T Z: R[k][m0] = (a1 + a2)_k, R[m0][m0] = nu,
  // B[k][m0] = q_k . z^ (the first pass's sums)
  const int tid = threadIdx.x;
  if (tid < m0) {
    S.R[tid * RT_RMAX + m0] = ac[tid];
    S.B[tid * RT_RMAX + m0] = S.qz[tid] * ixn;
  } else if (tid == 128) {
    S.R[m0 * RT_RMAX + m0] = nu;
  }
  // the new columns of Q and Z on the thread's own cells, and the new row of
  // B as direct dot products q . Z_j, q . z^ (forming it from the first
  // pass's sums, (x^ . Z_j - ac . B[:, j]) / nu, cancels to rounding and
  // divides that by nu)
  double part3[RT_RMAX + 1];
#pragma unroll
  for (int k = 0; k <= RT_RMAX; ++k) part3[k] = 0.0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    if (t < n) {
      const int c = c0 + t;
      double v = x[t] * ixn;
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k)
        if (k < m0) v = rt_fma(-ldg(&I.mhQ[(size_t)k * ld + c]), ac[k], v);
      v *= inu;
      const double zh = z[t] * ixn;
      stg(&I.mhQ[(size_t)m0 * ld + c], v);
      stg(&I.mhZ[(size_t)m0 * ld + c], zh);
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k)
        if (k < m0) part3[k] = rt_fma(v, ldg(&I.mhZ[(size_t)k * ld + c]), part3[k]);
      part3[RT_RMAX] = rt_fma(v, zh, part3[RT_RMAX]);
    }
  }
  wg_sum_fast<RT_RMAX + 1>(part3, S.red, S.out);
  if (tid < m0) S.B[m0 * RT_RMAX + tid] = S.out[tid];
  else if (tid == 128) S.B[m0 * RT_RMAX + m0] = S.out[RT_RMAX];
  __syncthreads();
  if (tid == 0) S.m = m0 + 1;
  __syncthreads();
}

// The correction d for the residual r (per thread on its cells); d = 0 when
// the model is empty or I - A~ is singular.  Returns 1 when applied.  Every
// thread calls.  Ends with a barrier.
template <int NW>
__device__ inline int mh_correct(const Inst &I, int c0, int n, const double (&r)[NW], double (&d)[NW], MhLds &S) {
  const int ld = I.ld, m = S.m;
#pragma unroll
  for (int t = 0; t < NW; ++t) d[t] = 0.0;
  if (m == 0) return 0;
  double part[RT_RMAX];
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) part[k] = 0.0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    if (t < n) {
      const int c = c0 + t;
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k)
        if (k < m) part[k] = rt_fma(ldg(&I.mhQ[(size_t)k * ld + c]), r[t], part[k]);
    }
  }
  wg_sum_fast<RT_RMAX>(part, S.red, S.out);  // S.out[k] = Q^T r
  // wave 0, lane i < m: row i of A~ = B R^{-1} (forward substitution along
  // the row), g_i = (A~ Q^T r)_i, row i of I - A~
  if (threadIdx.x < 64) {
    const int i = threadIdx.x;
    if (i < m) {
      double at[RT_RMAX];
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j) {
        if (j < m) {
          double v = S.B[i * RT_RMAX + j];
#pragma unroll
          for (int k = 0; k < RT_RMAX; ++k)
            if (k < j) v = rt_fma(-at[k], S.R[k * RT_RMAX + j], v);
          at[j] = v / S.R[j * RT_RMAX + j];
        } else {
          at[j] = 0.0;
        }
      }
      double g = 0.0;
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j)
        if (j < m) g = rt_fma(at[j], S.out[j], g);
      S.vec[i] = g;
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j)
        if (j < m) S.A[i * RT_KC + j] = (i == j ? 1.0 : 0.0) - at[j];
    }
  }
  __syncthreads();
  if (mh_solve_wave(S, m)) return 0;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    if (t < n) {
      const int c = c0 + t;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < RT_RMAX; ++k)
        if (k < m) v = rt_fma(ldg(&I.mhQ[(size_t)k * ld + c]), S.vec[k], v);
      d[t] = v;
    }
  }
  return 1;
}
