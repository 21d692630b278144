// rt_rom.h -- device code of the ROM work: DMD reduced solve (Sec. 3.1,
// eq. dmd-operator, eq. dmd-ig, eq. dmd-sa) and the incremental SVD update
// (App. B, eq. svd_core) with the reduced operator kept incrementally.
//
// The O(N r) projection passes run grid-wide (k_rom_pass1/2, or at the end
// of the cooperative SI kernel) or, for a small slab, inside one workgroup
// per (instance, ROM) (k_rom_post_small); the (r+1)^2 core SVD and the r x r
// LU run in one workgroup per ROM.  The O(N r^2) basis rotation
// U <- [U q] U_c, W <- [W b] V_c applies the "pending update" the core leaves
// behind: grid-wide (k_rom_update, the cooperative step tail) or, for a
// small slab, by the same post workgroup (rom_rotate_own_lu).  Cells are owned
// with a stride (c = tid, tid + NT, ...) so that every pass over a basis
// column is a coalesced stream.
#pragma once
#include "rt_arrow.h"
#include "rt_common.h"

struct RomSmem {
  double B[RT_KC * RT_KC];   // core matrix, rotated in place: B[col*RT_KC + row]
  double V[RT_KC * RT_KC];   // accumulated right rotations: V[col*RT_KC + row]
  double Mx[RT_KC * RT_KC];  // Q^T [W b]: Mx[row*RT_KC + col]
  double T1[RT_KC * RT_KC];  // Mx Vc[:, :k]
  double Uc[RT_KC * RT_KC];  // sorted left vectors of the core: Uc[row*RT_KC + j]
  double Vc[RT_KC * RT_KC];  // sorted right vectors: Vc[row*RT_KC + j]
  double A[RT_KC * RT_KC];   // reduced operator / LU workspace, stride RT_KC
  double sv[RT_KC];          // sorted singular values
  double nrm[RT_KC];
  double vec[48];            // reduction results
  double av[RT_RMAX], a2v[RT_RMAX], utbv[RT_RMAX], pwv[RT_RMAX];  // projection coefficients
  double red[RT_MAXWAVES * 48];
  double scratch[1024];      // sum_partials: one entry per thread
  int perm[RT_KC];
  arrow::Problem ap;         // secular core SVD: non-deflated poles
  double ap_tau[RT_KC], ap_zh[RT_KC];
  int ap_K[RT_KC], ap_defl[RT_KC], ap_ok;
  short pairs[RT_KC * RT_KC];  // round-robin pairing table (p, q) per round and slot
  int flag;
  int ibuf[4];
};

// ---------------------------------------------------------------------------
// 16-lane (one DPP row) sum: quad xor 1, quad xor 2, half-row mirror, row
// mirror leave the row total in every lane of the row.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}
// sum over a DPP quad (4 lanes), identical in every lane of the quad
struct QuadSum {
  __device__ double operator()(double v) const {
    v += dpp_d<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);  // quad_perm [2,3,0,1]
    return v;
  }
};
// sum over 8 lanes (two quads), identical in every lane of the eight:
// the quads' sums, then each half-row lane adds its mirror's (the other quad)
struct OctSum {
  __device__ double operator()(double v) const {
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    return v;
  }
};
// whole-wave sum, identical in every lane
__device__ __forceinline__ double wave_sum_fast(double v) {
  v = row16_sum(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Workgroup sum of NV per-thread partials; totals land in out[0..NV).
template <int NV>
__device__ __forceinline__ void wg_sum_fast(const double (&v)[NV], double *red, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = wave_sum_fast(v[k]);
    if (lane == 0) red[wave * NV + k] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ROM z of an instance: 0 the initial guess, 1 the correction of iteration
// 1, l the correction of iteration l
__device__ __forceinline__ const RomDev &rom_of(const Inst &I, int z) {
  return z == 0 ? I.ig : (z == 1 ? I.pc : I.pl[z - 2]);
}
__device__ __forceinline__ int *rom_rank_of(RtState *st, int z) {
  return z == 0 ? &st->rank_ig : (z == 1 ? &st->rank_pc : &st->rank_pl[z - 2]);
}
__device__ __forceinline__ int *rom_luok_of(RtState *st, int z) {
  return z == 0 ? &st->lu_ok_ig : (z == 1 ? &st->lu_ok_pc : &st->lu_ok_pl[z - 2]);
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of the n x n matrix in A (stride RT_KC, LDS), by
// wave 0.  Lane i keeps row i in registers for the whole factorisation; rows
// are not moved: step k picks the pivot among the rows not yet used (largest
// |a_ik|, lowest row on ties), reads the pivot row with lane reads and
// eliminates below it in place, so every row keeps its own multipliers, as in
// a factorisation with row interchanges.  A pivot below tol max|A| marks the
// system singular (tol: the ROM's lu_tol, 1e-14 unless the caller set it).  Writes the factors in pivot order (stride RT_RMAX)
// and the row permutation to global memory and returns 1 if singular.  Must
// be called by the whole workgroup; A's first row is overwritten (it carries
// the pivot rows once the matrix is in registers).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dpp_max16(double v) {
  v = fmax(v, dpp_d<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_d<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_d<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_d<0x140>(v));  // row_mirror
  return v;
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// The factorisation itself, by wave 0 alone (no workgroup barrier): the
// calling wave must be wave 0; returns 1 if singular (every lane).
__device__ inline int lu_factor_rows(double *A, int n, double *LUg, int *permg, double tol) {
  static_assert(RT_RMAX <= 32, "rows live in the first two DPP rows of the wave");
  int bad;
  {
    const int lane = threadIdx.x;
    const bool mine = lane < n;
    double row[RT_RMAX];
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < RT_RMAX; ++j) {
      row[j] = (mine && j < n) ? A[lane * RT_KC + j] : 0.0;
      m = fmax(m, fabs(row[j]));
    }
    m = dpp_max16(m);
    const double amax = fmax(lane_read(m, 0), lane_read(m, 16));
    bad = (amax == 0.0);
    bool active = mine;
    int pos = 0;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      if (k < n) {
        const double v = active ? fabs(row[k]) : -1.0;
        const double w = dpp_max16(v);
        const double vmax = fmax(lane_read(w, 0), lane_read(w, 16));
        const unsigned long long cand = __ballot(active && v == vmax);
        // no candidate only for a NaN column: take the lowest unused row
        const int p = cand ? __builtin_ctzll(cand) : __builtin_ctzll(__ballot(active));
        if (!cand) bad = 1;
        if (lane == p) {
          active = false;
          pos = k;
        }
        // the pivot row to every lane through LDS (A is free: rows live in
        // registers), one write and one broadcast read per entry
        if (lane == p) {
#pragma unroll
          for (int j = k; j < RT_RMAX; ++j) A[j] = row[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double prow[RT_RMAX];
#pragma unroll
        for (int j = k; j < RT_RMAX; ++j) prow[j] = A[j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double akk = prow[k];
        if (akk == 0.0 || fabs(akk) < tol * amax) {
          bad = 1;
          continue;
        }
        const double rinv = 1.0 / akk;
        const double l = row[k] * rinv;
        if (active) row[k] = l;
#pragma unroll
        for (int j = k + 1; j < RT_RMAX; ++j)
          if (active) row[j] = rt_fma(-l, prow[j], row[j]);
      }
    }
    if (mine) {
#pragma unroll
      for (int j = 0; j < RT_RMAX; ++j)
        if (j < n) stg(&LUg[pos * RT_RMAX + j], row[j]);
      stg(&permg[pos], lane);
    }
  }
  return bad;
}

__device__ inline int lu_factor_wave(double *A, int *perm_lds, int n, double *LUg, int *permg, int *flag,
                                     double tol) {
  (void)perm_lds;
  if (threadIdx.x < 64) {
    const int bad = lu_factor_rows(A, n, LUg, permg, tol);
    if (threadIdx.x == 0) *flag = bad;
  }
  __syncthreads();
  const int bad = *flag;
  __syncthreads();
  return bad;
}

// out[k] = sum over blocks b < nb of part[b * RT_NPART + k], k < ncol.  The
// blocks of a column are split into RT_SUMJ interleaved strands, each summed
// in block order, and the strands are then added in order: a fixed order, so
// the result is deterministic.  Needs blockDim.x a multiple of RT_SUMJ and
// scratch of blockDim.x doubles in LDS; every thread must call; ends with a
// barrier.
constexpr int RT_SUMJ = 8;
// partial rows: plain or (COH) agent-scope atomic accesses
template <bool COH>
__device__ __forceinline__ void part_store(double *p, double v) {
  if constexpr (COH) xstore(p, v);
  else stg(p, v);
}
template <bool COH>
__device__ __forceinline__ double part_load(const double *p) {
  if constexpr (COH) return xload(p);
  else return ldg(p);
}
template <bool COH>
__device__ inline void sum_partials(const double *part, int nb, int ncol, double *out, double *scratch) {
  const int tid = threadIdx.x, per = blockDim.x / RT_SUMJ;
  for (int k0 = 0; k0 < ncol; k0 += per) {
    const int k = k0 + tid % per, j = tid / per;
    double s = 0.0;
    if (k < ncol)
      for (int b = j; b < nb; b += RT_SUMJ) s += part_load<COH>(&part[b * RT_NPART + k]);
    scratch[tid] = s;
    __syncthreads();
    if (tid < per && k0 + tid < ncol) {
      double t = 0.0;
      for (int jj = 0; jj < RT_SUMJ; ++jj) t += scratch[jj * per + tid];
      out[k0 + tid] = t;
    }
    __syncthreads();
  }
}

// Solve A_r c = vec in place (vec in LDS) with the factors of lu_factor_wave
// (global or LDS), by wave 0: lane i holds row i of the factors; forward and
// back substitution broadcast one solved component per step, the back
// substitution multiplying by the pivots' reciprocals.
__device__ inline void lu_solve_wave(const double *LU, const int *perm, int n, double *vec) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int li = lane < RT_RMAX ? lane : RT_RMAX - 1;
    const bool mine = lane < n;
    // the row is read element by element as the substitution reaches it
    // (factors in LDS or cache): no register array of the whole row
    const double *row = LU + li * RT_RMAX;
    const double b = vec[perm[li]];
    // every lane inverts its own pivot at once, off the substitution chain
    const double rpiv = mine ? 1.0 / row[li] : 0.0;
    double s = mine ? b : 0.0;
    // forward substitution (unit lower factor): component j is final on lane j
#pragma unroll 4
    for (int j = 0; j < RT_RMAX; ++j) {
      const double bj = lane_read(s, j);
      const double l = row[j];
      if (mine && lane > j && j < n) s = rt_fma(-l, bj, s);
    }
#pragma unroll 4
    for (int j = RT_RMAX - 1; j >= 0; --j) {
      if (j < n) {
        const double u = row[j];
        const double xj = lane_read(s, j) * lane_read(rpiv, j);
        if (lane == j) s = xj;
        if (mine && lane < j) s = rt_fma(-u, xj, s);
      }
    }
    // every lane read vec[perm[lane]] before any lane writes
    __builtin_amdgcn_wave_barrier();
    if (mine) vec[lane] = s;
  }
  __syncthreads();
}

// out = U (A_r^{-1} (U^T rhs)), the DMD solve of the initial guess
// (eq. dmd-ig) and of the preconditioner correction (eq. dmd-sa).  rhs, out:
// global vectors; cells with a stride of NT <= blockDim (the instance's own
// thread count, so the summation order does not depend on the launch).  Ends
// with a barrier, so `out` is visible to the whole workgroup afterwards.
//
// Loads go in batches: CPT cells of the thread (c, c + NT, ...) times KB1
// basis columns for U^T rhs, CPT cells times KB2 columns for the expansion,
// each batch in flight at once.  Every column's sum runs over the thread's
// cells in increasing order and every cell's expansion over the columns in
// order, whatever the batch shape, so the result does not depend on it.
// Inside a batch, columns past the rank re-read column rank - 1 (finite, and
// from cache): their sums are not used, and in the expansion they meet
// c_k = 0.  luS (LDS, RT_RMAX^2 doubles followed by
// RT_RMAX ints), when given: the factors and the permutation are loaded
// beside the first basis batch and staged there, so the substitution reads
// LDS instead of waiting on global loads (needs blockDim >= RT_RMAX^2 / 2).
template <int CPT = 1, int KB1 = 4, int KB2 = 5>
__device__ __forceinline__ void rom_apply(const RomDev &R, int rank, int ld, int nc, int NT, const double *rhs,
                                 double *out, double *red, double *vec, double *luS = nullptr) {
  static_assert(RT_RMAX % KB1 == 0 && RT_RMAX % KB2 == 0, "column batches tile the capacity");
  rank = __builtin_amdgcn_readfirstlane(rank);  // uniform: column addresses in scalar registers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const bool act = (int)threadIdx.x < NT;
  constexpr int NLU = RT_RMAX * RT_RMAX;
  double lu_pre[2] = {0.0, 0.0};
  int perm_pre = 0;
  if (luS) {  // uniform
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + h * (int)blockDim.x;
      if (e < NLU) lu_pre[h] = ldg(&R.LU[e]);
    }
    if ((int)threadIdx.x < RT_RMAX) perm_pre = R.perm[threadIdx.x];
  }
  double s[RT_RMAX];
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) s[k] = 0.0;
  for (int c0 = threadIdx.x; c0 < nc && act; c0 += CPT * NT) {
    double v[CPT];
    bool ok[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      ok[i] = c0 + i * NT < nc;
      v[i] = ok[i] ? ldg(&rhs[c0 + i * NT]) : 0.0;
    }
#pragma unroll
    for (int k0 = 0; k0 < RT_RMAX; k0 += KB1) {
      {
        // columns past the rank read the last column again (cached: no
        // further memory traffic) instead of branching between batches
        double u[CPT][KB1];
#pragma unroll
        for (int q = 0; q < KB1; ++q) {
          const double *col = R.U + (size_t)min(k0 + q, rank - 1) * ld + c0;
#pragma unroll
          for (int i = 0; i < CPT; ++i) u[i][q] = ok[i] ? ldg(&col[i * NT]) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < CPT; ++i)
          if (ok[i])
#pragma unroll
            for (int q = 0; q < KB1; ++q) s[k0 + q] = rt_fma(u[i][q], v[i], s[k0 + q]);
      }
    }
  }
#pragma unroll
  for (int k0 = 0; k0 < RT_RMAX; k0 += KB1)
    if (k0 < rank)
#pragma unroll
      for (int q = 0; q < KB1; ++q) {
        const double t = wave_sum_fast(s[k0 + q]);
        if (lane == 0) red[wave * RT_RMAX + k0 + q] = t;
      }
  int *permS = reinterpret_cast<int *>(luS + NLU);
  if (luS) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + h * (int)blockDim.x;
      if (e < NLU) luS[e] = lu_pre[h];
    }
    if ((int)threadIdx.x < RT_RMAX) permS[threadIdx.x] = perm_pre;
  }
  __syncthreads();
  if ((int)threadIdx.x < RT_RMAX) {
    double t = 0.0;
    if ((int)threadIdx.x < rank)
      for (int w = 0; w < nw; ++w) t += red[w * RT_RMAX + threadIdx.x];
    vec[threadIdx.x] = t;  // zero past the rank
  }
  __syncthreads();
  if (luS) lu_solve_wave(luS, permS, rank, vec);
  else lu_solve_wave(R.LU, R.perm, rank, vec);
  // expansion U c; the batches stay a loop to keep the caller's registers free
  for (int c0 = threadIdx.x; c0 < nc && act; c0 += CPT * NT) {
    bool ok[CPT];
    double acc[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      ok[i] = c0 + i * NT < nc;
      acc[i] = 0.0;
    }
#pragma unroll 1
    for (int k0 = 0; k0 < rank; k0 += KB2) {
      double u[CPT][KB2];
#pragma unroll
      for (int q = 0; q < KB2; ++q) {
        const double *col = R.U + (size_t)min(k0 + q, rank - 1) * ld + c0;  // c_k = 0 past the rank
#pragma unroll
        for (int i = 0; i < CPT; ++i) u[i][q] = ok[i] ? ldg(&col[i * NT]) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < KB2; ++q) {
        const double cq = vec[k0 + q];
#pragma unroll
        for (int i = 0; i < CPT; ++i) acc[i] = rt_fma(u[i][q], cq, acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (ok[i]) stg(&out[c0 + i * NT], acc[i]);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of the rows x cols core (rows <= cols <= RT_KC) held in
// sm.B (column major).  Each round applies cols/2 disjoint column rotations
// (round-robin pairing), one 16-lane group per pair with row-local DPP sums.
// Sweeps stop when a full sweep rotates nothing (|gamma| <= 1e-15
// sqrt(alpha beta)).  Leaves sorted singular values in sm.sv, left vectors
// (B_j / s_j) in sm.Uc and right vectors in sm.Vc.
// ---------------------------------------------------------------------------
__device__ inline void core_svd(RomSmem &sm, int rows, int cols) {
  const int tid = threadIdx.x;
  const int ncp = cols + (cols & 1);
  const int npairs = ncp >> 1;
  for (int e = tid; e < RT_KC * RT_KC; e += blockDim.x) {
    const int c = e / RT_KC, r = e % RT_KC;
    sm.V[e] = (c == r) ? 1.0 : 0.0;
    if (c >= cols || r >= rows) sm.B[e] = 0.0;
  }
  // pairing of round t, slot k (circle method: position 0 fixed, the rest rotate)
  for (int e = tid; e < (ncp - 1) * npairs; e += blockDim.x) {
    const int t = e / npairs, k0 = e % npairs, k1 = ncp - 1 - k0;
    int p = (k0 == 0) ? 0 : ((k0 - 1 + t) % (ncp - 1)) + 1;
    int q = ((k1 - 1 + t) % (ncp - 1)) + 1;
    if (p > q) {
      const int x = p;
      p = q;
      q = x;
    }
    sm.pairs[2 * e] = (short)p;
    sm.pairs[2 * e + 1] = (short)q;
  }
  __syncthreads();
  const int grp = tid >> 4, gl = tid & 15;
  const int i0 = gl, i1 = gl + 16;
  for (int sweep = 0; sweep < 60; ++sweep) {
    // flag bit 0: a rotation was applied; bit 1: some pair's cosine was
    // above 1e-12.  A sweep whose pairs were all below 1e-12 leaves them
    // below 1e-15 (quadratic convergence), so it is the last one.
    if (tid == 0) sm.flag = 0;
    __syncthreads();
    for (int round = 0; round < ncp - 1; ++round) {
      if (grp < npairs) {
        const int p = sm.pairs[2 * (round * npairs + grp)];
        const int q = sm.pairs[2 * (round * npairs + grp) + 1];
        double bp0 = 0, bq0 = 0, bp1 = 0, bq1 = 0;
        if (i0 < rows) {
          bp0 = sm.B[p * RT_KC + i0];
          bq0 = sm.B[q * RT_KC + i0];
        }
        if (i1 < rows) {
          bp1 = sm.B[p * RT_KC + i1];
          bq1 = sm.B[q * RT_KC + i1];
        }
        const double al = row16_sum(rt_fma(bp0, bp0, bp1 * bp1));
        const double be = row16_sum(rt_fma(bq0, bq0, bq1 * bq1));
        const double ga = row16_sum(rt_fma(bp0, bq0, bp1 * bq1));
        const double g2 = ga * ga, ab = al * be;
        if (ga != 0.0 && g2 > 1e-30 * ab) {
          // tangent of the rotation angle: any accurate-enough t gives a valid
          // rotation; c = (1 + t^2)^(-1/2) to full precision keeps c^2 + s^2 = 1
          const double zeta = (be - al) * rt_rcp(2.0 * ga);
          const double z2 = rt_fma(zeta, zeta, 1.0);
          double y = __builtin_amdgcn_rsq(z2);
          y = y * rt_fma(-0.5 * z2 * y, y, 1.5);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rt_rcp(fabs(zeta) + z2 * y);
          const double t2 = rt_fma(t, t, 1.0);
          double c = __builtin_amdgcn_rsq(t2);
          c = c * rt_fma(-0.5 * t2 * c, c, 1.5);  // two Newton steps for (1 + t^2)^(-1/2)
          c = c * rt_fma(-0.5 * t2 * c, c, 1.5);
          const double s = c * t;
          if (i0 < rows) {
            sm.B[p * RT_KC + i0] = c * bp0 - s * bq0;
            sm.B[q * RT_KC + i0] = s * bp0 + c * bq0;
          }
          if (i1 < rows) {
            sm.B[p * RT_KC + i1] = c * bp1 - s * bq1;
            sm.B[q * RT_KC + i1] = s * bp1 + c * bq1;
          }
          if (i0 < cols) {
            const double vp = sm.V[p * RT_KC + i0], vq = sm.V[q * RT_KC + i0];
            sm.V[p * RT_KC + i0] = c * vp - s * vq;
            sm.V[q * RT_KC + i0] = s * vp + c * vq;
          }
          if (i1 < cols) {
            const double vp = sm.V[p * RT_KC + i1], vq = sm.V[q * RT_KC + i1];
            sm.V[p * RT_KC + i1] = c * vp - s * vq;
            sm.V[q * RT_KC + i1] = s * vp + c * vq;
          }
          if (gl == 0) atomicOr(&sm.flag, g2 > 1e-24 * ab ? 3 : 1);
        }
      }
      __syncthreads();
    }
    const int more = sm.flag;
    __syncthreads();
    if (!(more & 2)) break;
  }
  // column norms and a stable descending rank order
  if (tid < cols) {
    double a = 0.0;
    for (int i = 0; i < rows; ++i) a = rt_fma(sm.B[tid * RT_KC + i], sm.B[tid * RT_KC + i], a);
    sm.nrm[tid] = sqrt(a);
  }
  __syncthreads();
  if (tid < cols) {
    const double mine = sm.nrm[tid];
    int rk = 0;
    for (int j = 0; j < cols; ++j) {
      const double o = sm.nrm[j];
      rk += (o > mine) || (o == mine && j < tid);
    }
    sm.perm[rk] = tid;
  }
  __syncthreads();
  for (int e = tid; e < cols * RT_KC; e += blockDim.x) {
    const int jj = e / RT_KC, i = e % RT_KC;
    const int j = sm.perm[jj];
    const double s = sm.nrm[j];
    if (i == 0) sm.sv[jj] = s;
    if (i < rows) sm.Uc[i * RT_KC + jj] = (s > 0.0) ? sm.B[j * RT_KC + i] / s : 0.0;
    if (i < cols) sm.Vc[i * RT_KC + jj] = sm.V[j * RT_KC + i];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Core SVD by the secular equation (rt_arrow.h) for K = [[diag S, a], [0, nu]]
// (rows = r + 1) or [diag S, a] (rows = r, rank-deficient snapshot).  Wave 0
// does the work, lane = root.  Leaves the same outputs as core_svd: singular
// values descending in sm.sv[0..rows), left vectors in sm.Uc, right vectors in
// sm.Vc (columns < rows).  Returns false (outputs untouched) when two
// singular values of S coincide to rounding or nu is at rounding level: the
// secular equation is then degenerate and the caller runs one-sided Jacobi.
// ---------------------------------------------------------------------------
__device__ inline bool core_svd_secular(RomSmem &sm, const double *S, const double *a, double nu, int r,
                                        int rows, int cols) {
  const int tid = threadIdx.x;
  // The secular problem, built by wave 0 with lane j on core row j: the same
  // problem arrow::build forms with its loop (deflation threshold from the
  // same serial sum, poles in ascending order, equal-pole test against the
  // next smaller retained pole).
  if (tid < 64) {
    const int j = tid;
    const double eps = 2.220446049250313e-16;
    double z2 = rows > r ? nu * nu : 0.0;
    for (int i = 0; i < r; ++i) z2 += a[i] * a[i];
    const double scale = fmax(r > 0 ? S[0] : 0.0, sqrt(z2));
    const double tolz = 8.0 * eps * scale;
    const bool in = j < r;
    const bool keep = in && !(fabs(a[j]) <= tolz);
    const unsigned long long km = __ballot(keep);
    const int base = rows > r ? 1 : 0;  // the nu row is pole 0
    const unsigned long long above = (j < 63) ? (km >> (j + 1)) : 0ull;
    bool clash = false;
    if (keep) {
      const int pos = base + __popcll(above);
      sm.ap.s[pos] = S[j];
      sm.ap.z[pos] = a[j];
      sm.ap.row[pos] = j;
      if (above) {
        const int jn = j + 1 + __builtin_ctzll(above);
        clash = S[j] - S[jn] <= 8.0 * eps * S[j];
      } else if (base) {
        clash = S[j] <= 8.0 * eps * S[j];
      }
    }
    if (in) sm.ap_defl[j] = !keep;
    const bool any_clash = __ballot(clash) != 0ull;
    if (j == 0) {
      if (base) {
        sm.ap.s[0] = 0.0;
        sm.ap.z[0] = nu;
        sm.ap.row[0] = r;
      }
      sm.ap.m = base + __popcll(km);
      sm.ap.rows = rows;
      sm.ap.cols = cols;
      sm.ap.scale = scale;
      sm.ap_ok = (rows == r || nu > tolz) && !any_clash;
    }
  }
  __syncthreads();
  if (!sm.ap_ok) return false;
  const arrow::Problem &P = sm.ap;
  const int m = P.m;
  // eight lanes per root (half a DPP row; roots 0..7 on wave 0, 8..15 on
  // wave 1, the rest on wave 2), each summing every eighth term of the
  // secular function
  if (tid < 8 * m) {
    const int kq = tid >> 3, g = tid & 7;
    int K;
    double tau;
    arrow::root_g<8>(P, kq, g, OctSum(), K, tau);
    if (g == 0) {
      sm.ap_K[kq] = K;
      sm.ap_tau[kq] = tau;
    }
  }
  __syncthreads();
  if (tid < m) sm.ap_zh[tid] = arrow::zhat(P, tid, sm.ap_K, sm.ap_tau);
  __syncthreads();
  // columns: secular roots (unsorted), then deflated rows (s_j, e_j, e_j);
  // B holds u, V holds v, nrm the singular values
  if (tid < m)
    sm.nrm[tid] = arrow::vectors(P, tid, sm.ap_K, sm.ap_tau, sm.ap_zh, r, &sm.B[tid * RT_KC], 1,
                                 &sm.V[tid * RT_KC], 1);
  if (tid < 64) {
    const bool d = tid < r && sm.ap_defl[tid];
    const unsigned long long dm = __ballot(d);
    if (d) {
      const int j = tid;
      const int c = m + __popcll(dm & ((1ull << j) - 1ull));
      for (int i = 0; i < rows; ++i) sm.B[c * RT_KC + i] = (i == j) ? 1.0 : 0.0;
      for (int i = 0; i < cols; ++i) sm.V[c * RT_KC + i] = (i == j) ? 1.0 : 0.0;
      sm.nrm[c] = S[j];
    }
  }
  __syncthreads();
  // descending order, ties by column
  if (tid < rows) {
    const double mine = sm.nrm[tid];
    int rk = 0;
    for (int j = 0; j < rows; ++j) {
      const double o = sm.nrm[j];
      rk += (o > mine) || (o == mine && j < tid);
    }
    sm.perm[rk] = tid;
  }
  __syncthreads();
  for (int e = tid; e < rows * RT_KC; e += blockDim.x) {
    const int jj = e / RT_KC, i = e % RT_KC;
    const int j = sm.perm[jj];
    if (i == 0) sm.sv[jj] = sm.nrm[j];
    if (i < rows) sm.Uc[i * RT_KC + jj] = sm.B[j * RT_KC + i];
    if (i < cols) sm.Vc[i * RT_KC + jj] = sm.V[j * RT_KC + i];
  }
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Incremental SVD, small dense part (App. B, eq. svd_core), one workgroup:
// sums the projection partials of the three grid passes in a fixed order,
// builds the core [[diag S, U^T x], [0, ||p||]] and Q^T [W b] (Q = [U, p/||p||]),
// takes the core SVD, truncates, forms M_new = Uc^T Q^T [W b] Vc and
// A_r = M_new S^{-1} with its LU, and leaves the basis rotation in R.pend for
// k_rom_update.  Returns 1 for a rank-deficient snapshot (x in span U), 0
// otherwise, -1 if x = 0 at rank 0 (nothing added).  rank / luok updated.
// ---------------------------------------------------------------------------
// DEFER_LU: leave the LU of A_r to isvd_lu (the order of the factorised
// matrix in sm.ibuf[2]), so that a caller can factorise while other
// workgroups rotate the basis; luok is then not touched.
template <bool COH, bool DEFER_LU = false>
__device__ inline int isvd_core(const RomDev &R, const RomWork &Wk, int rmax, int &rank, int &luok,
                                RomSmem &sm) {
  const int tid = threadIdx.x, NT = blockDim.x;
  const int r = Wk.r, nb = Wk.nblk;
  RomPend *P = R.pend;
  // fixed-order block sums: pass 1 -> a = U^T x, U^T b, x.x, x.b; pass 2 ->
  // a2 = U^T v, W^T v, v.v, v.b for the first residual v = x - U a.  The
  // second Gram-Schmidt step p = v - U a2 is applied by the rotation; its
  // norm and p.b follow from pass 2 (U^T v = a2, U^T U = I to rounding, and
  // a2 is at rounding level, so neither difference cancels):
  //   ||p||^2 = v.v - a2.a2,   p.b = v.b - a2 . U^T b
  sum_partials<COH>(Wk.part1, nb, 2 * RT_RMAX + 2, sm.red, sm.scratch);
  sum_partials<COH>(Wk.part2, nb, 2 * RT_RMAX + 2, sm.red + 2 * RT_RMAX + 2, sm.scratch);
  const double xn = sqrt(sm.red[2 * RT_RMAX]);
  const double xb = sm.red[2 * RT_RMAX + 1];
  double nu2 = sm.red[4 * RT_RMAX + 2], pb = sm.red[4 * RT_RMAX + 3];
  for (int j = 0; j < r; ++j) {
    const double a2 = sm.red[2 * RT_RMAX + 2 + j];
    nu2 = rt_fma(-a2, a2, nu2);
    pb = rt_fma(-a2, sm.red[RT_RMAX + j], pb);
  }
  const double nu = sqrt(fmax(nu2, 0.0));
  // a2 for the rotation, zero past the rank
  if (tid < RT_RMAX) stg(&P->a2[tid], tid < r ? sm.red[2 * RT_RMAX + 2 + tid] : 0.0);
  if (r == 0) {
    if (xn == 0.0) {
      if (tid == 0) {
        stg(&P->pending, 0);
        if constexpr (DEFER_LU) sm.ibuf[2] = 0;  // no LU to factor
      }
      __syncthreads();
      return -1;
    }
    if (tid == 0) {
      const double m = xb / xn;
      stg(&R.M[0], m);
      stg(&R.S[0], xn);
      sm.A[0] = m / xn;
      stg(&P->pending, 1);
      stg(&P->r_old, 0);
      stg(&P->rows, 1);
      stg(&P->k, 1);
      stg(&P->deficient, 0);
      stg(&P->inv_nu, 1.0 / xn);
      stg(&P->Uc[0], 1.0);
      stg(&P->Vc[0], 1.0);
      stg(&P->p, Wk.p);
      stg(&P->b, Wk.b);
    }
    __syncthreads();
    if constexpr (DEFER_LU) {
      if (tid == 0) sm.ibuf[2] = 1;
    } else {
      luok = !lu_factor_wave(sm.A, sm.perm, 1, R.LU, R.perm, &sm.ibuf[0], R.lu_tol);
    }
    rank = 1;
    return 0;
  }
  const int deficient = !(nu > 1e-12 * xn);
  const int rows = deficient ? r : r + 1, cols = r + 1;
  // stage M (r x r, global) in LDS once: the products below read it repeatedly
  double *Ms = sm.T1;  // free until the M_new products
  for (int e = tid; e < RT_RMAX * RT_RMAX; e += NT) Ms[e] = ldg(&R.M[e]);
  __syncthreads();
  // coefficient vectors: a (total), U^T b, a2, p^T W = p1^T W - a2^T M
  if (tid < RT_RMAX) {
    const int j = tid;
    sm.av[j] = (j < r) ? sm.red[j] + sm.red[2 * RT_RMAX + 2 + j] : 0.0;
    sm.utbv[j] = (j < r) ? sm.red[RT_RMAX + j] : 0.0;
    double v = 0.0;
    if (j < r) {
      v = sm.red[3 * RT_RMAX + 2 + j];
      for (int i = 0; i < r; ++i) v = rt_fma(-sm.red[2 * RT_RMAX + 2 + i], Ms[i * RT_RMAX + j], v);
    }
    sm.pwv[j] = v;
  }
  __syncthreads();
  // core K = [[diag S, a], [0, nu]] and Mx = Q^T [W b]
  for (int e = tid; e < RT_KC * RT_KC; e += NT) {
    const int j = e / RT_KC, i = e % RT_KC;  // K column j, row i
    double v = 0.0;
    if (j < r && i == j) v = ldg(&R.S[j]);
    if (j == r && i < r) v = sm.av[i];
    if (j == r && i == r && !deficient) v = nu;
    sm.B[e] = (i < rows && j < cols) ? v : 0.0;
    const int mi = e / RT_KC, mj = e % RT_KC;  // Mx row mi, column mj
    double m = 0.0;
    if (mi < r && mj < r) m = Ms[mi * RT_RMAX + mj];
    else if (mi < r && mj == r) m = sm.utbv[mi];
    else if (mi == r && mj < r && !deficient) m = sm.pwv[mj] / nu;
    else if (mi == r && mj == r && !deficient) m = pb / nu;
    sm.Mx[e] = m;
  }
  __syncthreads();
  // S and a as the secular path reads them (LDS); B above is Jacobi's input
  if (tid < RT_RMAX) sm.a2v[tid] = tid < r ? ldg(&R.S[tid]) : 0.0;
  __syncthreads();
  if (!core_svd_secular(sm, sm.a2v, sm.av, nu, r, rows, cols)) core_svd(sm, rows, cols);
  if (tid == 0) {
    int k = rows;
    if (Wk.truncate) {
      double tot = 0.0;
      for (int i = 0; i < rows; ++i) tot += sm.sv[i];
      int kk = 0;
      for (int i = 0; i < rows; ++i)
        if (sm.sv[i] / tot > Wk.eps) kk = i + 1;
      k = kk > 0 ? kk : 1;
    }
    if (k > rmax) k = rmax;
    sm.ibuf[1] = k;
  }
  __syncthreads();
  const int k = sm.ibuf[1];
  // M_new = Uc[:, :k]^T Mx Vc[:, :k], A_r = M_new S^{-1}; pending rotation
  for (int e = tid; e < rows * k; e += NT) {
    const int i = e / k, j = e % k;
    double v = 0.0;
    for (int q = 0; q < cols; ++q) v = rt_fma(sm.Mx[i * RT_KC + q], sm.Vc[q * RT_KC + j], v);
    sm.T1[i * RT_KC + j] = v;
  }
  // the rotation for k_rom_update, zero outside rows x k (left) and cols x k
  // (right): that kernel multiplies over the full capacity
  for (int e = tid; e < RT_KC * RT_KC; e += NT) {
    const int i = e / RT_KC, j = e % RT_KC;
    stg(&P->Uc[e], (i < rows && j < k) ? sm.Uc[e] : 0.0);
    stg(&P->Vc[e], (i < cols && j < k) ? sm.Vc[e] : 0.0);
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    double v = 0.0;
    for (int q = 0; q < rows; ++q) v = rt_fma(sm.Uc[q * RT_KC + i], sm.T1[q * RT_KC + j], v);
    stg(&R.M[i * RT_RMAX + j], v);
    sm.A[i * RT_KC + j] = v / sm.sv[j];
  }
  if (tid == 0) {
    for (int j = 0; j < k; ++j) stg(&R.S[j], sm.sv[j]);
    stg(&P->pending, 1);
    stg(&P->r_old, r);
    stg(&P->rows, rows);
    stg(&P->k, k);
    stg(&P->deficient, deficient);
    stg(&P->inv_nu, deficient ? 0.0 : 1.0 / nu);
    stg(&P->p, Wk.p);
    stg(&P->b, Wk.b);
  }
  __syncthreads();
  if constexpr (DEFER_LU) {
    if (tid == 0) sm.ibuf[2] = k;
  } else {
    luok = !lu_factor_wave(sm.A, sm.perm, k, R.LU, R.perm, &sm.ibuf[0], R.lu_tol);
  }
  rank = k;
  return deficient;
}

// The LU of A_r that isvd_core<., true> left in sm; returns luok, or -1
// when the core factored nothing (an empty ROM met a zero snapshot).
__device__ inline int isvd_lu(const RomDev &R, RomSmem &sm) {
  __syncthreads();
  const int n = sm.ibuf[2];
  if (n == 0) return -1;  // uniform
  return !lu_factor_wave(sm.A, sm.perm, n, R.LU, R.perm, &sm.ibuf[0], R.lu_tol);
}

// p = v - U a2 for one cell from its old basis row (the second Gram-Schmidt
// step, in the order the passes use).  a2: LDS or constant-space pointer.
template <typename CP>
__device__ __forceinline__ double second_residual(double v, const double (&old)[RT_RMAX], CP a2) {
#pragma unroll
  for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(-old[k], a2[k], v);
  return v;
}

// Second half: U <- [U, p/nu] Uc[:, :k] (or W <- [W, b] Vc[:, :k]) for the
// cells c[0..NCELL) of one thread, given their old rows; works in place.  The
// coefficients Cc (stride RT_KC, at least RT_KC * RT_KC + 4 entries) are zero
// outside the core, and the old basis entries past r are masked, so every
// product runs over the full capacity without branches.  Cc is either LDS
// (each read serves NCELL cells) or the constant address space (uniform
// addresses: scalar loads, the products take them as scalar operands); the
// outputs go in blocks of JB columns, which bounds the registers the
// coefficients take.
template <int NCELL, typename CP, int JB = 4>
__device__ __forceinline__ void rotate_block(const double (&old)[NCELL][RT_RMAX], const double (&e)[NCELL], CP Cc,
                                             int r, int k, double *X, int ld, const int (&c)[NCELL],
                                             const bool (&ok)[NCELL]) {
#pragma unroll 1
  for (int j0 = 0; j0 < k; j0 += JB) {
    double acc[NCELL][JB];
#pragma unroll
    for (int i = 0; i < NCELL; ++i)
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) acc[i][jj] = 0.0;
#pragma unroll
    for (int q = 0; q < RT_RMAX; ++q)
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const double cf = Cc[q * RT_KC + j0 + jj];
#pragma unroll
        for (int i = 0; i < NCELL; ++i) acc[i][jj] = rt_fma(old[i][q], cf, acc[i][jj]);
      }
    // row r: the new direction (p / nu for U, b for W)
#pragma unroll
    for (int jj = 0; jj < JB; ++jj) {
      const double cf = Cc[r * RT_KC + j0 + jj];
#pragma unroll
      for (int i = 0; i < NCELL; ++i) acc[i][jj] = rt_fma(e[i], cf, acc[i][jj]);
    }
#pragma unroll
    for (int i = 0; i < NCELL; ++i)
      if (ok[i])
#pragma unroll
        for (int jj = 0; jj < JB; ++jj)
          if (j0 + jj < k) stg(&X[(size_t)(j0 + jj) * ld + c[i]], acc[i][jj]);
  }
}


// Cells per thread of the fused post's rotation (rom_rotate_own_lu).  Each
// coefficient read from LDS there is a wave-wide broadcast serving this many
// cells of a thread: the LDS return bandwidth, not the FMAs, bounds the loop,
// so the cells per read go as high as the registers allow (one output column
// at a time).
constexpr int ROT_CELLS = 3;

// The fused post's last stage after rom_core<., true>: the reduced
// operator's LU and the pending rotation of both bases at once, by the
// workgroup whose core just decided it.  The rotation record was written by
// this workgroup in this launch, so it is read with vector loads and the
// coefficients staged in LDS (sm.Mx, sm.T1, sm.av: free once the core is
// done).  Wave 0
// factors (lu_factor_rows) while the other waves start rotating; the cells
// are handed out in chunks of 64 * ROT_CELLS (U's chunks, then W's) through
// an LDS counter, so wave 0 takes what is left once its LU is done.  A cell's
// arithmetic does not depend on which wave rotates it.  Ends with the LU flag
// written to the state (z: 0 IG, 1 PC).
__device__ inline void rom_rotate_own_lu(const Inst &I, const RomDev &R, const RomWork &W, RomSmem &sm, int z) {
  const RomPend *P = R.pend;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NT = blockDim.x;
  __syncthreads();  // the core's results (sm.A, sm.ibuf[2], the rotation record) are complete
  const int n_lu = sm.ibuf[2];
  const int pending = xload(&P->pending);  // uniform
  int r = 0, k = 0, nchunk = 0;
  double inv_nu = 0.0;
  if (pending) {
    r = xload(&P->r_old);
    k = xload(&P->k);
    inv_nu = xload(&P->inv_nu);
    for (int e = threadIdx.x; e < RT_KC * RT_KC; e += NT) {
      sm.Mx[e] = ldg(&P->Uc[e]);
      sm.T1[e] = ldg(&P->Vc[e]);
    }
    if (threadIdx.x < RT_RMAX) sm.av[threadIdx.x] = ldg(&P->a2[threadIdx.x]);
    nchunk = (I.nc + 64 * ROT_CELLS - 1) / (64 * ROT_CELLS);
  }
  if (threadIdx.x == 0) sm.ibuf[3] = 0;
  __syncthreads();
  if (wave == 0 && n_lu > 0) {
    const int bad = lu_factor_rows(sm.A, n_lu, R.LU, R.perm, R.lu_tol);
    if (lane == 0) sm.ibuf[0] = bad;
  }
  const int nc = I.nc, ld = I.ld;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(&sm.ibuf[3], 1);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= 2 * nchunk) break;
    const int mat = t >= nchunk;
    const int cb = (t - mat * nchunk) * 64 * ROT_CELLS + lane;
    const double *cc = mat ? sm.T1 : sm.Mx;
    double *X = mat ? R.W : R.U;
    int cv[ROT_CELLS];
    bool ok[ROT_CELLS];
    double old[ROT_CELLS][RT_RMAX], e[ROT_CELLS];
#pragma unroll
    for (int i = 0; i < ROT_CELLS; ++i) {
      cv[i] = cb + 64 * i;
      ok[i] = cv[i] < nc;
      const int cl = ok[i] ? cv[i] : nc - 1;
#pragma unroll
      for (int q = 0; q < RT_RMAX; ++q) old[i][q] = q < r ? ldg(&X[(size_t)q * ld + cl]) : 0.0;
      e[i] = mat ? ldg(&W.b[cl]) : second_residual(ldg(&W.p[cl]), old[i], sm.av) * inv_nu;
    }
    rotate_block<ROT_CELLS, const double *, 1>(old, e, cc, r, k, X, ld, cv, ok);
  }
  __syncthreads();
  if (threadIdx.x == 0 && n_lu > 0) {
    const int luok = !sm.ibuf[0];
    *rom_luok_of(I.st, z) = luok;
  }
}

// ---------------------------------------------------------------------------
// Per-thread partial sums of ||rho^n||^2, ||rho^(0) - rho^n||^2 and
// ||dpc - (rho^n - rho^(1/2))||^2 (the error indicators of Sec. 3.2) over
// cells c0, c0 + stride, ...
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rom_norm_parts(const Inst &I, int c0, int stride, double (&part)[3 + RT_XLEV]) {
#pragma unroll
  for (int k = 0; k < 3 + RT_XLEV; ++k) part[k] = 0.0;
  const int used = I.nlev > 1 ? I.st->used_mask : 0;
  for (int c = c0; c < I.nc; c += stride) {
    const double r = I.rho[c];
    part[0] = rt_fma(r, r, part[0]);
    const double e1 = I.rho0[c] - r;
    part[1] = rt_fma(e1, e1, part[1]);
    const double e2 = I.dpc[c] - (r - I.rhalf[c]);
    part[2] = rt_fma(e2, e2, part[2]);
    // correction ROMs of iterations l >= 2 that applied: ||dlev - (rho^n - y_l)||^2
#pragma unroll
    for (int k = 0; k < RT_XLEV; ++k)
      if ((used >> (k + 1)) & 1) {
        const double e = I.dlev[k][c] - (r - I.ylev[k][c]);
        part[3 + k] = rt_fma(e, e, part[3 + k]);
      }
  }
}

// ---------------------------------------------------------------------------
// Alg. 2's decisions for a ROM instance from the error indicators (Sec. 3.2,
// normalised by ||rho^n||_2): which ROM takes a snapshot this step and
// whether it is truncated.  vec holds ||rho^n||^2, ||rho^(0) - rho^n||^2 and
// ||dpc - (rho^n - rho^(1/2))||^2 (read only when the IG ROM exists).  Pure:
// the workgroups of a cooperative launch call it on identical data.
// ---------------------------------------------------------------------------
struct RomPlan {
  int ig_on, ig_trunc, pc_on, pc_trunc;
  double e_ig, e_pc;
  int lv_on[RT_XLEV], lv_trunc[RT_XLEV];  // correction ROMs of iterations 2..nlev
};
__device__ __forceinline__ RomPlan rom_plan(const Inst &I, int flag_ig, int flag_pc, int used_pc, int iters,
                                            const double *vec) {
  RomPlan P{0, 0, 0, 0, -1.0, -1.0, {0}, {0}};
  const double rn = flag_ig ? sqrt(vec[0]) : 0.0;
  const double scale = (I.abs_up || rn == 0.0) ? 1.0 : 1.0 / rn;
  if (!flag_ig) {
    P.ig_on = 1;  // phase 1: untruncated snapshot (rho^n, b~^{n-1})
  } else {
    P.e_ig = sqrt(vec[1]) * scale;
    P.ig_on = P.ig_trunc = P.e_ig > I.eps_up;
    if (iters > 1) {  // no correction snapshot when the step converged at l = 1
      if (!flag_pc) {
        P.pc_on = 1;
      } else {
        if (used_pc) P.e_pc = sqrt(vec[2]) * scale;
        P.pc_on = P.pc_trunc = P.ig_on || !used_pc || P.e_pc > I.eps_up;
      }
    }
  }
  return P;
}

// The correction ROMs of iterations l = 2..nlev, after rom_plan decided the
// initial guess and iteration 1: level l takes the pair of its iteration
// (rho^n - rho^{(l-1/2)}, rho^{(l-1/2)} - rho^{(l-1)}) only once every level
// below it was complete when the step started and the step needed more than
// l iterations; while under construction every such pair is added
// untruncated, afterwards (truncated) when a ROM below it was updated in
// this step, when it could not apply its correction, or when its indicator
// ||dlev - (rho^n - rho^{(l-1/2)})|| / ||rho^n|| exceeds eps_UP.  vec[3 + l - 2]
// holds that indicator's square; used_mask bit l - 1 says level l applied.
__device__ __forceinline__ void rom_plan_levels(const Inst &I, const RtState *st, int flag_pc, int used_mask,
                                                int iters, const double *vec, RomPlan &P) {
  if (P.e_ig < 0.0) return;  // the initial-guess ROM is still being built
  const double rn = sqrt(vec[0]);
  const double scale = (I.abs_up || rn == 0.0) ? 1.0 : 1.0 / rn;
  int lower = P.ig_on || P.pc_on;
  int below_done = flag_pc;
  for (int l = 2; l <= I.nlev; ++l) {
    const int k = l - 2;
    if (!below_done || iters <= l) break;
    // mixed precision: no pair from an FP32-refined iterate of level l
    if (I.precision == RT_MIXED && !((used_mask >> (8 + k)) & 1)) break;
    const int done = st->flag_pl[k];
    if (!done) {
      P.lv_on[k] = 1;
    } else {
      const int used = (used_mask >> (l - 1)) & 1;
      const double e = used ? sqrt(vec[3 + k]) * scale : -1.0;
      P.lv_on[k] = P.lv_trunc[k] = lower || !used || e > I.eps_up;
    }
    lower |= P.lv_on[k];
    below_done = done;
  }
}

// What the end-of-step bookkeeping needs about the step just solved and the
// state's counters as they were when it started.  The slab SI kernel fills it
// from registers (no reloads of what it just wrote); step_in() reads it back
// from the state for kernels that run after the solve.
struct StepIn {
  int iters, conv, used_pc, ig_fb, pc_fb, phase, cur;
  int flag_ig, flag_pc, rank_ig, rank_pc, nonconv, fallbacks;
  double residual;
  long long steps, si_total, sweeps_total;
  int used_mask = 0;  // correction ROMs applied (bit l - 1: level l), levels >= 2
  int lv_fb = 0;      // levels >= 2 that were due but could not apply (singular)
};
__device__ inline StepIn step_in(const RtState *st) {
  return {st->iters,   st->conv,    st->used_pc, st->ig_fb,   st->pc_fb,    st->phase,    st->cur,
          st->flag_ig, st->flag_pc, st->rank_ig, st->rank_pc, st->nonconv, st->fallbacks, st->residual,
          st->steps,   st->si_total, st->sweeps_total, st->used_mask, st->lv_fb};
}

// ---------------------------------------------------------------------------
// End-of-step bookkeeping and, for the ROM method, the decisions of rom_plan
// written to the ROMs' work records.  vec: as for rom_plan; nb is the number
// of pass blocks the ROM work will use.  Called by every thread of one
// workgroup after the step's state is final; thread 0 writes.
// ---------------------------------------------------------------------------
__device__ inline void rom_decide(const Inst &I, const double *vec, int nb, const StepIn &S) {
  RtState *st = I.st;
  const int iters = S.iters;
  const long long step_no = S.steps + 1;
  double e_ig = -1.0, e_pc = -1.0;
  if (I.method == RT_ROM) {
    // the backward-Euler start of a BDF2 march solves with another operator
    // and is not a snapshot
    const bool start = I.bdf2 && S.steps == 0;
    RomPlan P = start ? RomPlan{0, 0, 0, 0, -1.0, -1.0, {0}, {0}} : rom_plan(I, S.flag_ig, S.flag_pc, S.used_pc, iters, vec);
    if (!start && I.nlev > 1) rom_plan_levels(I, st, S.flag_pc, S.used_mask, iters, vec, P);
    e_ig = P.e_ig;
    e_pc = P.e_pc;
    if (threadIdx.x == 0) {
      RomWork &wi = *I.ig.work;
      wi.active = P.ig_on;
      wi.truncate = P.ig_trunc;
      wi.r = S.rank_ig;
      wi.nblk = nb;
      wi.step_no = step_no;
      wi.eps = I.eps_ig;
      wi.x = I.rho;
      wi.b = I.bt2[S.cur];
      // its own row: the cooperative SI kernel stores the PC right-hand side
      // in row 0 with plain stores (cached per XCD) and this residual with
      // agent-scope stores in the same launch, and the two must not share
      // addresses
      wi.p = I.work + 4 * (size_t)I.nc;
      RomWork &wp = *I.pc.work;
      wp.active = P.pc_on;
      wp.truncate = P.pc_trunc;
      wp.r = S.rank_pc;
      wp.nblk = nb;
      wp.step_no = step_no;
      wp.eps = I.eps_pc;
      // correction snapshots (eq. correction_snapshot), formed by pass 1
      wp.x = I.work + 2 * (size_t)I.nc;
      wp.b = I.work + 3 * (size_t)I.nc;
      wp.p = I.work + I.nc;
      I.ig.pend->pending = 0;
      I.pc.pend->pending = 0;
      for (int k = 0; k + 2 <= I.nlev; ++k) {
        RomWork &wl = *I.pl[k].work;
        wl.active = P.lv_on[k];
        wl.truncate = P.lv_trunc[k];
        wl.r = st->rank_pl[k];
        wl.nblk = nb;
        wl.step_no = step_no;
        wl.eps = I.eps_pc;
        wl.x = I.wlev[k];
        wl.b = I.wlev[k] + I.nc;
        wl.p = I.wlev[k] + 2 * (size_t)I.nc;
        I.pl[k].pend->pending = 0;
      }
    }
  }
  if (threadIdx.x == 0) {
    const int fb = S.ig_fb + S.pc_fb + S.lv_fb;
    if (I.hist && step_no <= I.hist_cap) {
      RtStepRec &rec = I.hist[step_no - 1];
      rec.iters = iters;
      rec.phase = S.phase;
      rec.converged = S.conv;
      rec.ig_update = 0;
      rec.pc_update = 0;
      rec.rank_ig = S.rank_ig;
      rec.rank_pc = S.rank_pc;
      rec.fallback = fb > 0;
      rec.e_ig = e_ig;
      rec.e_pc = e_pc;
      rec.residual = S.residual;
    }
    st->fallbacks = S.fallbacks + fb;
    st->steps = step_no;
    st->si_total = S.si_total + iters;
    st->sweeps_total = S.sweeps_total + iters + 2;
    st->nonconv = S.nonconv + !S.conv;
  }
}

// s_r / sum(s) of the retained values (eq. ig_stop, eq. pc_stop)
__device__ inline double rom_tail_ratio(const RomDev &R, int rank) {
  double tot = 0.0;
  for (int i = 0; i < rank; ++i) tot += ldg(&R.S[i]);
  return tot > 0.0 ? ldg(&R.S[rank - 1]) / tot : 0.0;
}


// ---------------------------------------------------------------------------
// Projection passes (classical Gram-Schmidt applied twice).  Block b of nb
// takes cells b*blockDim + t, strided by nb*blockDim, and writes its partial
// sums to row b; later stages add the rows in block order.  The same bodies
// serve the grid kernels (grid (blocks, instance, ROM)) and the one-block
// fused post of small instances (nb = 1).  COH: the partial rows are written
// and read with agent-scope atomics (workgroups of one cooperative launch on
// different XCDs exchange them).
// ---------------------------------------------------------------------------
template <bool COH>
__device__ __forceinline__ void rom_pass1(const Inst &I, const RomDev &R, const RomWork &W, int z, int b,
                                          int nb, double *red, double *out) {
  const int r = W.r, ld = I.ld, NT = blockDim.x;
  double part[2 * RT_RMAX + 2];
#pragma unroll
  for (int k = 0; k < 2 * RT_RMAX + 2; ++k) part[k] = 0.0;
#pragma unroll 2
  for (int c = b * NT + threadIdx.x; c < I.nc; c += nb * NT) {
    double xv, bv;
    if (z >= 1) {  // x = rho^n - rho^(l-1/2), b = rho^(l-1/2) - rho^(l-1) (l = z)
      const double rh = z == 1 ? ldg(&I.rhalf[c]) : ldg(&I.ylev[z - 2][c]);
      xv = ldg(&I.rho[c]) - rh;
      bv = rh - (z == 1 ? ldg(&I.rho0[c]) : ldg(&I.rlev[z - 2][c]));
      // the PC ROM's x, b live in the work arrays (COH: read later by
      // workgroups on other XCDs)
      part_store<COH>(const_cast<double *>(W.x) + c, xv);
      part_store<COH>(const_cast<double *>(W.b) + c, bv);
    } else {
      xv = ldg(&W.x[c]);
      bv = ldg(&W.b[c]);
    }
    part[2 * RT_RMAX] = rt_fma(xv, xv, part[2 * RT_RMAX]);
    part[2 * RT_RMAX + 1] = rt_fma(xv, bv, part[2 * RT_RMAX + 1]);
    // basis columns up to the rank only (uniform branches: the loads are
    // still in flight together); the sums past the rank stay zero
    double u[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) u[k] = k < r ? ldg(&R.U[(size_t)k * ld + c]) : 0.0;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      part[k] = rt_fma(u[k], xv, part[k]);
      part[RT_RMAX + k] = rt_fma(u[k], bv, part[RT_RMAX + k]);
    }
  }
  wg_sum_fast<2 * RT_RMAX + 2>(part, red, out);
  if (threadIdx.x < 2 * RT_RMAX + 2) part_store<COH>(&W.part1[b * RT_NPART + threadIdx.x], out[threadIdx.x]);
}

template <bool COH>
__device__ __forceinline__ void rom_pass2(const Inst &I, const RomDev &R, const RomWork &W, int b, int nb,
                                          double *red, double *out, double *av, double *scratch) {
  const int r = W.r, ld = I.ld, NT = blockDim.x;
  // every column: pass 1 left zero sums past the rank, so av is zero there
  sum_partials<COH>(W.part1, nb, RT_RMAX, av, scratch);
  double part[2 * RT_RMAX + 2];
#pragma unroll
  for (int k = 0; k < 2 * RT_RMAX + 2; ++k) part[k] = 0.0;
#pragma unroll 2
  for (int c = b * NT + threadIdx.x; c < I.nc; c += nb * NT) {
    // loads up to the rank, issued up front; the arithmetic keeps its order
    double u[RT_RMAX], wv[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      u[k] = k < r ? ldg(&R.U[(size_t)k * ld + c]) : 0.0;
      wv[k] = k < r ? ldg(&R.W[(size_t)k * ld + c]) : 0.0;
    }
    double v = part_load<COH>(W.x + c);
    const double bv = part_load<COH>(W.b + c);
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(-u[k], av[k], v);
    part_store<COH>(W.p + c, v);  // first Gram-Schmidt residual; the rotation subtracts U a2
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      part[k] = rt_fma(u[k], v, part[k]);
      part[RT_RMAX + k] = rt_fma(wv[k], v, part[RT_RMAX + k]);
    }
    part[2 * RT_RMAX] = rt_fma(v, v, part[2 * RT_RMAX]);
    part[2 * RT_RMAX + 1] = rt_fma(v, bv, part[2 * RT_RMAX + 1]);
  }
  wg_sum_fast<2 * RT_RMAX + 2>(part, red, out);
  if (threadIdx.x < 2 * RT_RMAX + 2) part_store<COH>(&W.part2[b * RT_NPART + threadIdx.x], out[threadIdx.x]);
}


// ---------------------------------------------------------------------------
// Small dense part of the update (isvd_core) and Alg. 2's phase flags for
// ROM z of one instance; every thread of the workgroup calls it.  Block z
// writes only ROM z's state fields, so the two ROMs' workgroups may run at
// once.
// ---------------------------------------------------------------------------
template <bool COH, bool DEFER_LU = false>
__device__ __forceinline__ void rom_core(const Inst &I, const RomDev &R, const RomWork &W, int z, RomSmem &sm) {
  RtState *st = I.st;
  int rank = *rom_rank_of(st, z);
  int luok = *rom_luok_of(st, z);
  const int dfc = isvd_core<COH, DEFER_LU>(R, W, I.r_max, rank, luok, sm);
  if (threadIdx.x == 0) {
    const long long step_no = W.step_no;
    int updated = 0;
    if (!W.truncate) {
      // construction phase: stop tests eq. ig_stop / eq. pc_stop, the rank
      // cap, or a rank-deficient snapshot end it
      if (dfc >= 0) {
        updated = 1;
        if (rom_tail_ratio(R, rank) <= W.eps || rank >= I.r_max || dfc == 1) {
          if (z == 0) {
            st->flag_ig = 1;
            st->n0 = (int)step_no;
          } else if (z == 1) {
            // PC snapshots start only after the IG construction ended in an
            // earlier step, so n0 is settled here
            st->flag_pc = 1;
            st->n1 = (int)step_no - st->n0;
          } else {
            // level z collects only after the levels below it completed
            int prior = st->n0 + st->n1;
            for (int k = 0; k < z - 2; ++k) prior += st->n_pl[k];
            st->flag_pl[z - 2] = 1;
            st->n_pl[z - 2] = (int)step_no - prior;
          }
        }
      }
    } else {
      updated = 1;
    }
    *rom_rank_of(st, z) = rank;
    if (!DEFER_LU) *rom_luok_of(st, z) = luok;
    if (z == 0) st->ig_updates += updated;
    else if (z == 1) st->pc_updates += updated;
    else st->upd_pl[z - 2] += updated;
    if (I.hist && step_no <= I.hist_cap) {
      RtStepRec &rec = I.hist[step_no - 1];
      if (z == 0) {
        rec.ig_update = updated;
        rec.rank_ig = rank;
      } else if (z == 1) {
        rec.pc_update = updated;
        rec.rank_pc = rank;
      }
    }
  }
}

// The deferred LU of rom_core<., true> and its flag (every thread calls).
__device__ __forceinline__ void rom_core_lu(const Inst &I, const RomDev &R, int z, RomSmem &sm) {
  const int luok = isvd_lu(R, sm);
  if (threadIdx.x == 0 && luok >= 0) *rom_luok_of(I.st, z) = luok;
}
