// rt_rom.hip -- the per-step ROM work of Alg. 2 for every instance of a
// launch (slab or plane): error indicators and decisions, the incremental-SVD
// updates (App. B) split into grid-wide projection passes, a one-workgroup
// small dense core per ROM, and the grid-wide basis rotation.
#include "rt_common.h"
#include "rt_rom.h"

namespace {
constexpr int BLK = 256;  // threads per block of the grid passes

// One cell per thread up to 64 blocks an instance (rt_pass_blocks): the
// passes are short and latency-bound, so an instance's cells are spread wide.
__device__ __host__ __forceinline__ int pass_blocks(int nc) { return rt_pass_blocks(nc); }

__device__ __forceinline__ const RomDev &rom_of(const Inst &I, int z) { return z ? I.pc : I.ig; }
}  // namespace

// ---------------------------------------------------------------------------
// k_rom_norms: per-block partial sums of ||rho^n||^2, ||rho^(0) - rho^n||^2
// and ||dpc - (rho^n - rho^(1/2))||^2 for the error indicators of Sec. 3.2,
// grid (blocks of BLK cells, instance).  Written to the IG ROM's third
// partial buffer, which k_rom_pass3 reuses only after k_rom_decide.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLK) k_rom_norms(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || !I.st->flag_ig) return;
  const int nb = pass_blocks(I.nc);
  if ((int)blockIdx.x >= nb) return;
  __shared__ double red[(BLK / 64) * 3], out[3];
  double part[3];
  rom_norm_parts(I, blockIdx.x * BLK + threadIdx.x, nb * BLK, part);
  wg_sum_fast<3>(part, red, out);
  if (threadIdx.x < 3) I.ig.work->part3[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}

// ---------------------------------------------------------------------------
// k_rom_decide: rom_decide (step bookkeeping, error indicators and Alg. 2's
// decisions) for every instance, one workgroup each, from the partial sums
// of k_rom_norms.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rom_decide(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  __shared__ double scratch[256], vec[4];
  const int nb = pass_blocks(I.nc);
  if (I.method == RT_ROM && I.st->flag_ig) sum_partials(I.ig.work->part3, nb, 3, vec, scratch);
  rom_decide(I, vec, I.post_nb);
}

// ---------------------------------------------------------------------------
// Projection passes (classical Gram-Schmidt applied twice).  Block b of nb
// takes cells b*blockDim + t, strided by nb*blockDim, and writes its partial
// sums to row b; later stages add the rows in block order.  The same bodies
// serve the grid kernels (grid (blocks, instance, ROM)) and the one-block
// fused post of small instances (nb = 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rom_pass1(const Inst &I, const RomDev &R, const RomWork &W, int z, int b,
                                          int nb, double *red, double *out) {
  const int r = W.r, ld = I.ld, NT = blockDim.x;
  double part[2 * RT_RMAX + 2];
#pragma unroll
  for (int k = 0; k < 2 * RT_RMAX + 2; ++k) part[k] = 0.0;
  for (int c = b * NT + threadIdx.x; c < I.nc; c += nb * NT) {
    double xv, bv;
    if (z == 1) {  // x = rho^n - rho^(1/2), b = rho^(1/2) - rho^(0)
      const double rh = I.rhalf[c];
      xv = I.rho[c] - rh;
      bv = rh - I.rho0[c];
      const_cast<double *>(W.x)[c] = xv;  // the PC ROM's x, b live in the work arrays
      const_cast<double *>(W.b)[c] = bv;
    } else {
      xv = W.x[c];
      bv = W.b[c];
    }
    part[2 * RT_RMAX] = rt_fma(xv, xv, part[2 * RT_RMAX]);
    part[2 * RT_RMAX + 1] = rt_fma(xv, bv, part[2 * RT_RMAX + 1]);
    // all basis loads unconditional (finite columns past the rank, masked),
    // so they are in flight together; the sums past the rank stay zero
    double u[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      const double v = R.U[(size_t)k * ld + c];
      u[k] = k < r ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      part[k] = rt_fma(u[k], xv, part[k]);
      part[RT_RMAX + k] = rt_fma(u[k], bv, part[RT_RMAX + k]);
    }
  }
  wg_sum_fast<2 * RT_RMAX + 2>(part, red, out);
  if (threadIdx.x < 2 * RT_RMAX + 2) W.part1[b * RT_NPART + threadIdx.x] = out[threadIdx.x];
}

__device__ __forceinline__ void rom_pass2(const Inst &I, const RomDev &R, const RomWork &W, int b, int nb,
                                          double *red, double *out, double *av, double *scratch) {
  const int r = W.r, ld = I.ld, NT = blockDim.x;
  // every column: pass 1 left zero sums past the rank, so av is zero there
  sum_partials(W.part1, nb, RT_RMAX, av, scratch);
  double part[2 * RT_RMAX];
#pragma unroll
  for (int k = 0; k < 2 * RT_RMAX; ++k) part[k] = 0.0;
  for (int c = b * NT + threadIdx.x; c < I.nc; c += nb * NT) {
    // all loads issued up front and unconditionally (masked past the rank);
    // the arithmetic keeps its order
    double u[RT_RMAX], wv[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      const double x = R.U[(size_t)k * ld + c], y = R.W[(size_t)k * ld + c];
      u[k] = k < r ? x : 0.0;
      wv[k] = k < r ? y : 0.0;
    }
    double v = W.x[c];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(-u[k], av[k], v);
    W.p[c] = v;
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      part[k] = rt_fma(u[k], v, part[k]);
      part[RT_RMAX + k] = rt_fma(wv[k], v, part[RT_RMAX + k]);
    }
  }
  wg_sum_fast<2 * RT_RMAX>(part, red, out);
  if (threadIdx.x < 2 * RT_RMAX) W.part2[b * RT_NPART + threadIdx.x] = out[threadIdx.x];
}

__device__ __forceinline__ void rom_pass3(const Inst &I, const RomDev &R, const RomWork &W, int b, int nb,
                                          double *red, double *out, double *a2, double *scratch) {
  const int r = W.r, ld = I.ld, NT = blockDim.x;
  sum_partials(W.part2, nb, RT_RMAX, a2, scratch);  // zero past the rank
  double part[2] = {0.0, 0.0};
  for (int c = b * NT + threadIdx.x; c < I.nc; c += nb * NT) {
    double u[RT_RMAX];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) {
      const double x = R.U[(size_t)k * ld + c];
      u[k] = k < r ? x : 0.0;
    }
    double v = W.p[c];
#pragma unroll
    for (int k = 0; k < RT_RMAX; ++k) v = rt_fma(-u[k], a2[k], v);
    W.p[c] = v;
    part[0] = rt_fma(v, v, part[0]);
    part[1] = rt_fma(v, W.b[c], part[1]);
  }
  wg_sum_fast<2>(part, red, out);
  if (threadIdx.x < 2) W.part3[b * RT_NPART + threadIdx.x] = out[threadIdx.x];
}

__global__ void __launch_bounds__(BLK) k_rom_pass1(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused) return;
  const RomDev &R = rom_of(I, blockIdx.z);
  const RomWork &W = *R.work;
  if (!W.active || (int)blockIdx.x >= W.nblk) return;
  __shared__ double red[(BLK / 64) * (2 * RT_RMAX + 2)], out[2 * RT_RMAX + 2];
  rom_pass1(I, R, W, blockIdx.z, blockIdx.x, W.nblk, red, out);
}

__global__ void __launch_bounds__(BLK) k_rom_pass2(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused) return;
  const RomDev &R = rom_of(I, blockIdx.z);
  const RomWork &W = *R.work;
  if (!W.active || (int)blockIdx.x >= W.nblk) return;
  __shared__ double red[(BLK / 64) * 2 * RT_RMAX], out[2 * RT_RMAX], av[RT_RMAX], scratch[BLK];
  rom_pass2(I, R, W, blockIdx.x, W.nblk, red, out, av, scratch);
}

__global__ void __launch_bounds__(BLK) k_rom_pass3(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused) return;
  const RomDev &R = rom_of(I, blockIdx.z);
  const RomWork &W = *R.work;
  if (!W.active || (int)blockIdx.x >= W.nblk) return;
  __shared__ double red[(BLK / 64) * 2], out[2], a2[RT_RMAX], scratch[BLK];
  rom_pass3(I, R, W, blockIdx.x, W.nblk, red, out, a2, scratch);
}

// ---------------------------------------------------------------------------
// Small dense part of the update (isvd_core) and Alg. 2's phase flags for
// ROM z of one instance; every thread of the workgroup calls it.  Block z
// writes only ROM z's state fields, so the two ROMs' workgroups may run at
// once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rom_core(const Inst &I, const RomDev &R, const RomWork &W, int z, RomSmem &sm) {
  RtState *st = I.st;
  int rank = z ? st->rank_pc : st->rank_ig;
  int luok = z ? st->lu_ok_pc : st->lu_ok_ig;
  const int dfc = isvd_core(R, W, I.r_max, rank, luok, sm);
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
          } else {
            // PC snapshots start only after the IG construction ended in an
            // earlier step, so n0 is settled here
            st->flag_pc = 1;
            st->n1 = (int)step_no - st->n0;
          }
        }
      }
    } else {
      updated = 1;
    }
    if (z == 0) {
      st->rank_ig = rank;
      st->lu_ok_ig = luok;
      st->ig_updates += updated;
    } else {
      st->rank_pc = rank;
      st->lu_ok_pc = luok;
      st->pc_updates += updated;
    }
    if (I.hist && step_no <= I.hist_cap) {
      RtStepRec &rec = I.hist[step_no - 1];
      if (z == 0) {
        rec.ig_update = updated;
        rec.rank_ig = rank;
      } else {
        rec.pc_update = updated;
        rec.rank_pc = rank;
      }
    }
  }
}

// k_rom_core: rom_core after the grid passes, grid (instance, ROM).
__global__ void __launch_bounds__(256) k_rom_core(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if (I.method != RT_ROM || I.post_fused) return;
  const int z = blockIdx.y;
  const RomDev &R = rom_of(I, z);
  const RomWork &W = *R.work;
  if (!W.active) return;
  __shared__ RomSmem sm;
  rom_core(I, R, W, z, sm);
}

// ---------------------------------------------------------------------------
// k_rom_post_small: the whole incremental-SVD update but the rotation for a
// small instance (the slab path, whose SI kernel already took the step's
// decisions), one workgroup per (instance, ROM): the three passes with
// workgroup reductions (one partial row), then the core.  One launch instead
// of four, and no grid-wide partial sums.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rom_post_small(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if (I.method != RT_ROM || !I.post_fused) return;
  const int z = blockIdx.y;
  const RomDev &R = rom_of(I, z);
  const RomWork &W = *R.work;
  if (!W.active) return;
  __shared__ double red[(256 / 64) * (2 * RT_RMAX + 2)], out[2 * RT_RMAX + 2], av[RT_RMAX], scratch[256];
  __shared__ RomSmem sm;
  // each stage reads the partial row the previous one wrote to global memory
  rom_pass1(I, R, W, z, 0, 1, red, out);
  __syncthreads();
  rom_pass2(I, R, W, 0, 1, red, out, av, scratch);
  __syncthreads();
  rom_pass3(I, R, W, 0, 1, red, out, av, scratch);
  __syncthreads();
  rom_core(I, R, W, z, sm);
}

// ---------------------------------------------------------------------------
// k_rom_update: U <- [U, p/nu] Uc, W <- [W, b] Vc (App. B), grid (cell
// blocks, instance, 4) with z = 2 * ROM + (0: U, 1: W); each thread rotates
// UPD_CPT cells (strided by the block width, so every load is coalesced).
// Every cell's arithmetic is the same whatever UPD_CPT: one cell per thread
// spreads a small launch over more compute units, four per thread cut the
// LDS reads of the coefficients in a large one.
// ---------------------------------------------------------------------------
constexpr int UPD_BLK = 64;
template <int UPD_CPT>
__global__ void __launch_bounds__(UPD_BLK) k_rom_update(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  // four spare entries: the column blocks of the rotation read up to three
  // entries past the last row (discarded products)
  __shared__ double cc[RT_KC * RT_KC + 4];
  if (I.method != RT_ROM) return;
  const int cb = blockIdx.x * UPD_BLK * UPD_CPT;
  if (cb >= I.nc) return;
  const int rom = blockIdx.z >> 1, mat = blockIdx.z & 1;
  const RomDev &R = rom ? I.pc : I.ig;
  const RomPend &P = *R.pend;
  if (!P.pending) return;
  const double *src = mat ? P.Vc : P.Uc;
  for (int e = threadIdx.x; e < RT_KC * RT_KC; e += blockDim.x) cc[e] = src[e];
  __syncthreads();
  const int r = P.r_old, ld = I.ld;
  double *X = mat ? R.W : R.U;
  // the cells' old basis rows, all loads in flight together (masked past r;
  // cells past nc read the padded tail of the column, ld >= nc rounded up,
  // and are not written)
  int c[UPD_CPT];
  bool ok[UPD_CPT];
  double old[UPD_CPT][RT_RMAX], e[UPD_CPT];
#pragma unroll
  for (int i = 0; i < UPD_CPT; ++i) {
    c[i] = cb + i * UPD_BLK + threadIdx.x;
    ok[i] = c[i] < I.nc;
    const int cl = ok[i] ? c[i] : I.nc - 1;
#pragma unroll
    for (int q = 0; q < RT_RMAX; ++q) {
      const double v = X[(size_t)q * ld + cl];
      old[i][q] = q < r ? v : 0.0;
    }
    // row r: p / nu for U (inv_nu = 0 and a zero row when the snapshot was
    // rank-deficient), b for W
    e[i] = mat ? P.b[cl] : P.p[cl] * P.inv_nu;
  }
  rotate_block<UPD_CPT>(old, e, cc, r, P.k, X, ld, c, ok);
}

extern "C" hipError_t rt_launch_rom(const Inst *dinsts, int ninst, int nc_max, int any_rom, hipStream_t s) {
  const int nb = pass_blocks(nc_max);
  if (any_rom) hipLaunchKernelGGL(k_rom_norms, dim3(nb, ninst), dim3(BLK), 0, s, dinsts);
  hipLaunchKernelGGL(k_rom_decide, dim3(ninst), dim3(256), 0, s, dinsts);
  if (any_rom) {
    hipLaunchKernelGGL(k_rom_pass1, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass2, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass3, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_core, dim3(ninst, 2), dim3(256), 0, s, dinsts);
  }
  return hipGetLastError();
}

// Slab instances: the SI kernel took the decisions.  Fused instances take
// one launch; the others the grid passes and the core.  nc_grid: the largest
// non-fused instance (0: none).
extern "C" hipError_t rt_launch_rom_slab(const Inst *dinsts, int ninst, int any_fused, int nc_grid, hipStream_t s) {
  if (any_fused) hipLaunchKernelGGL(k_rom_post_small, dim3(ninst, 2), dim3(256), 0, s, dinsts);
  if (nc_grid > 0) {
    const int nb = pass_blocks(nc_grid);
    hipLaunchKernelGGL(k_rom_pass1, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass2, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass3, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_core, dim3(ninst, 2), dim3(256), 0, s, dinsts);
  }
  return hipGetLastError();
}

extern "C" hipError_t rt_launch_rom_update(const Inst *dinsts, int ninst, int nc_max, hipStream_t stream) {
  if ((long long)nc_max * ninst <= 65536) {
    hipLaunchKernelGGL(k_rom_update<1>, dim3((nc_max + UPD_BLK - 1) / UPD_BLK, ninst, 4), dim3(UPD_BLK), 0, stream,
                       dinsts);
  } else {
    const int cells = UPD_BLK * 4;
    hipLaunchKernelGGL(k_rom_update<4>, dim3((nc_max + cells - 1) / cells, ninst, 4), dim3(UPD_BLK), 0, stream,
                       dinsts);
  }
  return hipGetLastError();
}

// copies of every instance's phase-machine state, for one host read per batch
__global__ void __launch_bounds__(256) k_gather_states(const Inst *__restrict__ insts, int ninst, RtState *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) out[i] = *insts[i].st;
}

extern "C" hipError_t rt_launch_gather_states(const Inst *dinsts, int ninst, RtState *out, hipStream_t stream) {
  hipLaunchKernelGGL(k_gather_states, dim3((ninst + 255) / 256), dim3(256), 0, stream, dinsts, ninst, out);
  return hipGetLastError();
}
