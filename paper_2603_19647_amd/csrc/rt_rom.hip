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

}  // namespace

// ---------------------------------------------------------------------------
// k_rom_norms: per-block partial sums of ||rho^n||^2, ||rho^(0) - rho^n||^2
// and ||dpc - (rho^n - rho^(1/2))||^2 for the error indicators of Sec. 3.2,
// grid (blocks of BLK cells, instance).  Written to the IG ROM's third
// partial buffer, which the ROM passes do not use.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(BLK) k_rom_norms(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || !I.st->flag_ig) return;
  const int nb = pass_blocks(I.nc);
  if ((int)blockIdx.x >= nb) return;
  __shared__ double red[(BLK / 64) * (3 + RT_XLEV)], out[3 + RT_XLEV];
  double part[3 + RT_XLEV];
  rom_norm_parts(I, blockIdx.x * BLK + threadIdx.x, nb * BLK, part);
  wg_sum_fast<3 + RT_XLEV>(part, red, out);
  if (threadIdx.x < 3 + RT_XLEV) I.ig.work->part3[blockIdx.x * RT_NPART + threadIdx.x] = out[threadIdx.x];
}

// ---------------------------------------------------------------------------
// k_rom_decide: rom_decide (step bookkeeping, error indicators and Alg. 2's
// decisions) for every instance, one workgroup each, from the partial sums
// of k_rom_norms.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rom_decide(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  __shared__ double scratch[256], vec[3 + RT_XLEV];
  const int nb = pass_blocks(I.nc);
  if (I.method == RT_ROM && I.st->flag_ig) sum_partials<false>(I.ig.work->part3, nb, 3 + RT_XLEV, vec, scratch);
  rom_decide(I, vec, I.post_nb, step_in(I.st));
}

__global__ void __launch_bounds__(BLK) k_rom_pass1(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused || (int)blockIdx.z > I.nlev) return;
  const RomDev &R = rom_of(I, blockIdx.z);
  const RomWork &W = *R.work;
  if (!W.active || (int)blockIdx.x >= W.nblk) return;
  __shared__ double red[(BLK / 64) * (2 * RT_RMAX + 2)], out[2 * RT_RMAX + 2];
  rom_pass1<false>(I, R, W, blockIdx.z, blockIdx.x, W.nblk, red, out);
}

__global__ void __launch_bounds__(BLK) k_rom_pass2(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused || (int)blockIdx.z > I.nlev) return;
  const RomDev &R = rom_of(I, blockIdx.z);
  const RomWork &W = *R.work;
  if (!W.active || (int)blockIdx.x >= W.nblk) return;
  __shared__ double red[(BLK / 64) * (2 * RT_RMAX + 2)], out[2 * RT_RMAX + 2], av[RT_RMAX], scratch[BLK];
  rom_pass2<false>(I, R, W, blockIdx.x, W.nblk, red, out, av, scratch);
}


// k_rom_core: rom_core after the grid passes, grid (instance, ROM).
__global__ void __launch_bounds__(256) k_rom_core(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if (I.method != RT_ROM || I.post_fused || (int)blockIdx.y > I.nlev) return;
  const int z = blockIdx.y;
  const RomDev &R = rom_of(I, z);
  const RomWork &W = *R.work;
  if (!W.active) return;
  __shared__ RomSmem sm;
  rom_core<false>(I, R, W, z, sm);
}

// ---------------------------------------------------------------------------
// k_rom_post_small: the whole incremental-SVD update of a small instance (the
// slab path, whose SI kernel already took the step's decisions), one
// workgroup per (instance, ROM): the two passes with workgroup reductions
// (one partial row), the core, then the rotation of the ROM's two bases with
// the reduced operator's LU factored beside it.  One launch instead of four,
// no grid-wide partial sums, and the rotation's traffic overlaps the f-pass
// that runs beside this launch.
// ---------------------------------------------------------------------------
// two workgroups per CU: the registers stay within half the file
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_rom_post_small(
    const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.x];
  if (I.method != RT_ROM || !I.post_fused) return;
  const int z = blockIdx.y;  // 0: initial guess, l: correction of iteration l
  if (z > I.nlev) return;
  const RomDev &R = rom_of(I, z);
  const RomWork &W = *R.work;
  if (!W.active) return;
  __shared__ double red[(256 / 64) * (2 * RT_RMAX + 2)], out[2 * RT_RMAX + 2], av[RT_RMAX], scratch[256];
  __shared__ RomSmem sm;
  // each stage reads the partial row the previous one wrote to global memory
  rom_pass1<false>(I, R, W, z, 0, 1, red, out);
  __syncthreads();
  rom_pass2<false>(I, R, W, 0, 1, red, out, av, scratch);
  __syncthreads();
  rom_core<false, true>(I, R, W, z, sm);
  rom_rotate_own_lu(I, R, W, sm, z);  // the LU beside the rotation
}

// ---------------------------------------------------------------------------
// k_rom_update: U <- [U, p/nu] Uc, W <- [W, b] Vc (App. B), grid (cell
// blocks, instance, 4) with z = 2 * ROM + (0: U, 1: W); each thread rotates
// UPD_CPT cells (strided by the block width, so every load is coalesced).
// The coefficients are the same for every cell of a block and were written
// by an earlier launch, so they are read through the constant address space:
// scalar loads into scalar registers, which leaves the vector registers to
// the cells' basis rows (occupancy) and needs no LDS staging.
// ---------------------------------------------------------------------------
#define RT_CONST __attribute__((address_space(4)))
template <int UPD_BLK, int UPD_CPT>
__global__ void __launch_bounds__(UPD_BLK) k_rom_update(const Inst *__restrict__ insts) {
  const Inst &I = insts[blockIdx.y];
  if (I.method != RT_ROM || I.post_fused) return;  // fused posts rotate their own bases
  const int cb = blockIdx.x * UPD_BLK * UPD_CPT;
  if (cb >= I.nc) return;
  const int rom = blockIdx.z >> 1, mat = blockIdx.z & 1;
  if (rom > I.nlev) return;
  const RomDev &R = rom_of(I, rom);
  const RomPend &P = *R.pend;
  if (!P.pending) return;
  const RT_CONST double *cc = (const RT_CONST double *)(mat ? P.Vc : P.Uc);
  const RT_CONST double *a2 = (const RT_CONST double *)P.a2;
  const int r = P.r_old, ld = I.ld;
  double *X = mat ? R.W : R.U;
  // the cells' old basis rows up to r, all loads in flight together (zero
  // past r; cells past nc read the last cell and are not written)
  int c[UPD_CPT];
  bool ok[UPD_CPT];
  double old[UPD_CPT][RT_RMAX], e[UPD_CPT];
#pragma unroll
  for (int i = 0; i < UPD_CPT; ++i) {
    c[i] = cb + i * UPD_BLK + threadIdx.x;
    ok[i] = c[i] < I.nc;
    const int cl = ok[i] ? c[i] : I.nc - 1;
#pragma unroll
    for (int q = 0; q < RT_RMAX; ++q) old[i][q] = q < r ? ldg(&X[(size_t)q * ld + cl]) : 0.0;
    // row r: the new direction, (v - U a2) / nu for U (inv_nu = 0 and a zero
    // row when the snapshot was rank-deficient), b for W
    e[i] = mat ? ldg(&P.b[cl]) : second_residual(ldg(&P.p[cl]), old[i], a2) * P.inv_nu;
  }
  rotate_block<UPD_CPT>(old, e, cc, r, P.k, X, ld, c, ok);
}

extern "C" hipError_t rt_launch_rom(const Inst *dinsts, int ninst, int nc_max, int any_rom, int nrom,
                                    hipStream_t s) {
  const int nb = pass_blocks(nc_max);
  if (any_rom) hipLaunchKernelGGL(k_rom_norms, dim3(nb, ninst), dim3(BLK), 0, s, dinsts);
  hipLaunchKernelGGL(k_rom_decide, dim3(ninst), dim3(256), 0, s, dinsts);
  if (any_rom) {
    hipLaunchKernelGGL(k_rom_pass1, dim3(nb, ninst, nrom), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass2, dim3(nb, ninst, nrom), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_core, dim3(ninst, nrom), dim3(256), 0, s, dinsts);
  }
  return hipGetLastError();
}

// Slab instances: the SI kernel took the decisions.  Fused instances take
// one launch; the others the grid passes and the core.  nc_grid: the largest
// non-fused instance (0: none).
extern "C" hipError_t rt_launch_rom_slab(const Inst *dinsts, int ninst, int any_fused, int nc_grid, int nrom,
                                         hipStream_t s) {
  if (any_fused) hipLaunchKernelGGL(k_rom_post_small, dim3(ninst, nrom), dim3(256), 0, s, dinsts);
  if (nc_grid > 0) {
    const int nb = pass_blocks(nc_grid);
    hipLaunchKernelGGL(k_rom_pass1, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_pass2, dim3(nb, ninst, 2), dim3(BLK), 0, s, dinsts);
    hipLaunchKernelGGL(k_rom_core, dim3(ninst, 2), dim3(256), 0, s, dinsts);
  }
  return hipGetLastError();
}

extern "C" hipError_t rt_launch_rom_update(const Inst *dinsts, int ninst, int nc_max, int nrom, hipStream_t stream) {
  if ((long long)nc_max * ninst <= 65536) {
    // small: one cell per thread in narrow blocks, spread over many CUs
    hipLaunchKernelGGL((k_rom_update<64, 1>), dim3((nc_max + 63) / 64, ninst, 2 * nrom), dim3(64), 0, stream,
                       dinsts);
  } else {
    hipLaunchKernelGGL((k_rom_update<256, 1>), dim3((nc_max + 255) / 256, ninst, 2 * nrom), dim3(256), 0, stream,
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
