// rt_host.h -- host-side problem object of librtrom (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/rtrom.h"
#include "rt_common.h"

struct rtrom_problem {
  rtrom_problem_desc d;  // copy; array pointers cleared
  int id = 0;            // creation order in the process (diagnostics)
  int device = 0;
  int nc = 0, nv = 0;
  std::vector<double> ox, oy, oz, w;  // quadrature (host copy)
  // device memory
  char *arena = nullptr;
  size_t arena_bytes = 0;
  RtStepRec *dhist = nullptr;
  int64_t hist_cap = 0;
  Inst hinst{};          // descriptor with device pointers
  Inst *dinst = nullptr; // device copy of hinst
  hipStream_t own_stream = nullptr, stream = nullptr;
  hipStream_t aux_stream = nullptr;          // ROM updates overlap the f-pass here
  hipEvent_t ev_si = nullptr, ev_rom = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int64_t steps = 0;     // host mirror of the step counter
  double t_total = 0.0;
  // 2D launch geometry / scratch
  void *plane = nullptr;
};

// launch helpers implemented in the .hip kernel files
extern "C" hipError_t rt_launch_slab_si_coop(const Inst *dinst, int ng, int nthreads, int cmax, hipStream_t stream);
extern "C" int rt_slab_coop_fits(int device, int ng, int nthreads, int cmax, int npair, int nc);
extern "C" hipError_t rt_launch_slab_tail_coop(const Inst *dinst, int npair, int nc, int nthreads, int cmax,
                                               hipStream_t stream);
extern "C" hipError_t rt_launch_slab_si(const Inst *dinsts, int ninst, int nthreads, int cmax,
                                        hipStream_t stream);
extern "C" hipError_t rt_launch_slab_fpass(const Inst *dinsts, int ninst, int nthreads, int cmax, int npair_max,
                                           int nc_max, int pairs_total, hipStream_t stream);
// nrom: 1 + the largest number of correction levels in the launch
extern "C" hipError_t rt_launch_rom(const Inst *dinsts, int ninst, int nc_max, int any_rom, int nrom, hipStream_t s);
// nrom: 1 + the largest number of correction levels in the launch
extern "C" hipError_t rt_launch_rom_slab(const Inst *dinsts, int ninst, int any_fused, int nc_grid, int nrom,
                                         hipStream_t s);
extern "C" hipError_t rt_launch_rom_update(const Inst *dinsts, int ninst, int nc_max, int nrom, hipStream_t stream);
extern "C" hipError_t rt_launch_slab_rhs(const Inst *dinsts, int ninst, int nthreads, int cmax, int npair_max,
                                         int nc_max, hipStream_t stream);
// kinds: bit 0 -- the launch holds instances of the default configuration,
// bit 1 -- instances of the variant (SI: McClarren-Haut; f-pass: BDF2),
// bit 2 -- piecewise-linear DG instances, bit 3 -- DG instances with
// McClarren-Haut (SI launch only), bit 4 -- DG instances with BDF2 (f-pass
// only)
extern "C" hipError_t rt_launch_slab_si_wave(const Inst *dinsts, int ninst, int kinds, hipStream_t stream);
extern "C" hipError_t rt_launch_slab_fpass_wave(const Inst *dinsts, int ninst, int rhs_only, int kinds,
                                                hipStream_t stream);
extern "C" hipError_t rt_launch_slab_setup(const Inst *dinsts, int ninst, int nc_max, int alt, hipStream_t stream);
extern "C" hipError_t rt_launch_setup_dsa_dg(const Inst *dinsts, int ninst, int alt, hipStream_t stream);
extern "C" hipError_t rt_launch_gather_states(const Inst *dinsts, int ninst, RtState *out, hipStream_t stream);

// 2D
int rt_plane_create(rtrom_problem *p);
void rt_plane_destroy(rtrom_problem *p);
int rt_plane_step(rtrom_problem *p, int nsteps);
int rt_plane_rhs(rtrom_problem *p);
size_t rt_plane_extra_bytes(const rtrom_problem_desc *d);
int rt_plane_max_nx_cyclic();
int rt_plane_dsa_iters(const rtrom_problem *p);
int rt_plane_needs_cyclic(int ny);
int rt_plane_unfold(const rtrom_problem *p, double *f_host);  // folded f -> full ordinate order

void rt_set_error(const std::string &msg);

// Diagnostics.  RTROM_LOG (read once per process) sets what goes to stderr:
// 0 nothing (default), 1 errors, 2 also problem creation / destruction and
// ROM phase changes, 3 also one line per time step.  Phases and marches are
// marked with roctx ranges and marks for rocprofv3 (--marker-trace); these
// cost nothing measurable when no profiler is attached.
int rt_log_level();
void rt_log(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void rt_mark(const char *msg);
struct RtRange {
  explicit RtRange(const char *name);
  ~RtRange();
  RtRange(const RtRange &) = delete;
  RtRange &operator=(const RtRange &) = delete;
};
rtrom_status rt_validate(const rtrom_problem_desc *d);  // host-only checks of a description

// Kernel timing (rtrom_profile_*): bracket a launch with events when enabled.
enum { RT_K_SLAB_SI = 0, RT_K_SLAB_FPASS = 1, RT_K_POST = 2, RT_K_PLANE_SWEEP = 3, RT_K_PLANE_DSA = 4,
       RT_K_PLANE_FPASS = 5, RT_K_PLANE_OTHER = 6, RT_K_ROM_UPDATE = 7, RT_NKINDS = 8 };
void rt_prof_begin(int kind, hipStream_t s);
void rt_prof_end(int kind, hipStream_t s);
void rt_prof_collect();  // after the stream(s) synchronised
bool rt_prof_on();
