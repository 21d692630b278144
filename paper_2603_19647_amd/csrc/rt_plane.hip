// rt_plane.hip -- X-Y (2D) path of librtrom.
#include "rt_host.h"

size_t rt_plane_extra_bytes(const rtrom_problem_desc *d) { (void)d; return 0; }
int rt_plane_create(rtrom_problem *p) {
  (void)p;
  rt_set_error("2D problems are not available in this build");
  return RTROM_EINVAL;
}
void rt_plane_destroy(rtrom_problem *p) { (void)p; }
int rt_plane_step(rtrom_problem *p, int nsteps) { (void)p; (void)nsteps; return RTROM_EINVAL; }
int rt_plane_rhs(rtrom_problem *p) { (void)p; return RTROM_EINVAL; }
