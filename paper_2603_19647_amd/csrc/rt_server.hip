// rt_server.hip -- serving (continuous batching) for librtrom.
#include "rt_host.h"

struct rtrom_server {
  int dummy;
};

extern "C" rtrom_status rtrom_server_create(const rtrom_server_desc *d, rtrom_server **out) {
  (void)d;
  if (out) *out = nullptr;
  rt_set_error("server not available in this build");
  return RTROM_EINVAL;
}
extern "C" rtrom_status rtrom_server_submit(rtrom_server *s, const rtrom_problem_desc *d, int32_t nsteps,
                                            uint64_t *ticket) {
  (void)s; (void)d; (void)nsteps; (void)ticket;
  return RTROM_EINVAL;
}
extern "C" rtrom_status rtrom_server_poll(rtrom_server *s, uint64_t ticket, int32_t *state) {
  (void)s; (void)ticket; (void)state;
  return RTROM_EINVAL;
}
extern "C" rtrom_status rtrom_server_drain(rtrom_server *s) { (void)s; return RTROM_EINVAL; }
extern "C" rtrom_status rtrom_server_fetch(rtrom_server *s, uint64_t ticket, double *rho, int64_t n,
                                           rtrom_stats *st, double *lat, int64_t nlat, double *mlat) {
  (void)s; (void)ticket; (void)rho; (void)n; (void)st; (void)lat; (void)nlat; (void)mlat;
  return RTROM_EINVAL;
}
extern "C" void rtrom_server_destroy(rtrom_server *s) { (void)s; }
