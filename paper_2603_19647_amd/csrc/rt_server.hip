// rt_server.hip -- serving: continuous batching of independent time-marching
// problems on one device.
//
// Requests queue in submission order.  A pool of max_slots worker threads
// admits the head of the queue as soon as a slot is free and the request's
// device footprint fits the remaining HBM budget; the worker then creates the
// problem (its own streams and device state), marches it step by step and
// records each step's latency.  Several admitted problems march at once, each
// on its own streams, so their kernels overlap on the device.  When a march
// ends, the scalar flux and statistics are copied to the host and the device
// state is released, which frees budget for the next admission.
//
// A result depends only on its own request: every problem has its own state,
// launch shapes and fixed-order reductions, so it is the same alone and in
// the mix.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rt_host.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  rtrom_problem_desc d{};
  std::vector<double> ss, sa, G, f0;  // owned copies of the description's arrays
  int32_t nsteps = 0;
  uint64_t bytes = 0;
  int32_t state = RTROM_REQ_QUEUED;
  rtrom_status status = RTROM_OK;
  std::string err;
  std::vector<double> rho;   // result (host)
  rtrom_stats stats{};
  std::vector<double> lat;   // per-step seconds
  double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct rtrom_server {
  rtrom_server_desc d{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t used = 0, next_ticket = 1;
  int pending = 0;  // queued + running
  bool stop = false;
  std::vector<std::thread> workers;
};

static void march_request(rtrom_server *s, Req *r) {
  if (hipSetDevice(s->d.device) != hipSuccess) {
    r->status = RTROM_EDEVICE;
    r->err = "server: cannot select the device";
    return;
  }
  rtrom_problem *p = nullptr;
  rtrom_status st = rtrom_create_problem(&r->d, &p);
  if (st != RTROM_OK) {
    r->status = st;
    r->err = rtrom_last_error();
    return;
  }
  r->lat.resize(r->nsteps);
  rtrom_status worst = RTROM_OK;
  for (int32_t k = 0; k < r->nsteps; ++k) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) {
        worst = RTROM_EINVAL;
        r->err = "server: destroyed while the request was running";
        break;
      }
    }
    const double t0 = now_s();
    st = rtrom_step(p);  // returns once the device finished the step
    r->lat[k] = now_s() - t0;
    if (st == RTROM_ENOCONV) {
      worst = RTROM_ENOCONV;  // the state advanced; keep marching (R8)
    } else if (st != RTROM_OK) {
      worst = st;
      r->err = rtrom_last_error();
      r->lat.resize(k + 1);
      break;
    }
  }
  if (worst == RTROM_OK || worst == RTROM_ENOCONV) {
    r->rho.resize((size_t)r->d.nx * r->d.ny * (r->d.scheme == RTROM_DG1 ? 2 : 1));  // unknowns
    st = rtrom_get_scalar_flux(p, r->rho.data(), (int64_t)r->rho.size());
    if (st == RTROM_OK) st = rtrom_stats_get(p, &r->stats);
    if (st != RTROM_OK) {
      worst = st;
      r->err = rtrom_last_error();
    }
  }
  rtrom_destroy_problem(p);
  r->status = worst;
}

static void worker_loop(rtrom_server *s) {
  for (;;) {
    Req *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // admit the head of the queue when it fits the remaining budget
      s->cv_work.wait(lk, [&] {
        return s->stop || (!s->queue.empty() && s->used + s->queue.front()->bytes <= s->d.hbm_budget_bytes);
      });
      if (s->stop) return;
      r = s->queue.front();
      s->queue.pop_front();
      s->used += r->bytes;
      r->state = RTROM_REQ_RUNNING;
      r->t_admit = now_s();
    }
    march_request(s, r);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->used -= r->bytes;
      r->t_done = now_s();
      r->state = (r->status == RTROM_OK || r->status == RTROM_ENOCONV) ? RTROM_REQ_DONE : RTROM_REQ_FAILED;
      s->pending--;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
}

extern "C" rtrom_status rtrom_server_create(const rtrom_server_desc *d, rtrom_server **out) {
  if (!d || !out) {
    rt_set_error("server: null argument");
    return RTROM_EINVAL;
  }
  *out = nullptr;
  if (d->max_slots < 1 || d->max_slots > 256 || d->hbm_budget_bytes == 0 || d->device < 0) {
    rt_set_error("server: max_slots must be 1..256, hbm_budget_bytes > 0, device >= 0");
    return RTROM_EINVAL;
  }
  // Bring the HIP runtime up on the creating thread before any worker uses
  // it: a process whose only HIP calls came from worker threads that have
  // since exited crashed during runtime teardown at process exit.
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d->device >= ndev || hipSetDevice(d->device) != hipSuccess ||
      hipFree(nullptr) != hipSuccess) {
    rt_set_error("server: cannot initialise the HIP device");
    return RTROM_EDEVICE;
  }
  rtrom_server *s = new rtrom_server();
  s->d = *d;
  try {
    for (int i = 0; i < d->max_slots; ++i) s->workers.emplace_back(worker_loop, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    delete s;
    rt_set_error("server: cannot start worker threads");
    return RTROM_ENOMEM;
  }
  *out = s;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_server_submit(rtrom_server *s, const rtrom_problem_desc *d, int32_t nsteps,
                                            uint64_t *ticket) {
  if (!s || !d || !ticket) {
    rt_set_error("server: null argument");
    return RTROM_EINVAL;
  }
  if (nsteps < 0) {
    rt_set_error("server: nsteps must be >= 0");
    return RTROM_EINVAL;
  }
  // served problems run one workgroup each (RTROM_F_SINGLE_WG): many march
  // at once, so none may rely on co-resident workgroups of its own
  rtrom_problem_desc dd = *d;
  dd.flags |= RTROM_F_SINGLE_WG;
  d = &dd;
  rtrom_status v = rt_validate(d);
  if (v != RTROM_OK) return v;
  uint64_t bytes = 0;
  v = rtrom_estimate_bytes(d, &bytes);
  if (v != RTROM_OK) return v;
  bytes += (uint64_t)nsteps * sizeof(rtrom_step_record);  // the step history grows with the march
  if (bytes > s->d.hbm_budget_bytes) {
    rt_set_error("server: the request can never fit the HBM budget");
    return RTROM_ENOMEM;
  }
  auto r = std::make_unique<Req>();
  const size_t nc = (size_t)d->nx * d->ny;
  r->d = *d;
  r->ss.assign(d->sigma_s, d->sigma_s + nc);
  r->sa.assign(d->sigma_a, d->sigma_a + nc);
  r->G.assign(d->source, d->source + nc);
  if (d->f0) r->f0.assign(d->f0, d->f0 + nc);
  r->d.sigma_s = r->ss.data();
  r->d.sigma_a = r->sa.data();
  r->d.source = r->G.data();
  r->d.f0 = d->f0 ? r->f0.data() : nullptr;
  r->nsteps = nsteps;
  r->bytes = bytes;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->pending++;
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_all();
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_server_poll(rtrom_server *s, uint64_t ticket, int32_t *state) {
  if (!s || !state) {
    rt_set_error("server: null argument");
    return RTROM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    rt_set_error("server: unknown ticket");
    return RTROM_EINVAL;
  }
  *state = it->second->state;
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_server_drain(rtrom_server *s) {
  if (!s) {
    rt_set_error("server: null argument");
    return RTROM_EINVAL;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending == 0; });
  return RTROM_OK;
}

extern "C" rtrom_status rtrom_server_fetch(rtrom_server *s, uint64_t ticket, double *rho, int64_t n,
                                           rtrom_stats *st, double *lat, int64_t nlat, double *mlat) {
  if (!s) {
    rt_set_error("server: null argument");
    return RTROM_EINVAL;
  }
  std::unique_ptr<Req> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
      rt_set_error("server: unknown ticket");
      return RTROM_EINVAL;
    }
    Req *q = it->second.get();
    if (q->state == RTROM_REQ_QUEUED || q->state == RTROM_REQ_RUNNING) {
      rt_set_error("server: request not finished");
      return RTROM_EBUSY;
    }
    if (q->state == RTROM_REQ_DONE && rho && n < (int64_t)q->rho.size()) {
      rt_set_error("server: output buffer too small");
      return RTROM_EINVAL;
    }
    r = std::move(it->second);
    s->reqs.erase(it);
  }
  if (r->state == RTROM_REQ_FAILED) {
    rt_set_error(r->err.empty() ? "server: request failed" : r->err);
    return r->status;
  }
  if (rho) memcpy(rho, r->rho.data(), r->rho.size() * sizeof(double));
  if (st) *st = r->stats;
  if (lat && nlat > 0) {
    const size_t m = std::min<size_t>((size_t)nlat, r->lat.size());
    memcpy(lat, r->lat.data(), m * sizeof(double));
  }
  if (mlat) *mlat = r->t_done - r->t_admit;
  return r->status;
}

extern "C" void rtrom_server_destroy(rtrom_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  delete s;
}
