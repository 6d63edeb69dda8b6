// Continuous-batching solve server: admits space-time solve requests of
// different meshes and horizons as device memory frees up, overlaps their
// work on the GPU (one non-blocking stream per active request) and reports
// latency percentiles and throughput.
//
// Life of a request: submitted (host copies of its inputs) -> host setup on
// a worker thread (assembly, hierarchy, orderings, symbolic factorisation,
// front plans; no HIP calls) -> admitted by the scheduler thread once its
// estimated device bytes fit the HBM budget and a slot is free -> device
// setup on a worker thread, on the request's own stream (numeric
// factorisation on the GPU, uploads, right-hand side) -> iterations driven
// by the scheduler (one in flight per request; the residual norm comes back
// through pinned memory and an event, polled without blocking) -> result
// copied to pinned host memory -> device memory released on its stream.
// Device setup never runs on the scheduler thread, so a large request's
// factorisation does not stall the iterations of the requests in flight.
// Requests whose next iterations are due at the same time and whose V-cycles
// take the same steps (same N_t, DG degree, precision form and smoother) run
// those iterations batched, on one of the server's shared streams: the slab
// and nodal solves of each level step of all of them in one launch per tree
// height (up to 8 requests). Every request computes its values with the same
// instructions in the same order as alone, batched or not, so its result
// does not depend on the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "solver.hpp"

using namespace stmg;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum State { PENDING, HOST_SETUP, READY, ADMITTED, DEVICE_SETUP, RUNNING, FINISHING, DONE, FAILED };

// Deep copy of a problem description (the ABI borrows arrays for one call).
struct ProblemCopy {
  std::vector<std::vector<double>> coords;
  std::vector<std::vector<int32_t>> tets, vparent, tparent;
  std::vector<stmg_mesh> meshes;
  std::vector<double> sigma, nu;
  stmg_problem prob{};

  void take(const stmg_problem &p) {
    const int nm = p.n_meshes;
    coords.resize(nm);
    tets.resize(nm);
    vparent.resize(nm);
    tparent.resize(nm);
    meshes.resize(nm);
    for (int j = 0; j < nm; ++j) {
      const stmg_mesh &m = p.meshes[j];
      STMG_REQUIRE(m.coords && m.tets && m.n_vertices > 0 && m.n_tets > 0, STMG_EINVAL, "empty mesh");
      coords[j].assign(m.coords, m.coords + 3 * (size_t)m.n_vertices);
      tets[j].assign(m.tets, m.tets + 4 * (size_t)m.n_tets);
      meshes[j] = m;
      meshes[j].coords = coords[j].data();
      meshes[j].tets = tets[j].data();
      if (j > 0) {
        STMG_REQUIRE(m.vertex_parent && m.tet_parent, STMG_EINVAL, "coarse mesh without parent maps");
        vparent[j].assign(m.vertex_parent, m.vertex_parent + 2 * (size_t)p.meshes[j - 1].n_vertices);
        tparent[j].assign(m.tet_parent, m.tet_parent + (size_t)p.meshes[j - 1].n_tets);
        meshes[j].vertex_parent = vparent[j].data();
        meshes[j].tet_parent = tparent[j].data();
      }
    }
    STMG_REQUIRE(p.sigma && p.nu, STMG_EINVAL, "sigma/nu missing");
    sigma.assign(p.sigma, p.sigma + p.meshes[0].n_tets);
    nu.assign(p.nu, p.nu + p.meshes[0].n_tets);
    prob = p;
    prob.meshes = meshes.data();
    prob.sigma = sigma.data();
    prob.nu = nu.data();
  }
};

struct Request {
  uint64_t ticket = 0;
  State state = PENDING;
  int code = STMG_OK;
  std::string message;
  ProblemCopy pc;
  stmg_options opt{};
  std::vector<double> rhs, u0;  // host copies, full layout
  std::vector<double> x;        // result, full layout
  stmg_handle *h = nullptr;
  hipStream_t stream = nullptr;
  double *d_rhs = nullptr, *d_u0 = nullptr, *d_x = nullptr;
  double *pin_norm = nullptr, *pin_x = nullptr;
  hipEvent_t ev = nullptr;
  bool in_flight = false;
  bool want_iteration = false;  // the previous iteration is done and another is due
  int64_t est_bytes = 0;
  int64_t dofs = 0;  // n_e * N_t * q of the finest level
  double bnorm = 0.0;
  std::vector<double> history;
  double t_submit = 0, t_ready = 0, t_admit = 0, t_done = 0, setup_s = 0;
};

}  // namespace

struct stmg_server {
  stmg_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending, ready, admitted;
  std::vector<std::shared_ptr<Request>> active;
  int32_t n_setting_up = 0;  // admitted requests not yet running
  std::map<uint64_t, std::shared_ptr<Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t reserved = 0, peak = 0;
  int64_t submitted = 0, completed = 0, failed = 0;
  double t_first_submit = -1, t_last_done = 0, dof_updates = 0;
  std::vector<double> latencies;
  std::vector<std::thread> workers;
  std::thread scheduler;
  int device = 0;
  std::vector<hipStream_t> batch_streams;  // shared streams of batched iterations
  size_t next_batch_stream = 0;
  int64_t batched_iterations = 0, batched_members = 0;

  void worker_loop();
  void host_setup(const std::shared_ptr<Request> &r);
  void device_setup(const std::shared_ptr<Request> &r);
  void scheduler_loop();
  bool admit_one();
  bool progress(Request &r);
  void launch_iterations();
  void start_iteration(Request &q);
  void finish(Request &r, int code, const char *msg);
  void release(Request &r);
};

namespace {

void hipc(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? STMG_ENOMEM : STMG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

void stmg_server::worker_loop() {
  // a failure here shows in the first HIP call of each request, whose error is reported per request
  (void)hipSetDevice(device);
  for (;;) {
    std::shared_ptr<Request> r;
    bool dev = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !admitted.empty() || !pending.empty(); });
      if (stop) return;
      if (!admitted.empty()) {  // admitted requests hold reservations: first
        r = admitted.front();
        admitted.pop_front();
        r->state = DEVICE_SETUP;
        dev = true;
      } else {
        r = pending.front();
        pending.pop_front();
        r->state = HOST_SETUP;
      }
    }
    if (dev)
      device_setup(r);
    else
      host_setup(r);
  }
}

void stmg_server::host_setup(const std::shared_ptr<Request> &r) {
  stmg_handle *h = nullptr;
  int code = STMG_OK;
  std::string msg;
  const double t0 = now_s();
  try {
    h = internal::setup_host(&r->pc.prob, &r->opt);
    r->est_bytes = internal::estimate_bytes(h);
  } catch (const StmgError &e) {
    code = e.code;
    msg = e.what();
  } catch (const std::bad_alloc &) {
    code = STMG_ENOMEM;
    msg = "host allocation failed";
  } catch (const std::exception &e) {
    code = STMG_EINVAL;
    msg = e.what();
  }
  std::unique_lock<std::mutex> lk(mu);
  r->setup_s = now_s() - t0;
  if (code == STMG_OK && r->est_bytes > opt.hbm_budget) {
    code = STMG_ENOMEM;
    msg = "request needs more device memory than the server's budget";
  }
  if (code != STMG_OK) {
    if (h) internal::destroy(h);
    r->state = FAILED;
    r->code = code;
    r->message = msg;
    r->t_done = now_s();
    failed++;
    cv_done.notify_all();
    return;
  }
  r->h = h;
  r->state = READY;
  r->t_ready = now_s();
  ready.push_back(r);
  cv_work.notify_all();
}

// Device setup of an admitted request on its own stream (worker thread).
void stmg_server::device_setup(const std::shared_ptr<Request> &r) {
  Request &q = *r;
  const double t0 = now_s();
  int code = STMG_OK;
  std::string msg;
  double bn = 0.0;
  try {
    hipc(hipStreamCreateWithFlags(&q.stream, hipStreamNonBlocking), "hipStreamCreate");
    q.h->stream_ordered = true;
    internal::setup_device(q.h, q.stream);
    stmg_info_t info;
    stmg_info(q.h, &info);
    const int64_t n = (int64_t)info.n_edges * q.pc.prob.Nt * (q.pc.prob.pt + 1);
    STMG_REQUIRE((int64_t)q.rhs.size() == n, STMG_EINVAL, "rhs length does not match the mesh");
    stmg_level_info_t li;
    stmg_level_info(q.h, 0, &li);
    q.dofs = (int64_t)li.n_e * q.pc.prob.Nt * (q.pc.prob.pt + 1);
    hipc(hipMallocAsync((void **)&q.d_rhs, n * sizeof(double), q.stream), "hipMallocAsync");
    hipc(hipMallocAsync((void **)&q.d_x, n * sizeof(double), q.stream), "hipMallocAsync");
    hipc(hipMemcpyAsync(q.d_rhs, q.rhs.data(), n * sizeof(double), hipMemcpyHostToDevice, q.stream), "upload");
    if (!q.u0.empty()) {
      hipc(hipMallocAsync((void **)&q.d_u0, q.u0.size() * sizeof(double), q.stream), "hipMallocAsync");
      hipc(hipMemcpyAsync(q.d_u0, q.u0.data(), q.u0.size() * sizeof(double), hipMemcpyHostToDevice, q.stream),
           "upload");
    }
    hipc(hipHostMalloc((void **)&q.pin_norm, sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    hipc(hipHostMalloc((void **)&q.pin_x, n * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    hipc(hipEventCreateWithFlags(&q.ev, hipEventDisableTiming), "hipEventCreate");
    const int rc = stmg_load(q.h, q.d_rhs, q.d_u0, nullptr, &bn);
    if (rc != STMG_OK) fail(rc, internal::last_error());
  } catch (const StmgError &e) {
    code = e.code;
    msg = e.what();
  } catch (const std::bad_alloc &) {
    code = STMG_ENOMEM;
    msg = "host allocation failed";
  }
  std::unique_lock<std::mutex> lk(mu);
  n_setting_up--;
  q.setup_s += now_s() - t0;
  q.t_admit = now_s();
  q.state = RUNNING;
  active.push_back(r);
  if (code != STMG_OK)
    finish(q, code, msg.c_str());
  else {
    q.bnorm = bn;
    if (bn == 0.0) finish(q, STMG_OK, "");
  }
  cv_work.notify_all();
}

// Admit the oldest ready request if its device bytes fit and a slot is free
// (caller holds mu): reserve its bytes and queue its device setup.
bool stmg_server::admit_one() {
  if (ready.empty() || (int32_t)active.size() + n_setting_up >= opt.max_active) return false;
  std::shared_ptr<Request> r = ready.front();
  if (reserved + r->est_bytes > opt.hbm_budget) return false;
  ready.pop_front();
  reserved += r->est_bytes;
  peak = std::max(peak, reserved);
  r->state = ADMITTED;
  n_setting_up++;
  admitted.push_back(r);
  cv_work.notify_all();
  return true;
}

// Advance one running request without blocking; true if anything changed.
bool stmg_server::progress(Request &q) {
  if (q.state == RUNNING) {
    if (q.in_flight) {
      const hipError_t e = hipEventQuery(q.ev);
      if (e == hipErrorNotReady) return false;
      q.in_flight = false;
      if (e != hipSuccess) {
        finish(q, STMG_EHIP, hipGetErrorString(e));
        return true;
      }
      const double rel = std::sqrt(*q.pin_norm) / q.bnorm;
      q.history.push_back(rel);
      if (!std::isfinite(rel)) {
        finish(q, STMG_ENUMERIC, "non-finite residual");
        return true;
      }
      if (rel <= q.opt.rtol) {
        finish(q, STMG_OK, "");
        return true;
      }
      if ((int32_t)q.history.size() >= q.opt.max_cycles) {
        finish(q, STMG_ENOTCONV, "max_cycles reached before rtol");
        return true;
      }
    }
    if (q.want_iteration) return false;
    q.want_iteration = true;
    return true;
  }
  if (q.state == FINISHING) {
    const hipError_t e = hipEventQuery(q.ev);
    if (e == hipErrorNotReady) return false;
    q.x.assign(q.pin_x, q.pin_x + q.rhs.size());
    q.state = q.code == STMG_OK || q.code == STMG_ENOTCONV ? DONE : FAILED;
    q.t_done = now_s();
    release(q);
    if (q.state == DONE) {
      completed++;
      latencies.push_back(q.t_done - q.t_submit);
      t_last_done = std::max(t_last_done, q.t_done);
      dof_updates += (double)q.dofs * (double)q.history.size();
    } else {
      failed++;
    }
    cv_done.notify_all();
    return true;
  }
  return false;
}

// Start copying the result out; on failure release the request at once.
void stmg_server::finish(Request &q, int code, const char *msg) {
  q.code = code;
  q.message = msg ? msg : "";
  if ((code == STMG_OK || code == STMG_ENOTCONV) && q.ev) {
    if (stmg_store(q.h, q.d_x) == STMG_OK &&
        hipMemcpyAsync(q.pin_x, q.d_x, q.rhs.size() * sizeof(double), hipMemcpyDeviceToHost, q.stream) ==
            hipSuccess &&
        hipEventRecord(q.ev, q.stream) == hipSuccess) {
      q.state = FINISHING;
      return;
    }
    q.code = STMG_EHIP;
    q.message = "result copy failed";
  }
  if (q.code == STMG_OK) q.code = STMG_EHIP;
  q.state = FAILED;
  q.t_done = now_s();
  release(q);
  failed++;
  cv_done.notify_all();
}

// Free the request's device resources on its stream and its reservation.
void stmg_server::release(Request &q) {
  if (q.h) {
    if (q.d_rhs) (void)hipFreeAsync(q.d_rhs, q.stream);
    if (q.d_u0) (void)hipFreeAsync(q.d_u0, q.stream);
    if (q.d_x) (void)hipFreeAsync(q.d_x, q.stream);
    internal::destroy(q.h);
    q.h = nullptr;
  }
  if (q.ev) (void)hipEventDestroy(q.ev);
  if (q.stream) (void)hipStreamDestroy(q.stream);
  if (q.pin_norm) (void)hipHostFree(q.pin_norm);
  if (q.pin_x) (void)hipHostFree(q.pin_x);
  q.ev = nullptr;
  q.stream = nullptr;
  q.pin_norm = q.pin_x = nullptr;
  q.d_rhs = q.d_u0 = q.d_x = nullptr;
  reserved -= q.est_bytes;
  std::vector<double>().swap(q.rhs);
  std::vector<double>().swap(q.u0);
}

// One iteration of a request alone, on its own stream.
void stmg_server::start_iteration(Request &q) {
  try {
    internal::iteration(q.h, q.h->d_scalar);
    hipc(hipMemcpyAsync(q.pin_norm, q.h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, q.stream), "copy");
    hipc(hipEventRecord(q.ev, q.stream), "hipEventRecord");
    q.in_flight = true;
  } catch (const StmgError &e) {
    finish(q, e.code, e.what());
  }
}

// Start the iterations that are due: requests of the same cycle shape in
// batches of up to 8 on a shared stream, the others alone. A request is due
// only when its previous iteration has completed, so it has no work in
// flight on any stream when a batch takes it.
void stmg_server::launch_iterations() {
  std::vector<Request *> due;
  for (auto &r : active)
    if (r->state == RUNNING && r->want_iteration) due.push_back(r.get());
  std::vector<bool> taken(due.size(), false);
  for (size_t a = 0; a < due.size(); ++a) {
    if (taken[a]) continue;
    taken[a] = true;
    std::vector<Request *> group{due[a]};
    if (opt.batch)
      for (size_t b = a + 1; b < due.size() && group.size() < (size_t)SOLVE_GROUP_MAX; ++b)
        if (!taken[b] && internal::batchable(due[a]->h, due[b]->h)) {
          taken[b] = true;
          group.push_back(due[b]);
        }
    for (Request *q : group) q->want_iteration = false;
    if (group.size() == 1) {
      start_iteration(*group[0]);
      continue;
    }
    hipStream_t s = batch_streams[next_batch_stream++ % batch_streams.size()];
    std::vector<stmg_handle *> hs;
    for (Request *q : group) hs.push_back(q->h);
    try {
      internal::batched_iteration(hs, s);
      for (Request *q : group) {
        hipc(hipMemcpyAsync(q->pin_norm, q->h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
        hipc(hipEventRecord(q->ev, s), "hipEventRecord");
        q->in_flight = true;
      }
      batched_iterations++;
      batched_members += (int64_t)group.size();
    } catch (const StmgError &e) {
      for (Request *q : group)
        if (!q->in_flight) finish(*q, e.code, e.what());
    }
  }
}

void stmg_server::scheduler_loop() {
  (void)hipSetDevice(device);  // as in worker_loop
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    bool moved = false;
    while (admit_one()) moved = true;
    for (auto &r : active) moved |= progress(*r);
    launch_iterations();
    active.erase(std::remove_if(active.begin(), active.end(),
                                [](const std::shared_ptr<Request> &r) { return r->state == DONE || r->state == FAILED; }),
                 active.end());
    if (!moved) {
      if (active.empty())
        cv_work.wait_for(lk, std::chrono::milliseconds(5));
      else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
    }
  }
}

// =================================================================== ABI
extern "C" {

void stmg_server_default_options(stmg_server_options *o) {
  if (!o) return;
  o->hbm_budget = 0;
  o->max_active = 16;
  o->setup_threads = 4;
  o->batch = 1;
}

int stmg_server_create(const stmg_server_options *opt, stmg_server **out) {
  if (!out) return STMG_EINVAL;
  *out = nullptr;
  auto *s = new stmg_server();
  if (opt)
    s->opt = *opt;
  else
    stmg_server_default_options(&s->opt);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return STMG_EHIP;
  }
  if (s->opt.hbm_budget <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return STMG_EHIP;
    }
    s->opt.hbm_budget = (int64_t)(0.9 * (double)free_b);
  }
  if (s->opt.max_active <= 0) s->opt.max_active = 16;
  if (s->opt.setup_threads <= 0) s->opt.setup_threads = 4;
  for (int i = 0; i < 4; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->batch_streams) (void)hipStreamDestroy(x);
      delete s;
      return STMG_EHIP;
    }
    s->batch_streams.push_back(st);
  }
  for (int i = 0; i < s->opt.setup_threads; ++i) s->workers.emplace_back([s] { s->worker_loop(); });
  s->scheduler = std::thread([s] { s->scheduler_loop(); });
  *out = s;
  return STMG_OK;
}

int stmg_submit(stmg_server *s, const stmg_problem *prob, const stmg_options *opt, const double *rhs_host,
                const double *u0_host, uint64_t *ticket) {
  if (!s || !prob || !rhs_host || !ticket) return STMG_EINVAL;
  auto r = std::make_shared<Request>();
  try {
    STMG_REQUIRE(prob->n_meshes >= 1 && prob->meshes, STMG_EINVAL, "no meshes");
    r->pc.take(*prob);
    if (opt)
      r->opt = *opt;
    else
      stmg_default_options(&r->opt);
    r->opt.host_only = 0;
    // the full-layout length needs the edge count: count edges of mesh 0 now
    const stmg_mesh &m = prob->meshes[0];
    std::vector<int64_t> keys;
    keys.reserve(6 * (size_t)m.n_tets);
    for (int32_t t = 0; t < m.n_tets; ++t) {
      int32_t v[4] = {m.tets[4 * t], m.tets[4 * t + 1], m.tets[4 * t + 2], m.tets[4 * t + 3]};
      std::sort(v, v + 4);
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) keys.push_back((int64_t)v[a] * m.n_vertices + v[b]);
    }
    std::sort(keys.begin(), keys.end());
    const int64_t E = std::unique(keys.begin(), keys.end()) - keys.begin();
    const int64_t n = E * prob->Nt * (prob->pt + 1);
    r->rhs.assign(rhs_host, rhs_host + n);
    if (u0_host) r->u0.assign(u0_host, u0_host + E);
  } catch (const StmgError &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    return STMG_ENOMEM;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  if (s->t_first_submit < 0) s->t_first_submit = r->t_submit;
  s->pending.push_back(r);
  s->all[r->ticket] = r;
  s->submitted++;
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return STMG_OK;
}

int stmg_poll(stmg_server *s, uint64_t ticket, double *x_host, stmg_report *rep) {
  if (!s) return STMG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return STMG_EINVAL;
  Request &r = *it->second;
  if (r.state != DONE && r.state != FAILED) return STMG_EAGAIN;
  if (x_host && !r.x.empty()) std::copy(r.x.begin(), r.x.end(), x_host);
  if (rep) {
    rep->cycles = (int32_t)r.history.size();
    rep->rel_res = r.history.empty() ? 0.0 : r.history.back();
    rep->setup_s = r.setup_s;
    rep->solve_s = r.t_done - r.t_admit;
    rep->res_history = nullptr;
  }
  const int code = r.code;
  s->all.erase(it);
  return code;
}

int stmg_server_wait(stmg_server *s, uint64_t ticket, double timeout_s) {
  if (!s) return STMG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return STMG_EINVAL;
  std::shared_ptr<Request> r = it->second;
  const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                      [&] { return r->state == DONE || r->state == FAILED; });
  return ok ? STMG_OK : STMG_EAGAIN;
}

int stmg_server_stats(stmg_server *s, stmg_server_stats_t *st) {
  if (!s || !st) return STMG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->active = (int64_t)s->active.size();
  st->pending = (int64_t)(s->pending.size() + s->ready.size()) + s->n_setting_up;
  std::vector<double> l = s->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double p) {
    if (l.empty()) return 0.0;
    const size_t i = (size_t)std::min<double>(l.size() - 1, std::ceil(p * l.size()) - 1);
    return l[i];
  };
  st->p50_s = pct(0.50);
  st->p99_s = pct(0.99);
  double sum = 0;
  for (double v : l) sum += v;
  st->mean_s = l.empty() ? 0.0 : sum / l.size();
  const double span = s->t_last_done - s->t_first_submit;
  st->throughput_req_s = span > 0 ? s->completed / span : 0.0;
  st->throughput_dofs = span > 0 ? s->dof_updates / span : 0.0;
  st->hbm_reserved = s->reserved;
  st->hbm_peak = s->peak;
  st->hbm_budget = s->opt.hbm_budget;
  st->batched_iterations = s->batched_iterations;
  st->batched_members = s->batched_members;
  return STMG_OK;
}

void stmg_server_destroy(stmg_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (auto &t : s->workers) t.join();
  if (s->scheduler.joinable()) s->scheduler.join();
  // drain and free whatever is still on the device or set up on the host
  for (auto x : s->batch_streams) (void)hipStreamSynchronize(x);
  for (auto &r : s->active) {
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    s->release(*r);
  }
  for (auto x : s->batch_streams) (void)hipStreamDestroy(x);
  for (auto &r : s->ready)
    if (r->h) internal::destroy(r->h);
  for (auto &r : s->admitted)
    if (r->h) internal::destroy(r->h);
  delete s;
}

}  // extern "C"
