// Request server: continuous batching of solve requests on one device.
//
// A request names a resident mechanism and device-resident state/environment of any cell
// count. Requests wait in a FIFO; one admission thread takes them in order: it resolves the
// request's launch (autotuning a cold (mechanism, size) bucket, with the trials' scratch
// reserved against the budget while they run), computes the request's device footprint for
// that launch, waits until the footprint fits the budget and a stream slot is free, and
// enqueues the solve on the slot's HIP stream. Tuning and launching happen outside the
// server lock, so submit / poll / progress never wait on a launch. Each admitted request is
// one fused-engine solve (a persistent kernel that pulls the request's cells from its
// queue), so several requests' kernels are resident together and the hardware dispatcher
// fills CUs freed by one request with workgroups of another. The same thread retires
// finished requests (event query) and reads their failed-cell counts.
// Each cell is solved exactly as by camp_solve_device: no arithmetic crosses cells or
// requests, so a request's result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.hpp"

using namespace camp;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  long long ticket;
  camp_mech* mech;
  int n_cells;
  double* d_state;
  camp_env env;
  double dt, rtol, atol;
  camp_opts opts;
  bool has_opts;
  int* d_status;
  size_t footprint = 0;
  Clock::time_point t_submit, t_done;
  int slot = -1;
  bool done = false;
  int n_failed = 0;
  int rc = CAMP_OK;
};

}  // namespace

struct camp_server {
  int device = 0;
  long long budget = 0;
  long long in_use = 0;
  int n_slots = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<long long> slot_ticket;   // 0: free; > 0: request in flight; < 0: held by
                                        // the admission thread (trials or an enqueue)
  int* pinned = nullptr;                // [n_slots] failed counts
  int* d_counts = nullptr;              // [n_slots] device failed counts
  std::mutex mu;
  std::condition_variable cv;           // a request finished
  std::deque<long long> pending;
  long long admitting = 0;              // ticket taken from the FIFO, not yet launched
  std::map<long long, Request> reqs;
  long long next_ticket = 1;
  std::atomic<bool> stop{false};
  std::thread worker;
};

namespace {

// Bytes of a request's own device arrays (state, environment, status).
size_t array_bytes(const camp_mech* mh, int n_cells) {
  const Compiled& C = mh->C;
  const size_t per_cell = 8 * ((size_t)C.n_state + 3 + 2 * (size_t)C.n_inst + C.n_ext) + 4;
  return per_cell * (size_t)n_cells;
}

// Retire finished requests. Caller holds srv->mu. Returns whether any finished.
bool retire_locked(camp_server* srv) {
  bool any = false;
  for (int s = 0; s < srv->n_slots; ++s) {
    const long long t = srv->slot_ticket[s];
    if (t <= 0) continue;
    if (hipEventQuery(srv->events[s]) != hipSuccess) continue;
    Request& r = srv->reqs[t];
    r.done = true;
    r.t_done = Clock::now();
    r.n_failed = srv->pinned[s];
    srv->in_use -= (long long)r.footprint;
    srv->slot_ticket[s] = 0;
    any = true;
  }
  return any;
}

// Blocks (retiring finished requests meanwhile) until `bytes` fit the budget, or nothing is
// in flight (a lone request always runs), and, with want_slot, a stream slot is free; then
// reserves the bytes. Returns the slot (or 0 without want_slot), -1 when stopping.
int reserve(camp_server* srv, size_t bytes, bool want_slot) {
  while (!srv->stop.load()) {
    bool finished;
    int slot = -1;
    {
      std::lock_guard<std::mutex> g(srv->mu);
      finished = retire_locked(srv);
      if (want_slot)
        for (int s = 0; s < srv->n_slots && slot < 0; ++s)
          if (!srv->slot_ticket[s]) slot = s;
      const bool fits = srv->in_use + (long long)bytes <= srv->budget || srv->in_use == 0;
      if (fits && (slot >= 0 || !want_slot)) {
        srv->in_use += (long long)bytes;
        return want_slot ? slot : 0;
      }
    }
    if (finished) srv->cv.notify_all();
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  return -1;
}

void finish_failed(camp_server* srv, Request& r, int rc) {
  {
    std::lock_guard<std::mutex> g(srv->mu);
    r.rc = rc;
    r.done = true;
    r.t_done = Clock::now();
    r.n_failed = r.n_cells;
    srv->admitting = 0;
  }
  srv->cv.notify_all();
}

// Resolve, size and launch the request at the head of the FIFO.
void admit(camp_server* srv, Request& r) {
  camp_mech* mh = r.mech;
  const camp_opts* opts = r.has_opts ? &r.opts : nullptr;
  int rc = check_solve_args(mh, r.n_cells, r.d_state, &r.env, r.dt, r.rtol, r.atol);
  const DevMech* dm = nullptr;
  if (rc == CAMP_OK) rc = resident(mh, &dm);
  if (rc != CAMP_OK) return finish_failed(srv, r, rc);
  const SolveParams sp = make_params(r.dt, r.rtol, r.atol, opts);
  const size_t arrays = array_bytes(mh, r.n_cells);
  Tuning tu;
  const bool forced = opts && opts->engine != CAMP_ENGINE_AUTO;
  if (r.n_cells > 0 && !forced && !cached_tuning(mh, *dm, r.n_cells, sp, &tu)) {
    // cold bucket: the trials run on a free slot's stream, with their scratch (and the
    // request's arrays) reserved against the budget while they run
    const size_t trial = arrays + autotune_scratch_bytes(*dm, r.n_cells);
    const int slot = reserve(srv, trial, true);
    if (slot < 0) return finish_failed(srv, r, CAMP_EINVAL);
    {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->slot_ticket[slot] = -r.ticket;   // held by the trials
    }
    rc = resolve_tuning(mh, *dm, r.n_cells, r.d_state, &r.env, sp, opts, srv->streams[slot], true, &tu);
    {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->slot_ticket[slot] = 0;
      srv->in_use -= (long long)trial;
    }
    if (rc != CAMP_OK) return finish_failed(srv, r, rc);
  } else if (r.n_cells > 0) {
    rc = resolve_tuning(mh, *dm, r.n_cells, r.d_state, &r.env, sp, opts, nullptr, false, &tu);
    if (rc != CAMP_OK) return finish_failed(srv, r, rc);
  }
  r.footprint = arrays + (r.n_cells > 0 ? solve_scratch_bytes(*dm, tu, r.n_cells,
                                                              opts && opts->cell_order) : 0);
  const int slot = reserve(srv, r.footprint, true);
  if (slot < 0) return finish_failed(srv, r, CAMP_EINVAL);
  hipStream_t st = srv->streams[slot];
  r.slot = slot;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->slot_ticket[slot] = -r.ticket;   // reserved while the launch is enqueued
  }
  rc = r.n_cells > 0 ? solve_device_tuned(mh, *dm, r.n_cells, r.d_state, &r.env, sp, opts,
                                          r.d_status, nullptr, st, tu)
                     : CAMP_OK;
  hipError_t e = hipSuccess;
  if (rc == CAMP_OK) {
    e = launch_count_failed(r.n_cells, r.d_status, srv->d_counts + slot, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(srv->pinned + slot, srv->d_counts + slot, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(srv->events[slot], st);
    if (e != hipSuccess) rc = hip_fail(e, "server completion record");
  }
  if (rc != CAMP_OK) {
    // nothing of this request is left in flight that the slot must wait for
    hipStreamSynchronize(st);
    {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->slot_ticket[slot] = 0;
      srv->in_use -= (long long)r.footprint;
    }
    return finish_failed(srv, r, rc);
  }
  std::lock_guard<std::mutex> g(srv->mu);
  srv->slot_ticket[slot] = r.ticket;
  srv->admitting = 0;
}

void worker_loop(camp_server* srv) {
  hipSetDevice(srv->device);
  while (!srv->stop.load()) {
    Request* r = nullptr;
    bool finished;
    {
      std::lock_guard<std::mutex> g(srv->mu);
      finished = retire_locked(srv);
      if (!srv->pending.empty()) {
        srv->admitting = srv->pending.front();
        srv->pending.pop_front();
        r = &srv->reqs[srv->admitting];   // std::map: stable while other entries are added
      }
    }
    if (finished) srv->cv.notify_all();
    if (r) {
      admit(srv, *r);
      continue;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace

extern "C" {

int camp_serve_create(long long max_bytes, int max_inflight, camp_server** out) {
  if (!out || max_inflight < 1 || max_inflight > 64 || max_bytes < 0) {
    set_error("camp_serve_create: bad argument");
    return CAMP_EINVAL;
  }
  camp_server* srv = new camp_server();
  hipGetDevice(&srv->device);
  size_t free_b = 0, total_b = 0;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) {
    delete srv;
    return hip_fail(e, "hipMemGetInfo");
  }
  srv->budget = max_bytes > 0 ? max_bytes : (long long)(free_b / 2);
  srv->n_slots = max_inflight;
  srv->streams.resize(max_inflight);
  srv->events.resize(max_inflight);
  srv->slot_ticket.assign(max_inflight, 0);
  for (int s = 0; s < max_inflight; ++s) {
    if ((e = hipStreamCreateWithFlags(&srv->streams[s], hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&srv->events[s], hipEventDisableTiming)) != hipSuccess) {
      delete srv;
      return hip_fail(e, "server stream/event");
    }
  }
  if ((e = hipHostMalloc((void**)&srv->pinned, sizeof(int) * max_inflight, hipHostMallocDefault)) != hipSuccess ||
      (e = hipMalloc((void**)&srv->d_counts, sizeof(int) * max_inflight)) != hipSuccess) {
    delete srv;
    return hip_fail(e, "server buffers");
  }
  srv->worker = std::thread(worker_loop, srv);
  *out = srv;
  return CAMP_OK;
}

int camp_serve_submit(camp_server* srv, camp_mech* mech, int n_cells, double* d_state,
                      const camp_env* d_env, double dt, double rtol, double atol,
                      const camp_opts* opts, int* d_cell_status, long long* ticket) {
  if (!srv || !mech || !ticket || !d_env || n_cells < 0 || (n_cells > 0 && (!d_state || !d_cell_status))) {
    set_error("camp_serve_submit: bad argument");
    return CAMP_EINVAL;
  }
  if (!(dt > 0) || !(rtol > 0) || !(atol >= 0)) {
    set_error("camp_serve_submit: dt and rtol must be positive, atol >= 0");
    return CAMP_EINVAL;
  }
  std::lock_guard<std::mutex> g(srv->mu);
  Request r;
  r.ticket = srv->next_ticket++;
  r.mech = mech;
  r.n_cells = n_cells;
  r.d_state = d_state;
  r.env = *d_env;
  r.dt = dt;
  r.rtol = rtol;
  r.atol = atol;
  r.has_opts = opts != nullptr;
  if (opts) r.opts = *opts;
  r.d_status = d_cell_status;
  r.t_submit = Clock::now();
  srv->reqs[r.ticket] = r;
  srv->pending.push_back(r.ticket);
  *ticket = r.ticket;
  return CAMP_OK;
}

int camp_serve_poll(camp_server* srv, long long ticket, int* done, int* n_failed, double* latency_s) {
  if (!srv || !done) {
    set_error("camp_serve_poll: bad argument");
    return CAMP_EINVAL;
  }
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_error("camp_serve_poll: unknown ticket");
    return CAMP_EINVAL;
  }
  const Request& r = it->second;
  *done = r.done ? 1 : 0;
  if (n_failed) *n_failed = r.done ? r.n_failed : 0;
  if (latency_s)
    *latency_s = r.done ? std::chrono::duration<double>(r.t_done - r.t_submit).count() : 0.0;
  return r.done ? r.rc : CAMP_OK;
}

int camp_serve_wait(camp_server* srv, long long ticket) {
  if (!srv) {
    set_error("camp_serve_wait: bad argument");
    return CAMP_EINVAL;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_error("camp_serve_wait: unknown ticket");
    return CAMP_EINVAL;
  }
  srv->cv.wait(lk, [&] { return srv->reqs[ticket].done; });
  return srv->reqs[ticket].rc;
}

int camp_serve_progress(camp_server* srv, int* inflight, int* queued) {
  if (!srv) {
    set_error("camp_serve_progress: bad argument");
    return CAMP_EINVAL;
  }
  std::lock_guard<std::mutex> g(srv->mu);
  int n = 0;
  for (long long t : srv->slot_ticket) n += t > 0;
  if (srv->admitting) ++n;
  if (inflight) *inflight = n;
  if (queued) *queued = (int)srv->pending.size();
  return CAMP_OK;
}

void camp_serve_destroy(camp_server* srv) {
  if (!srv) return;
  srv->stop.store(true);
  if (srv->worker.joinable()) srv->worker.join();
  for (size_t s = 0; s < srv->streams.size(); ++s) {
    if (srv->streams[s]) {
      hipStreamSynchronize(srv->streams[s]);
      hipStreamDestroy(srv->streams[s]);
    }
    if (srv->events[s]) hipEventDestroy(srv->events[s]);
  }
  if (srv->pinned) hipHostFree(srv->pinned);
  if (srv->d_counts) hipFree(srv->d_counts);
  delete srv;
}

}  // extern "C"
