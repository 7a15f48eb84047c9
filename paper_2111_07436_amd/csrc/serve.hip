// Request server: continuous batching of solve requests on one device.
//
// A request names a resident mechanism and device-resident state/environment of any cell
// count. Requests wait in a FIFO until their device-memory footprint fits the budget and a
// stream slot is free; each admitted request is enqueued on its own HIP stream as one
// fused-engine solve (a persistent kernel that pulls the request's cells from its queue),
// so several requests' kernels are resident together and the hardware dispatcher fills
// CUs freed by one request with workgroups of another. A progress thread retires finished
// requests (event query), reads their failed-cell counts and admits waiting ones.
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
  size_t footprint;
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
  std::vector<long long> slot_ticket;   // 0: free
  int* pinned = nullptr;                // [n_slots] failed counts
  int* d_counts = nullptr;              // [n_slots] device failed counts
  std::mutex mu;
  std::condition_variable cv;
  std::deque<long long> pending;
  std::map<long long, Request> reqs;
  long long next_ticket = 1;
  std::atomic<bool> stop{false};
  std::thread worker;
};

namespace {

// Device bytes a request occupies while in flight: its resident arrays plus the engine's
// scratch (the lane engines carry per-cell slabs; the wavefront engine only a counter).
size_t footprint(const camp_mech* mh, int n_cells, const camp_opts* o) {
  const Compiled& C = mh->C;
  size_t per_cell = 8 * ((size_t)C.n_state + 3 + 2 * (size_t)C.n_inst + C.n_ext) + 4;
  size_t bytes = per_cell * (size_t)n_cells + 4096;
  const int engine = o ? o->engine : CAMP_ENGINE_AUTO;
  if (engine == CAMP_ENGINE_PLAIN || engine == CAMP_ENGINE_FUSED_LANE) {
    const size_t np = std::max<size_t>(C.n_partials, C.n_rxn);
    bytes += 8 * ((size_t)C.n_rxn + np + C.nnz + 14 * (size_t)C.n_state + 16) * (size_t)n_cells;
  }
  return bytes;
}

// Retire finished requests and admit waiting ones. Caller holds srv->mu.
void pump_locked(camp_server* srv) {
  for (int s = 0; s < srv->n_slots; ++s) {
    const long long t = srv->slot_ticket[s];
    if (!t) continue;
    if (hipEventQuery(srv->events[s]) != hipSuccess) continue;
    Request& r = srv->reqs[t];
    r.done = true;
    r.t_done = Clock::now();
    r.n_failed = srv->pinned[s];
    srv->in_use -= (long long)r.footprint;
    srv->slot_ticket[s] = 0;
  }
  while (!srv->pending.empty()) {
    Request& r = srv->reqs[srv->pending.front()];
    int slot = -1;
    for (int s = 0; s < srv->n_slots; ++s)
      if (!srv->slot_ticket[s]) {
        slot = s;
        break;
      }
    const bool fits = srv->in_use + (long long)r.footprint <= srv->budget ||
                      srv->in_use == 0;   // a lone request always runs
    if (slot < 0 || !fits) break;
    srv->pending.pop_front();
    hipStream_t st = srv->streams[slot];
    r.slot = slot;
    r.rc = camp_solve_device(r.mech, r.n_cells, r.d_state, &r.env, r.dt, r.rtol, r.atol,
                             r.has_opts ? &r.opts : nullptr, r.d_status, nullptr, st);
    if (r.rc == CAMP_OK) {
      launch_count_failed(r.n_cells, r.d_status, srv->d_counts + slot, st);
      hipMemcpyAsync(srv->pinned + slot, srv->d_counts + slot, sizeof(int), hipMemcpyDeviceToHost, st);
      hipEventRecord(srv->events[slot], st);
      srv->slot_ticket[slot] = r.ticket;
      srv->in_use += (long long)r.footprint;
    } else {
      r.done = true;
      r.t_done = Clock::now();
      r.n_failed = r.n_cells;
    }
  }
}

void worker_loop(camp_server* srv) {
  hipSetDevice(srv->device);
  while (!srv->stop.load()) {
    {
      std::lock_guard<std::mutex> g(srv->mu);
      pump_locked(srv);
    }
    srv->cv.notify_all();
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
  r.footprint = footprint(mech, n_cells, opts);
  r.t_submit = Clock::now();
  srv->reqs[r.ticket] = r;
  srv->pending.push_back(r.ticket);
  *ticket = r.ticket;
  pump_locked(srv);
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
  pump_locked(srv);
  int n = 0;
  for (long long t : srv->slot_ticket) n += t != 0;
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
