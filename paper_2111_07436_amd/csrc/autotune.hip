// Autotuner: picks the engine and launch shape per (mechanism, device, cell-count bucket).
//
// On the first call for a bucket it times short trials of each candidate on a copy of the
// call's own first cells (the caller's arrays are never written by a trial) and caches
// the fastest. Candidates: the wavefront engine with one wavefront or one workgroup per
// cell, in each launch mode (table staging, rate constants in LDS or in global scratch), at
// the cells per workgroup that keep the most cells resident, with a persistent grid sized to that capacity or one workgroup per cell
// batch; the lane-per-cell fused engine only when no wavefront launch fits. With
// CAMP_TUNE_CACHE set to a file path, choices persist across processes (keyed by a hash of
// the compiled mechanism, the device name and the bucket).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "runtime.hpp"

namespace camp {

Tuning default_tuning(const DevMech& dm, int n_cells);

namespace {

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t mech_hash(const camp_mech* mh) {
  const Compiled& C = mh->C;
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &C.n_state, sizeof(int));
  h = fnv(h, &C.n_rxn, sizeof(int));
  for (const auto& sb : mh->stage) h = fnv(h, sb.bytes.data(), sb.bytes.size());
  for (const RateSpec& r : C.rate) h = fnv(h, &r, sizeof(RateSpec));
  h = fnv(h, C.term_coef.data(), 8 * C.term_coef.size());
  return h;
}

std::string device_name() {
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  for (char& c : s)
    if (c == ' ') c = '_';
  return s;
}

std::string cache_key(const camp_mech* mh, int bucket, const SolveParams& sp) {
  std::ostringstream k;
  k << std::hex << mech_hash(mh) << std::dec << ' ' << device_name() << ' ' << bucket << ' '
    << sp.full_newton;
  return k.str();
}

bool load_cached(const std::string& key, Tuning* t) {
  const char* path = std::getenv("CAMP_TUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != '|')
      continue;
    std::istringstream v(line.substr(key.size() + 1));
    Tuning x;
    if (v >> x.engine >> x.persistent >> x.grid_mult >> x.waves >> x.stage >> x.lanes >> x.ms) {
      *t = x;
      found = true;   // last entry wins
    }
  }
  return found;
}

void store_cached(const std::string& key, const Tuning& t) {
  const char* path = std::getenv("CAMP_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << '|' << t.engine << ' ' << t.persistent << ' ' << t.grid_mult << ' ' << t.waves << ' '
    << t.stage << ' ' << t.lanes << ' ' << t.ms << '\n';
}

int n_cus_dev() {
  int dev = 0, cus = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

std::vector<Tuning> candidates(const DevMech& dm) {
  std::vector<Tuning> out;
  const bool wave_ok = wave_lanes_ok(dm.N, 64) && dm.stage;
  if (wave_ok) {
    // per lanes-per-cell and launch mode, the cells per workgroup that keep the most cells
    // resident per CU (ties: the larger workgroup); persistent, and for one wavefront per
    // cell with rate constants in LDS also one workgroup per cell batch
    for (int lanes : {64, 128, 256}) {
      if (!wave_lanes_ok(dm.N, lanes) || !dm.sv[lanes / 128].base) continue;
      for (int stage : {2, 1, 0, 4, 3}) {
        // mechanisms with Parameters run every launch in one mode (see wave_effective_mode)
        if (wave_effective_mode(dm, stage) != stage && stage != 3) continue;
        const int wmax = wave_max_waves(dm.N, stage, lanes);
        const int cap = wave_resident_cells_per_cu(dm.N, stage, lanes);
        Tuning best;
        int best_cells = 0;
        for (int w = 1; w <= wmax; ++w) {
          const size_t b = wave_wg_lds_bytes(dm, w, stage, lanes);
          if (b > kLdsBytes) break;
          const int wgs = (int)(kLdsBytes / b);   // resident workgroups per CU by LDS
          const int cells = std::min(wgs * w, cap);
          if (cells >= best_cells) {
            best_cells = cells;
            best.engine = CAMP_ENGINE_FUSED_WAVE;
            best.lanes = lanes;
            best.waves = w;
            best.stage = stage;
            best.persistent = 1;
            best.grid_mult = std::max(1, std::min(wgs, std::max(1, cap / w)));
          }
        }
        if (best_cells == 0) continue;
        out.push_back(best);
        if (lanes == 64 && stage <= 2) {
          Tuning np = best;
          np.persistent = 0;
          out.push_back(np);
        }
      }
    }
  }
  // The lane-per-cell engine (matrix in HBM) only when no wavefront launch fits.
  if (out.empty()) {
    Tuning lane;
    lane.engine = CAMP_ENGINE_FUSED_LANE;
    out.push_back(lane);
  }
  return out;
}

}  // namespace

namespace {
int size_bucket(int n_cells) { return n_cells <= 1 ? 0 : (int)std::ceil(std::log2((double)n_cells)); }
}  // namespace

bool cached_tuning(camp_mech* mh, const DevMech& dm, int n_cells, const SolveParams& sp,
                   Tuning* out) {
  (void)dm;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return false;
  std::lock_guard<std::mutex> g(mh->mu);
  auto it = mh->tune.find(std::make_pair(device, size_bucket(n_cells) * 2 + sp.full_newton));
  if (it == mh->tune.end()) return false;
  *out = it->second;
  return true;
}

namespace {
// Trial sizes: enough cells for several per resident slot, and four times that for the
// throughput round of a large call.
int trial_cells(int n_cells) { return std::min(n_cells, std::max(4096, n_cus_dev() * 64)); }
}  // namespace

size_t autotune_scratch_bytes(const DevMech& dm, int n_cells) {
  const int big = std::min(n_cells, 4 * trial_cells(n_cells));
  return 2 * sizeof(double) * (size_t)big * dm.N + 4 * (size_t)big + 256;
}

int autotuned(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
              const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
              hipStream_t stream, Tuning* out) {
  int device = 0;
  hipGetDevice(&device);
  const int bucket = size_bucket(n_cells);
  const auto key = std::make_pair(device, bucket * 2 + sp.full_newton);
  {
    std::lock_guard<std::mutex> g(mh->mu);
    auto it = mh->tune.find(key);
    if (it != mh->tune.end()) {
      *out = it->second;
      return CAMP_OK;
    }
  }
  const std::string ckey = cache_key(mh, bucket, sp);
  Tuning best;
  if (load_cached(ckey, &best)) {
    std::lock_guard<std::mutex> g(mh->mu);
    mh->tune[key] = best;
    *out = best;
    return CAMP_OK;
  }

  // Trial on a copy of the first cells of this call: enough cells for several per resident
  // slot. Then, for a larger call, the three fastest launches run again on four times as
  // many cells: near the trial size the lowest per-cell latency wins (the last cells finish
  // alone), while a large call is decided by throughput.
  const int trial = trial_cells(n_cells);
  const int big = std::min(n_cells, 4 * trial);
  const size_t sbytes = sizeof(double) * (size_t)big * dm.N;
  char* buf = nullptr;
  hipError_t e = hipMallocAsync((void**)&buf, autotune_scratch_bytes(dm, n_cells), stream);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(autotune)");
  double* src = reinterpret_cast<double*>(buf);
  double* work = reinterpret_cast<double*>(buf + sbytes);
  int* st = reinterpret_cast<int*>(buf + 2 * sbytes);
  e = hipMemcpyAsync(src, d_state, sbytes, hipMemcpyDeviceToDevice, stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  best = default_tuning(dm, n_cells);
  best.ms = 1e30;
  // trials take cells in index order (a caller's cell order spans the whole call)
  camp_opts topts{};
  if (opts) topts = *opts;
  topts.cell_order = nullptr;
  // up to `reps` timed runs of launch t on identical copies of the first n cells (min); a
  // launch far slower than `bound` is not run again. Returns a negative time if t cannot
  // be launched for this mechanism.
  auto timed = [&](const Tuning& t, int n, int reps, float bound) -> float {
    float best_ms = 1e30f;
    for (int rep = 0; rep < reps; ++rep) {
      if (hipMemcpyAsync(work, src, sizeof(double) * (size_t)n * dm.N, hipMemcpyDeviceToDevice,
                         stream) != hipSuccess)
        return -1.f;
      hipEventRecord(a, stream);
      int rc = solve_device_tuned(mh, dm, n, work, d_env, sp, &topts, st, nullptr, stream, t);
      hipEventRecord(b, stream);
      if (hipEventSynchronize(b) != hipSuccess) rc = CAMP_EDEVICE;
      if (rc != CAMP_OK) return -1.f;
      float ms = 0.f;
      hipEventElapsedTime(&ms, a, b);
      best_ms = std::min(best_ms, ms);
      if (ms > 2.0f * bound) break;
    }
    return best_ms;
  };
  std::vector<Tuning> ranked;
  if (e == hipSuccess) {
    for (Tuning t : candidates(dm)) {
      const float ms = timed(t, trial, 2, (float)best.ms);
      if (ms < 0.f) continue;   // candidate not launchable for this mechanism
      t.ms = ms;
      ranked.push_back(t);
      if (t.ms < best.ms) best = t;
    }
  }
  if (big > trial && ranked.size() > 1) {
    std::sort(ranked.begin(), ranked.end(),
              [](const Tuning& x, const Tuning& y) { return x.ms < y.ms; });
    ranked.resize(std::min<size_t>(ranked.size(), 3));
    best.ms = 1e30;
    for (Tuning t : ranked) {
      const float ms = timed(t, big, 1, 1e30f);
      if (ms < 0.f) continue;
      t.ms = ms;
      if (t.ms < best.ms) best = t;
    }
    if (best.ms >= 1e30) best = ranked.front();
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFreeAsync(buf, stream);
  hipStreamSynchronize(stream);
  if (best.ms >= 1e30) {
    best = default_tuning(dm, n_cells);
    best.ms = 0.0;
  } else {
    store_cached(ckey, best);
  }
  std::lock_guard<std::mutex> g(mh->mu);
  mh->tune[key] = best;
  *out = best;
  return CAMP_OK;
}

}  // namespace camp
