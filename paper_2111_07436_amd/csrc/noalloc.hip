// Device solve that allocates nothing: for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The fused wavefront engine needs a little scratch per launch (queue counter and flags,
// the rate-constant scratch of launch modes 3/4, the per-cell counters of a cell-order
// check). Here it lives in a fixed file-scope device array, one copy per GPU, held until the
// process ends. Host code never passes the array's name to a kernel (on the host it is only
// a stand-in for the symbol): the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "runtime.hpp"

namespace camp {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB per GPU

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, char*> g_scratch;   // device id -> address of that device's `scratch`

// The current device's copy of `scratch` (looked up on the first call on each device).
int scratch_address(char** out) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    it = g_scratch.emplace(device, static_cast<char*>(p)).first;
  }
  *out = it->second;
  return CAMP_OK;
}

}  // namespace
}  // namespace camp

using namespace camp;

extern "C" {

size_t camp_noalloc_scratch_bytes(void) { return kScratchBytes; }

int camp_solve_device_noalloc(camp_mech* mh, int n_cells, double* d_state, const camp_env* d_env,
                              double dt, double rtol, double atol, const camp_opts* opts,
                              int* d_cell_status, camp_cell_stats* d_cell_stats, void* stream) {
  int rc = check_solve_args(mh, n_cells, d_state, d_env, dt, rtol, atol);
  if (rc != CAMP_OK) return rc;
  if (n_cells > 0 && !d_cell_status) { set_error("d_cell_status is required"); return CAMP_EINVAL; }
  if (n_cells == 0) return CAMP_OK;
  char* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != CAMP_OK) return rc;
  const DevMech* dm = resident_if_uploaded(mh);
  if (!dm) {
    set_error("mechanism tables are not resident on this device: run camp_solve_device or "
              "camp_plan_create with it on this device first");
    return CAMP_EINVAL;
  }
  const SolveParams sp = make_params(dt, rtol, atol, opts);
  Tuning tu;
  rc = resolve_tuning(mh, *dm, n_cells, d_state, d_env, sp, opts, (hipStream_t)stream, false, &tu);
  if (rc != CAMP_OK) return rc;
  if (tu.engine != CAMP_ENGINE_FUSED_WAVE) {
    set_error("the no-allocation solve runs the fused wavefront engine (engine AUTO or FUSED_WAVE)");
    return CAMP_EINVAL;
  }
  const int* order = opts ? opts->cell_order : nullptr;
  WaveShape w;
  rc = wave_launch_shape(*dm, tu, n_cells, order != nullptr, &w);
  if (rc != CAMP_OK) return rc;
  if (w.bytes > kScratchBytes) {
    set_error("this solve needs " + std::to_string(w.bytes) + " bytes of scratch, more than the " +
              std::to_string(kScratchBytes) + " the no-allocation entry point holds");
    return CAMP_EINVAL;
  }
  hipError_t e = enqueue_wave(*dm, make_env(d_env), d_state, n_cells, sp, order, d_cell_status,
                              d_cell_stats, w, ws, false, (hipStream_t)stream);
  return e == hipSuccess ? CAMP_OK : hip_fail(e, "solve launch");
}

}  // extern "C"
