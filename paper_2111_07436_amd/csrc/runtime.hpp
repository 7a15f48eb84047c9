// Host runtime: mechanism residency on the device, workspaces, engine launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "camp.h"
#include "device.hpp"
#include "mech.hpp"

namespace camp {

struct LaneCtx;

// Tunable launch choice for one (mechanism, cell-count bucket).
struct Tuning {
  int engine = CAMP_ENGINE_FUSED_WAVE;
  int persistent = 1;        // wave engine: 1 = queue-driven persistent grid
  int grid_mult = 8;         // wave engine: workgroups per CU when persistent
  int waves = 1;             // wave engine: wavefronts (cells) per workgroup
  int lanes = 64;            // wave engine: lanes per cell (64: one wavefront; 128, 256: a
                             // whole workgroup per cell)
  int stage = 1;             // wave engine launch mode: tables staged in LDS (0 none, 1 index,
                             // 2 all); 3 / 4 as 0 / 1 with rate constants in global scratch
  double ms = 0.0;           // measured trial time
};

// Launch shape and scratch bytes of one fused wavefront launch (see wave_launch_shape).
struct WaveShape {
  int lanes = 64, waves = 1, stage = 0, grid = 1;
  bool persistent = true;
  size_t kc_bytes = 0, seen_bytes = 0, bytes = 0;
};

// Device scratch reused by the fused launches of one (mechanism, device, stream).
struct Workspace {
  char* ptr = nullptr;
  size_t bytes = 0;
};

struct DeviceTables {
  int device = -1;
  void* blob = nullptr;
  size_t bytes = 0;
  DevMech dm{};
};

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Launchers (defined in the engine files).
size_t wave_lds_bytes(const DevMech& m);
size_t wave_cell_bytes(const DevMech& m);
size_t wave_wg_lds_bytes(const DevMech& m, int waves, int stage, int lanes);
int wave_max_waves(int n_state, int mode, int lanes);
int wave_lanes_ok(int n_state, int lanes);
// The launch mode a wavefront launch of mechanism m in mode `mode` (0..4) runs in: the
// parameter mode (as mode 3, with the Parameter passes) for mechanisms with Parameters.
int wave_effective_mode(const DevMech& m, int mode);
int wave_resident_cells_per_cu(int n_state, int mode, int lanes);
// attr_only: set the kernel's launch attributes (LDS size) and return without launching.
hipError_t launch_bdf_wave(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                           const SolveParams& sp, int* status, camp_cell_stats* stats, int* queue,
                           double* kc_glob, int grid, int waves, int stage, int lanes,
                           bool attr_only, hipStream_t stream);
constexpr size_t kLdsBytes = 160 * 1024;
hipError_t launch_wave_step(const DevMech& m, int op, int n_cells, const double* kin,
                            const double* yin, double* out, double gamma, hipStream_t stream);
hipError_t launch_rates_step(const DevMech& m, const DevEnv& env, int n_cells, double* k_out,
                             hipStream_t stream);
hipError_t run_plain(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                     const SolveParams& sp, int* status, camp_cell_stats* stats, int use_graph,
                     hipStream_t stream);
hipError_t run_fused_lane(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                          const SolveParams& sp, int* status, camp_cell_stats* stats,
                          int n_slots, hipStream_t stream);
hipError_t launch_count_failed(int n, const int* status, int* out, hipStream_t stream);
// Device scratch one lane-engine call allocates (for the call's duration): n_slots = 0 for
// the plain engine, else the fused engine's slot count.
size_t lane_scratch_bytes(const DevMech& m, int n_cells, int n_slots);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t stream);
// Zeroes seen[0..n) and raises *bad (not cleared here) unless order[0..n) is a permutation.
hipError_t launch_check_order(const int* order, int n, int* seen, int* bad, hipStream_t stream);

// Solve plumbing shared by the entry points (api.hip).
int check_solve_args(camp_mech* mh, int n_cells, const void* state, const camp_env* env,
                     double dt, double rtol, double atol);
SolveParams make_params(double dt, double rtol, double atol, const camp_opts* o);
DevEnv make_env(const camp_env* e);
int resident(camp_mech* mh, const DevMech** dm);
const DevMech* resident_if_uploaded(camp_mech* mh);
int resolve_tuning(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
                   const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
                   hipStream_t stream, bool run_trials, Tuning* out);
bool cached_tuning(camp_mech* mh, const DevMech& dm, int n_cells, const SolveParams& sp,
                   Tuning* out);
// Device bytes the autotuner's trials allocate for a call of n_cells (freed when it returns).
size_t autotune_scratch_bytes(const DevMech& dm, int n_cells);
// Device bytes a solve with tuning `tu` uses beyond its inputs and outputs: the lane
// engines' per-call slabs, or the fused wavefront launch's stream workspace (cached per
// mechanism and stream, at least 1 MiB once allocated).
size_t solve_scratch_bytes(const DevMech& dm, const Tuning& tu, int n_cells, bool has_order);
int solve_device_tuned(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
                       const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
                       int* d_status, camp_cell_stats* d_stats, hipStream_t stream, const Tuning& tu);
int wave_launch_shape(const DevMech& dm, const Tuning& tu, int n_cells, bool has_order,
                      WaveShape* out);
hipError_t enqueue_wave(const DevMech& dm, const DevEnv& env, double* d_state, int n_cells,
                        const SolveParams& sp, const int* order, int* d_status,
                        camp_cell_stats* d_stats, const WaveShape& w, char* ws, bool attr_only,
                        hipStream_t stream);

}  // namespace camp

struct camp_mech {
  camp::Compiled C;
  // term lists for 1, 2 and 4 wavefronts per cell (with the dense tail), and for one
  // wavefront without it (the single-step kernels, which return conventional factors)
  camp::StageBlock stage[4];
  std::mutex mu;
  std::map<int, camp::DeviceTables> dev;            // per device id
  std::map<std::pair<int, int>, camp::Tuning> tune; // (device, cell bucket)
  std::map<std::pair<int, void*>, camp::Workspace> ws;   // (device, stream)
};
