// C ABI: mechanism lifecycle, device residency, solve dispatch, single-step entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "camp.h"
#include "bdf_common.hpp"
#include "runtime.hpp"

namespace camp {

namespace {
thread_local std::string g_err;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Copies every table of the compiled mechanism into one device allocation.
int upload(camp_mech* mh, int device, DeviceTables& out) {
  const Compiled& C = mh->C;
  struct Item {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Item> items;
  size_t total = 0;
  auto add = [&](const void* src, size_t bytes) {
    items.push_back({src, bytes, total});
    size_t off = total;
    total = align256(total + std::max<size_t>(bytes, 1));
    return off;
  };
  const int R = C.n_rxn;
  std::vector<int> kind(R), ext(R), inst(R), nr(R);
  std::vector<double> v((size_t)R * kRateParams);
  for (int k = 0; k < R; ++k) {
    kind[k] = C.rate[k].kind;
    ext[k] = C.rate[k].ext;
    inst[k] = C.rate[k].inst;
    nr[k] = C.rate[k].nr;
    for (int j = 0; j < kRateParams; ++j) v[(size_t)k * kRateParams + j] = C.rate[k].v[j];
  }
  std::vector<uint8_t> is_diag(C.nnz, 0);
  for (int t = 0; t < C.n_state; ++t) is_diag[C.diag[t]] = 1;
  auto pairs = [](const std::vector<int>& a, const std::vector<int>& b) {
    std::vector<int> p(2 * a.size());
    for (size_t i = 0; i < a.size(); ++i) {
      p[2 * i] = a[i];
      p[2 * i + 1] = b[i];
    }
    return p;
  };
  std::vector<int> lup = pairs(C.lu_pa, C.lu_pb), fwp = pairs(C.fwd_pa, C.fwd_pb),
                   bwp = pairs(C.bwd_pa, C.bwd_pb);
  static_assert(sizeof(Task) == sizeof(DTask), "task layout");

  size_t o_kind = add(kind.data(), 4 * R), o_ext = add(ext.data(), 4 * R), o_inst = add(inst.data(), 4 * R),
         o_nr = add(nr.data(), 4 * R), o_v = add(v.data(), 8 * v.size()),
         o_react = add(C.rx_react.data(), 4 * C.rx_react.size()),
         o_pofs = add(C.rx_pofs.data(), 4 * C.rx_pofs.size()),
         o_pptr = add(C.param_ptr.data(), 4 * C.param_ptr.size()),
         o_par = add(C.param.data(), 4 * C.param.size()),
         o_parw = add(C.param_w.data(), 8 * C.param_w.size()),
         o_tptr = add(C.term_ptr.data(), 4 * C.term_ptr.size()),
         o_trxn = add(C.term_rxn.data(), 4 * C.term_rxn.size()),
         o_tcoef = add(C.term_coef.data(), 8 * C.term_coef.size()),
         o_jptr = add(C.jc_ptr.data(), 4 * C.jc_ptr.size()),
         o_jpart = add(C.jc_part.data(), 4 * C.jc_part.size()),
         o_jcoef = add(C.jc_coef.data(), 8 * C.jc_coef.size()),
         o_isd = add(is_diag.data(), is_diag.size()), o_diag = add(C.diag.data(), 4 * C.diag.size()),
         o_perm = add(C.perm.data(), 4 * C.perm.size()),
         o_lut = add(C.lu_tasks.data(), sizeof(Task) * C.lu_tasks.size()),
         o_fwt = add(C.fwd_tasks.data(), sizeof(Task) * C.fwd_tasks.size()),
         o_bwt = add(C.bwd_tasks.data(), sizeof(Task) * C.bwd_tasks.size()),
         o_lup = add(lup.data(), 4 * lup.size()), o_fwp = add(fwp.data(), 4 * fwp.size()),
         o_bwp = add(bwp.data(), 4 * bwp.size()),
         o_stage[4] = {add(mh->stage[0].bytes.data(), mh->stage[0].bytes.size()),
                       add(mh->stage[1].bytes.data(), mh->stage[1].bytes.size()),
                       add(mh->stage[2].bytes.data(), mh->stage[2].bytes.size()),
                       add(mh->stage[3].bytes.data(), mh->stage[3].bytes.size())};

  std::vector<char> host(total, 0);
  for (auto& it : items)
    if (it.bytes) std::memcpy(host.data() + it.off, it.src, it.bytes);
  void* blob = nullptr;
  hipError_t e = hipMalloc(&blob, total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(mechanism tables)");
  e = hipMemcpy(blob, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(blob);
    return hip_fail(e, "hipMemcpy(mechanism tables)");
  }
  char* b = static_cast<char*>(blob);
  DevMech& d = out.dm;
  d.N = C.n_state;
  d.R = R;
  d.Z = C.nnz;
  d.n_inst = C.n_inst;
  d.n_ext = C.n_ext;
  d.n_part = C.n_partials;
  d.n_gas = C.n_gas;
  d.lu_levels = C.lu_levels();
  d.fwd_levels = C.fwd_levels();
  d.bwd_levels = C.bwd_levels();
  d.rs_kind = (const int*)(b + o_kind);
  d.rs_ext = (const int*)(b + o_ext);
  d.rs_inst = (const int*)(b + o_inst);
  d.rs_nr = (const int*)(b + o_nr);
  d.rs_v = (const double*)(b + o_v);
  d.rx_react = (const int*)(b + o_react);
  d.rx_pofs = (const int*)(b + o_pofs);
  d.param_ptr = (const int*)(b + o_pptr);
  d.param = (const int*)(b + o_par);
  d.param_w = (const double*)(b + o_parw);
  d.n_param = (int)C.param_ptr.size() - 1;
  d.term_ptr = (const int*)(b + o_tptr);
  d.term_rxn = (const int*)(b + o_trxn);
  d.term_coef = (const double*)(b + o_tcoef);
  d.jc_ptr = (const int*)(b + o_jptr);
  d.jc_part = (const int*)(b + o_jpart);
  d.jc_coef = (const double*)(b + o_jcoef);
  d.is_diag = (const uint8_t*)(b + o_isd);
  d.diag = (const int*)(b + o_diag);
  d.perm = (const int*)(b + o_perm);
  d.lu_task = (const DTask*)(b + o_lut);
  d.n_lu_task = (int)C.lu_tasks.size();
  d.fwd_task = (const DTask*)(b + o_fwt);
  d.n_fwd_task = (int)C.fwd_tasks.size();
  d.bwd_task = (const DTask*)(b + o_bwt);
  d.n_bwd_task = (int)C.bwd_tasks.size();
  d.lu_pair = (const int2*)(b + o_lup);
  d.fwd_pair = (const int2*)(b + o_fwp);
  d.bwd_pair = (const int2*)(b + o_bwp);
  for (int v = 0; v < 4; ++v) {
    const StageBlock& sb = mh->stage[v];
    StageView& w = d.sv[v];
    w = StageView{};
    if (!sb.ok) continue;
    w.base = (const uint8_t*)(b + o_stage[v]);
    w.bytes = (int)sb.bytes.size();
    w.core_bytes = sb.core_bytes;
    w.so_rx = sb.off_rx;
    w.so_diag = sb.off_diag;
    w.so_sf = sb.off_sf;
    w.so_sf_lp = sb.off_sf_lp;
    w.so_sb = sb.off_sb;
    w.so_sb_lp = sb.off_sb_lp;
    w.so_lt = sb.off_lt;
    w.so_lt_lp = sb.off_lt_lp;
    w.so_lf = sb.off_lf;
    w.so_lf_lp = sb.off_lf_lp;
    w.so_us = sb.off_us;
    w.n_sf_lev = sb.n_sf_lev;
    w.n_sb_lev = sb.n_sb_lev;
    w.n_us = sb.n_us;
    w.so_ft = sb.off_ft;
    w.so_ft_coef = sb.off_ft_coef;
    w.so_jt = sb.off_jt;
    w.so_jt_coef = sb.off_jt_coef;
    w.n_ft = sb.n_ft;
    w.n_jt = sb.n_jt;
    w.so_ft_lp = sb.off_ft_lp;
    w.so_jt_lp = sb.off_jt_lp;
    w.wave_lists = sb.wave_lists;
    w.n_lu_lev = sb.n_lu_lev;
    w.tail_k = sb.tail_k;
    w.tail_s = sb.tail_s;
    w.so_tail = sb.off_tail;
    w.so_tail_lp = sb.off_tail_lp;
    w.n_tail = sb.n_tail;
    w.so_tail_rs = sb.off_tail_rs;
  }
  d.stage = d.sv[0].base;
  out.device = device;
  out.blob = blob;
  out.bytes = total;
  return CAMP_OK;
}

}  // namespace

// Device-resident tables of `mh` for the current device, if already uploaded (else null).
const DevMech* resident_if_uploaded(camp_mech* mh) {
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> g(mh->mu);
  auto it = mh->dev.find(device);
  return it == mh->dev.end() ? nullptr : &it->second.dm;
}

// Device-resident tables of `mh` for the current device (uploaded on first use).
int resident(camp_mech* mh, const DevMech** dm) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> g(mh->mu);
  auto it = mh->dev.find(device);
  if (it == mh->dev.end()) {
    DeviceTables t;
    int rc = upload(mh, device, t);
    if (rc != CAMP_OK) return rc;
    it = mh->dev.emplace(device, t).first;
  }
  *dm = &it->second.dm;
  return CAMP_OK;
}

int check_solve_args(camp_mech* mh, int n_cells, const void* state, const camp_env* env,
                     double dt, double rtol, double atol) {
  if (!mh) { set_error("mechanism is NULL"); return CAMP_EINVAL; }
  if (n_cells < 0) { set_error("n_cells < 0"); return CAMP_EINVAL; }
  if (n_cells > 0 && (!state || !env || !env->T_K || !env->P_Pa)) {
    set_error("state, env, env->T_K and env->P_Pa are required");
    return CAMP_EINVAL;
  }
  if (n_cells > 0 && mh->C.n_inst > 0 && (!env->radius_m || !env->aer_mass_kg_m3)) {
    set_error("mechanism has aerosol phases: env->radius_m and env->aer_mass_kg_m3 are required");
    return CAMP_EINVAL;
  }
  if (!(dt > 0) || !std::isfinite(dt)) { set_error("dt must be positive and finite"); return CAMP_EINVAL; }
  if (!(rtol > 0) || !std::isfinite(rtol)) { set_error("rtol must be positive and finite"); return CAMP_EINVAL; }
  if (!(atol >= 0) || !std::isfinite(atol)) { set_error("atol must be >= 0 and finite"); return CAMP_EINVAL; }
  return CAMP_OK;
}

SolveParams make_params(double dt, double rtol, double atol, const camp_opts* o) {
  SolveParams sp;
  sp.dt = dt;
  sp.rtol = rtol;
  sp.atol = atol;
  sp.atol_call = atol;
  sp.max_order = (o && o->max_order >= 1 && o->max_order <= kMaxOrder) ? o->max_order : kMaxOrder;
  sp.max_steps = (o && o->max_steps > 0) ? o->max_steps : 100000;
  sp.newton_maxit = (o && o->newton_max_iter > 0) ? std::min(o->newton_max_iter, 16) : 4;
  sp.h_min = (o && o->h_min > 0) ? o->h_min : 0.0;
  sp.h_init = (o && o->h_init > 0) ? o->h_init : 0.0;
  sp.newton_tol = (o && o->newton_tol > 0) ? o->newton_tol : kNewtonTol;
  sp.lu_drift = (o && o->lu_gamma_drift > 0) ? o->lu_gamma_drift : kLuGammaDrift;
  sp.lu_max_age = (o && o->lu_max_age > 0) ? o->lu_max_age : kLuMaxAge;
  sp.full_newton = (o && o->full_newton) ? 1 : 0;
  sp.order = nullptr;
  sp.order_bad = nullptr;
  return sp;
}

DevEnv make_env(const camp_env* e) {
  return DevEnv{e->T_K, e->P_Pa, e->cos_sza, e->radius_m, e->aer_mass_kg_m3, e->rate_override};
}

int n_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}


void set_error(const std::string& msg) { g_err = msg; }

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? CAMP_ENOMEM : CAMP_EDEVICE;
}

// Launch shape and device scratch of a fused wavefront launch with a resolved tuning: 256
// bytes for the queue counter (int 0) and the cell-order flag (int 16); in launch modes 3
// and 4 the rate-constant scratch of every resident cell slot; with a caller's cell order,
// one counter per cell for its permutation check.
int wave_launch_shape(const DevMech& dm, const Tuning& tu, int n_cells, bool has_order,
                      WaveShape* out) {
  if (!wave_lanes_ok(dm.N, 64) || !dm.stage) {
    set_error("wavefront engine supports at most 576 state variables per cell");
    return CAMP_EINVAL;
  }
  if (!wave_lanes_ok(dm.N, tu.lanes)) {
    set_error("lanes per cell must be 64, 128 (65..640 state variables) or 256 (129..768)");
    return CAMP_EINVAL;
  }
  WaveShape w;
  w.lanes = tu.lanes;
  w.waves = tu.lanes == 64 ? std::max(1, tu.waves) : 1;
  w.stage = wave_effective_mode(dm, std::max(0, std::min(4, tu.stage)));
  if (wave_wg_lds_bytes(dm, w.waves, w.stage, tu.lanes) > kLdsBytes) {
    set_error("mechanism does not fit the wavefront engine's LDS budget");
    return CAMP_EINVAL;
  }
  const int wg_total = (n_cells + w.waves - 1) / w.waves;
  w.persistent = tu.persistent || w.stage >= 3;
  w.grid = w.persistent ? std::max(1, std::min(wg_total, n_cus() * std::max(1, tu.grid_mult)))
                        : wg_total;
  w.kc_bytes = w.stage >= 3 ? sizeof(double) * (size_t)w.grid * w.waves * dm.R : 0;
  w.seen_bytes = (w.persistent && has_order) ? sizeof(int) * (size_t)n_cells : 0;
  w.bytes = w.persistent ? 256 + w.kc_bytes + w.seen_bytes : 0;
  *out = w;
  return CAMP_OK;
}

// Enqueues a fused wavefront solve on `stream` using `ws` (at least shape.bytes of device
// memory, stream-ordered: nothing else may use it until the stream has passed this solve).
// Launches only kernels: the queue counter and flags are cleared by a fill kernel.
hipError_t enqueue_wave(const DevMech& dm, const DevEnv& env, double* d_state, int n_cells,
                        const SolveParams& sp, const int* order, int* d_status,
                        camp_cell_stats* d_stats, const WaveShape& w, char* ws, bool attr_only,
                        hipStream_t stream) {
  if (!w.persistent)
    return launch_bdf_wave(dm, env, d_state, n_cells, sp, d_status, d_stats, nullptr, nullptr,
                           w.grid, w.waves, w.stage, w.lanes, attr_only, stream);
  if (attr_only)
    return launch_bdf_wave(dm, env, d_state, n_cells, sp, d_status, d_stats, nullptr, nullptr,
                           w.grid, w.waves, w.stage, w.lanes, true, stream);
  int* queue = reinterpret_cast<int*>(ws);
  double* kc = w.stage >= 3 ? reinterpret_cast<double*>(ws + 256) : nullptr;
  SolveParams spo = sp;
  hipError_t e = launch_fill_int(queue, 64, 0, stream);
  if (e == hipSuccess && order) {
    spo.order = order;
    spo.order_bad = queue + 16;
    e = launch_check_order(order, n_cells, reinterpret_cast<int*>(ws + 256 + w.kc_bytes),
                           queue + 16, stream);
  }
  if (e == hipSuccess)
    e = launch_bdf_wave(dm, env, d_state, n_cells, spo, d_status, d_stats, queue, kc, w.grid,
                        w.waves, w.stage, w.lanes, false, stream);
  return e;
}

// Scratch of fused launches on `stream`, kept per (mechanism, device, stream) and grown when
// a launch needs more: stream order makes reuse by later solves on the same stream safe.
int stream_workspace(camp_mech* mh, hipStream_t stream, size_t bytes, char** out) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> g(mh->mu);
  Workspace& w = mh->ws[std::make_pair(device, (void*)stream)];
  if (w.bytes < bytes) {
    if (w.ptr) {
      e = hipStreamSynchronize(stream);   // earlier solves on this stream may still use it
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(workspace)");
      hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    const size_t want = std::max(bytes, (size_t)1 << 20);
    e = hipMalloc((void**)&w.ptr, want);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(solve workspace)");
    w.bytes = want;
  }
  *out = w.ptr;
  return CAMP_OK;
}

namespace {
int fused_lane_slots() { return std::max(256, n_cus() * 4 * 64 * 2); }
}  // namespace

size_t solve_scratch_bytes(const DevMech& dm, const Tuning& tu, int n_cells, bool has_order) {
  if (n_cells <= 0) return 0;
  if (tu.engine == CAMP_ENGINE_PLAIN) return lane_scratch_bytes(dm, n_cells, 0);
  if (tu.engine == CAMP_ENGINE_FUSED_LANE) return lane_scratch_bytes(dm, n_cells, fused_lane_slots());
  WaveShape w;
  if (wave_launch_shape(dm, tu, n_cells, has_order, &w) != CAMP_OK) return 0;
  return w.bytes ? std::max(w.bytes, (size_t)1 << 20) : 0;
}

// Dispatch of one device solve with a resolved tuning.
int solve_device_tuned(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
                       const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
                       int* d_status, camp_cell_stats* d_stats, hipStream_t stream, const Tuning& tu) {
  DevEnv env = make_env(d_env);
  const int use_graph = opts ? opts->use_graph : 0;
  hipError_t e = hipSuccess;
  if (tu.engine == CAMP_ENGINE_PLAIN) {
    e = run_plain(dm, env, d_state, n_cells, sp, d_status, d_stats, use_graph, stream);
  } else if (tu.engine == CAMP_ENGINE_FUSED_LANE) {
    e = run_fused_lane(dm, env, d_state, n_cells, sp, d_status, d_stats, fused_lane_slots(), stream);
  } else {
    const int* order = opts ? opts->cell_order : nullptr;
    WaveShape w;
    int rc = wave_launch_shape(dm, tu, n_cells, order != nullptr, &w);
    if (rc != CAMP_OK) return rc;
    char* ws = nullptr;
    if (w.bytes) {
      rc = stream_workspace(mh, stream, w.bytes, &ws);
      if (rc != CAMP_OK) return rc;
    }
    e = enqueue_wave(dm, env, d_state, n_cells, sp, order, d_status, d_stats, w, ws, false, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "solve launch");
  return CAMP_OK;
}

// Occupancy-driven default: lanes per cell, launch mode and cells per workgroup such that
// the CU runs the most wavefronts (cells resident by LDS, times wavefronts per cell, capped
// by the registers the kernel uses), preferring fewer lanes per cell, then the most tables
// staged and rate constants in LDS.
Tuning default_tuning(const DevMech& dm, int n_cells) {
  Tuning t;
  const bool fits_wave = wave_lanes_ok(dm.N, 64) && dm.stage &&
                         wave_wg_lds_bytes(dm, 1, 0, 64) <= kLdsBytes;
  t.engine = fits_wave ? CAMP_ENGINE_FUSED_WAVE : CAMP_ENGINE_FUSED_LANE;
  t.persistent = 1;
  int best = 0;
  t.stage = -1;
  for (int lanes : {64, 128, 256}) {
    if (!wave_lanes_ok(dm.N, lanes) || !dm.sv[lanes / 128].base) continue;
    for (int stage : {2, 1, 0, 4, 3}) {
      const int wmax = wave_max_waves(dm.N, stage, lanes);
      const int cap = wave_resident_cells_per_cu(dm.N, stage, lanes);
      for (int w = 1; w <= wmax; ++w) {
        const size_t b = wave_wg_lds_bytes(dm, w, stage, lanes);
        if (b > kLdsBytes) break;
        const int wgs = (int)(kLdsBytes / b);
        const int cells = std::min(wgs * w, cap);
        const int score = cells * (lanes / 64);
        if (score > best) {
          best = score;
          t.lanes = lanes;
          t.waves = w;
          t.stage = stage;
          t.grid_mult = std::max(1, std::min(wgs, cap / w));
        }
      }
    }
  }
  (void)n_cells;
  return t;
}

int autotuned(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
              const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
              hipStream_t stream, Tuning* out);

// The launch choice of a device solve: the autotuner's for engine AUTO (run_trials = false:
// its cached choice for this size bucket, else the occupancy default, never a trial), else
// the occupancy default for the requested engine with the caller's overrides.
int resolve_tuning(camp_mech* mh, const DevMech& dm, int n_cells, double* d_state,
                   const camp_env* d_env, const SolveParams& sp, const camp_opts* opts,
                   hipStream_t stream, bool run_trials, Tuning* out) {
  Tuning tu;
  const int engine = opts ? opts->engine : CAMP_ENGINE_AUTO;
  if (engine == CAMP_ENGINE_AUTO) {
    if (run_trials) {
      int rc = autotuned(mh, dm, n_cells, d_state, d_env, sp, opts, stream, &tu);
      if (rc != CAMP_OK) return rc;
    } else if (!cached_tuning(mh, dm, n_cells, sp, &tu)) {
      tu = default_tuning(dm, n_cells);
    }
  } else {
    tu = default_tuning(dm, n_cells);
    tu.engine = engine;
  }
  if (opts && engine != CAMP_ENGINE_AUTO) {
    if (opts->persistent >= 0) tu.persistent = opts->persistent ? 1 : 0;
    if (opts->wg_per_cu > 0) tu.grid_mult = opts->wg_per_cu;
    if (opts->waves_per_wg > 0) tu.waves = std::min(opts->waves_per_wg, 12);
    if (opts->lanes_per_cell > 0) tu.lanes = opts->lanes_per_cell;
    if (opts->stage_tables >= 0) tu.stage = std::min(opts->stage_tables, 4);
    if (opts->waves_per_wg <= 0 && tu.engine == CAMP_ENGINE_FUSED_WAVE && tu.lanes == 64 &&
        tu.stage >= 0) {
      // cells per workgroup not given: the most that this launch mode allows and LDS holds
      int w = std::min(tu.waves, wave_max_waves(dm.N, tu.stage, 64));
      while (w > 1 && wave_wg_lds_bytes(dm, w, tu.stage, 64) > kLdsBytes) --w;
      tu.waves = std::max(1, w);
    }
  }
  *out = tu;
  return CAMP_OK;
}

}  // namespace camp

using namespace camp;

extern "C" {

const char* camp_last_error(void) { return g_err.c_str(); }

int camp_mech_load(const camp_reaction* rxns, int n_rxn, const camp_species* species, int n_species,
                   const camp_phase* phases, int n_phases, camp_mech** out) {
  if (!out) { set_error("out is NULL"); return CAMP_EINVAL; }
  *out = nullptr;
  camp_mech* mh = new (std::nothrow) camp_mech();
  if (!mh) { set_error("out of host memory"); return CAMP_ENOMEM; }
  try {
    std::string err = compile_mechanism(rxns, n_rxn, species, n_species, phases, n_phases, mh->C);
    if (!err.empty()) {
      delete mh;
      set_error(err);
      return CAMP_EINVAL;
    }
    for (int v = 0; v < 3; ++v) mh->stage[v] = build_stage_block(mh->C, 1 << v, true);
    mh->stage[3] = build_stage_block(mh->C, 1, false);
  } catch (const std::bad_alloc&) {
    delete mh;
    set_error("out of host memory");
    return CAMP_ENOMEM;
  }
  *out = mh;
  return CAMP_OK;
}

int camp_mech_load_json(const char* text, camp_mech** out) {
  if (!out || !text) { set_error("NULL argument"); return CAMP_EINVAL; }
  *out = nullptr;
  MechDescription d;
  std::string err;
  try {
    err = parse_mechanism_json(text, std::strlen(text), d);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory");
    return CAMP_ENOMEM;
  }
  if (!err.empty()) { set_error(err); return CAMP_EINVAL; }
  std::vector<camp_species> sp(d.species.size());
  for (size_t i = 0; i < sp.size(); ++i)
    sp[i] = camp_species{d.species[i].name.c_str(), d.species[i].phase, d.species[i].mw,
                         d.species[i].diff, d.species[i].accom};
  std::vector<camp_phase> ph(d.phases.size());
  for (size_t i = 0; i < ph.size(); ++i)
    ph[i] = camp_phase{d.phases[i].name.c_str(), (int)d.phases[i].species.size(),
                       d.phases[i].species.data(), d.phases[i].n_instances, d.phases[i].density,
                       d.phases[i].mw_absorber, d.phases[i].radius_from_state};
  return camp_mech_load(d.reactions.data(), (int)d.reactions.size(), sp.data(), (int)sp.size(),
                        ph.data(), (int)ph.size(), out);
}

int camp_mech_pack(const camp_mech* mh, void* buf, size_t capacity, size_t* size) {
  if (!mh || !size) { set_error("NULL argument"); return CAMP_EINVAL; }
  std::vector<uint8_t> b;
  try {
    b = pack_compiled(mh->C, mh->stage);
  } catch (const std::bad_alloc&) {
    set_error("out of host memory");
    return CAMP_ENOMEM;
  }
  *size = b.size();
  if (!buf) return CAMP_OK;
  if (capacity < b.size()) { set_error("buffer too small for the packed mechanism"); return CAMP_EINVAL; }
  std::memcpy(buf, b.data(), b.size());
  return CAMP_OK;
}

int camp_mech_unpack(const void* buf, size_t size, camp_mech** out) {
  if (!out || !buf) { set_error("NULL argument"); return CAMP_EINVAL; }
  *out = nullptr;
  camp_mech* mh = new (std::nothrow) camp_mech();
  if (!mh) { set_error("out of host memory"); return CAMP_ENOMEM; }
  std::string err;
  try {
    err = unpack_compiled(static_cast<const uint8_t*>(buf), size, mh->C, mh->stage);
  } catch (const std::bad_alloc&) {
    err = "out of host memory";
  }
  if (!err.empty()) {
    delete mh;
    set_error(err);
    return err == "out of host memory" ? CAMP_ENOMEM : CAMP_EINVAL;
  }
  *out = mh;
  return CAMP_OK;
}

int camp_mech_info(const camp_mech* mh, camp_mech_info_t* info) {
  if (!mh || !info) { set_error("NULL argument"); return CAMP_EINVAL; }
  const Compiled& C = mh->C;
  info->n_state = C.n_state;
  info->n_gas = C.n_gas;
  info->n_instances = C.n_inst;
  info->n_rxn_expanded = C.n_rxn;
  info->n_external = C.n_ext;
  info->nnz_pattern = C.nnz0;
  info->nnz_fill = C.nnz;
  info->lu_pairs = C.lu_pairs;
  info->lu_levels = C.lu_levels();
  info->fwd_levels = C.fwd_levels();
  info->bwd_levels = C.bwd_levels();
  info->n_partials = C.n_partials;
  info->n_terms = (int)C.term_rxn.size();
  info->n_jac_contrib = (int)C.jc_part.size();
  info->tail_k = C.tail_k;
  info->nnz_lu = C.nnz_lu;
  return CAMP_OK;
}

int camp_mech_export(const camp_mech* mh, int* perm, int* row_ptr, int* col, int* pattern0) {
  if (!mh) { set_error("NULL mechanism"); return CAMP_EINVAL; }
  const Compiled& C = mh->C;
  if (perm) std::copy(C.perm.begin(), C.perm.end(), perm);
  if (row_ptr) std::copy(C.row_ptr.begin(), C.row_ptr.end(), row_ptr);
  if (col) std::copy(C.col.begin(), C.col.end(), col);
  if (pattern0)
    for (int s = 0; s < C.nnz; ++s) pattern0[s] = C.pattern0[s];
  return CAMP_OK;
}

int camp_mech_layout_info(const camp_mech* mh, int lanes_per_cell, int* tail_k, int* fwd_levels,
                          int* bwd_levels, int* lu_levels, int* staged_bytes) {
  if (!mh) { set_error("NULL mechanism"); return CAMP_EINVAL; }
  const int v = lanes_per_cell == 64 ? 0 : lanes_per_cell == 128 ? 1 : lanes_per_cell == 256 ? 2 : -1;
  if (v < 0) { set_error("lanes_per_cell must be 64, 128 or 256"); return CAMP_EINVAL; }
  const StageBlock& sb = mh->stage[v];
  if (!sb.ok) { set_error("mechanism exceeds the wavefront engine's table ranges"); return CAMP_EINVAL; }
  if (tail_k) *tail_k = sb.tail_k;
  if (fwd_levels) *fwd_levels = sb.n_sf_lev;
  if (bwd_levels) *bwd_levels = sb.n_sb_lev;
  if (lu_levels) *lu_levels = sb.n_lu_lev;
  if (staged_bytes) *staged_bytes = (int)sb.bytes.size();
  return CAMP_OK;
}

int camp_tuned_launch(camp_mech* mh, int n_cells, int* engine, int* lanes_per_cell, int* launch_mode,
                      int* cells_per_wg, int* wg_per_cu) {
  if (!mh || n_cells < 1) { set_error("bad argument"); return CAMP_EINVAL; }
  const DevMech* dm = resident_if_uploaded(mh);
  Tuning tu;
  if (!dm || !cached_tuning(mh, *dm, n_cells, make_params(1.0, 1e-4, 0.0, nullptr), &tu)) {
    set_error("no autotuned launch for this mechanism, device and size bucket yet");
    return CAMP_EINVAL;
  }
  if (engine) *engine = tu.engine;
  if (lanes_per_cell) *lanes_per_cell = tu.lanes;
  if (launch_mode) *launch_mode = tu.stage;
  if (cells_per_wg) *cells_per_wg = tu.lanes == 64 ? tu.waves : 1;
  if (wg_per_cu) *wg_per_cu = tu.persistent ? tu.grid_mult : 0;
  return CAMP_OK;
}

int camp_emulate_factor_solve(const camp_mech* mh, int lanes_per_cell, int dense_tail, double* m,
                              double* x) {
  if (!mh || !m || !x) { set_error("NULL argument"); return CAMP_EINVAL; }
  const int v = lanes_per_cell == 64 ? (dense_tail ? 0 : 3)
                : lanes_per_cell == 128 ? 1 : lanes_per_cell == 256 ? 2 : -1;
  if (v < 0 || (!dense_tail && v != 3)) {
    set_error("lanes_per_cell must be 64, 128 or 256 (64 only without the dense tail)");
    return CAMP_EINVAL;
  }
  const StageBlock& sb = mh->stage[v];
  if (!sb.ok) { set_error("mechanism exceeds the wavefront engine's table ranges"); return CAMP_EINVAL; }
  if (!emulate_factor_solve(mh->C, sb, m, x)) {
    set_error("zero or non-finite pivot");
    return CAMP_ESOLVE;
  }
  return CAMP_OK;
}

void camp_mech_free(camp_mech* mh) {
  if (!mh) return;
  int cur = 0;
  hipGetDevice(&cur);
  for (auto& kv : mh->dev) {
    hipSetDevice(kv.first);
    hipDeviceSynchronize();
    hipFree(kv.second.blob);
  }
  for (auto& kv : mh->ws) {
    hipSetDevice(kv.first.first);
    hipDeviceSynchronize();
    hipFree(kv.second.ptr);
  }
  hipSetDevice(cur);
  delete mh;
}

int camp_solve_device(camp_mech* mh, int n_cells, double* d_state, const camp_env* d_env, double dt,
                      double rtol, double atol, const camp_opts* opts, int* d_status,
                      camp_cell_stats* d_stats, void* stream) {
  int rc = check_solve_args(mh, n_cells, d_state, d_env, dt, rtol, atol);
  if (rc != CAMP_OK) return rc;
  if (n_cells > 0 && !d_status) { set_error("d_cell_status is required"); return CAMP_EINVAL; }
  if (n_cells == 0) return CAMP_OK;
  const DevMech* dm = nullptr;
  rc = resident(mh, &dm);
  if (rc != CAMP_OK) return rc;
  const SolveParams sp = make_params(dt, rtol, atol, opts);
  Tuning tu;
  rc = resolve_tuning(mh, *dm, n_cells, d_state, d_env, sp, opts, (hipStream_t)stream, true, &tu);
  if (rc != CAMP_OK) return rc;
  return solve_device_tuned(mh, *dm, n_cells, d_state, d_env, sp, opts, d_status, d_stats,
                            (hipStream_t)stream, tu);
}

// ---------------------------------------------------------------- plans (captured graphs)
}  // extern "C"

struct camp_plan {
  camp_mech* mh = nullptr;
  int device = 0;
  char* ws = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
void plan_release(camp_plan* p) {
  if (!p) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(p->device);
  hipDeviceSynchronize();   // replays on any stream may still use the workspace
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap) hipStreamDestroy(p->cap);
  if (p->ws) hipFree(p->ws);
  hipSetDevice(cur);
  delete p;
}
}  // namespace

extern "C" {

int camp_plan_create(camp_mech* mh, int n_cells, double* d_state, const camp_env* d_env, double dt,
                     double rtol, double atol, const camp_opts* opts, int* d_status,
                     camp_cell_stats* d_stats, void* stream, camp_plan** out) {
  if (!out) { set_error("out is NULL"); return CAMP_EINVAL; }
  *out = nullptr;
  int rc = check_solve_args(mh, n_cells, d_state, d_env, dt, rtol, atol);
  if (rc != CAMP_OK) return rc;
  if (n_cells < 1 || !d_status) { set_error("a plan needs n_cells >= 1 and d_cell_status"); return CAMP_EINVAL; }
  const DevMech* dm = nullptr;
  rc = resident(mh, &dm);
  if (rc != CAMP_OK) return rc;
  const SolveParams sp = make_params(dt, rtol, atol, opts);
  Tuning tu;
  rc = resolve_tuning(mh, *dm, n_cells, d_state, d_env, sp, opts, (hipStream_t)stream, true, &tu);
  if (rc != CAMP_OK) return rc;
  if (tu.engine != CAMP_ENGINE_FUSED_WAVE) {
    set_error("plans run the fused wavefront engine (engine AUTO or FUSED_WAVE)");
    return CAMP_EINVAL;
  }
  const int* order = opts ? opts->cell_order : nullptr;
  WaveShape w;
  rc = wave_launch_shape(*dm, tu, n_cells, order != nullptr, &w);
  if (rc != CAMP_OK) return rc;
  camp_plan* p = new (std::nothrow) camp_plan();
  if (!p) { set_error("out of host memory"); return CAMP_ENOMEM; }
  p->mh = mh;
  hipGetDevice(&p->device);
  const DevEnv env = make_env(d_env);
  hipError_t e = hipSuccess;
  if (w.bytes) e = hipMalloc((void**)&p->ws, w.bytes);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  // launch attributes are host state: set them before the capture
  if (e == hipSuccess)
    e = enqueue_wave(*dm, env, d_state, n_cells, sp, order, d_status, d_stats, w, p->ws, true, p->cap);
  if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t el = enqueue_wave(*dm, env, d_state, n_cells, sp, order, d_status, d_stats, w,
                                 p->ws, false, p->cap);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (el != hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    rc = hip_fail(e, "plan capture");
    plan_release(p);
    return rc;
  }
  *out = p;
  return CAMP_OK;
}

int camp_plan_launch(camp_plan* p, void* stream) {
  if (!p || !p->exec) { set_error("invalid plan"); return CAMP_EINVAL; }
  int device = 0;
  hipGetDevice(&device);
  if (device != p->device) { set_error("plan belongs to another device"); return CAMP_EINVAL; }
  hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
  return e == hipSuccess ? CAMP_OK : hip_fail(e, "hipGraphLaunch");
}

void camp_plan_free(camp_plan* p) { plan_release(p); }

int camp_solve(camp_mech* mh, int n_cells, double* state, const camp_env* env, double dt, double rtol,
               double atol, const camp_opts* opts, int* cell_status, camp_cell_stats* cell_stats) {
  int rc = check_solve_args(mh, n_cells, state, env, dt, rtol, atol);
  if (rc != CAMP_OK) return rc;
  if (n_cells == 0) return CAMP_OK;
  const Compiled& C = mh->C;
  const size_t n = (size_t)n_cells;
  const size_t bytes_state = 8 * n * C.n_state;
  const size_t bytes_inst = 8 * n * C.n_inst;
  const size_t bytes_ovr = 8 * n * C.n_ext;
  struct Part {
    const void* src;
    size_t bytes;
    size_t off;
  } parts[7];
  size_t total = 0;
  auto add = [&](int i, const void* src, size_t bytes) {
    parts[i] = {src, src ? bytes : 0, total};
    total = align256(total + (src ? bytes : 0));
  };
  add(0, state, bytes_state);
  add(1, env->T_K, 8 * n);
  add(2, env->P_Pa, 8 * n);
  add(3, env->cos_sza, 8 * n);
  add(4, C.n_inst ? env->radius_m : nullptr, bytes_inst);
  add(5, C.n_inst ? env->aer_mass_kg_m3 : nullptr, bytes_inst);
  add(6, env->rate_override, bytes_ovr);
  const int* order = opts ? opts->cell_order : nullptr;
  if (order) {
    std::vector<char> seen(n, 0);
    for (size_t i = 0; i < n; ++i) {
      const int c = order[i];
      if (c < 0 || (size_t)c >= n || seen[c]) {
        set_error("opts->cell_order must be a permutation of 0..n_cells-1");
        return CAMP_EINVAL;
      }
      seen[c] = 1;
    }
  }
  const size_t off_status = total;
  total = align256(total + 4 * n);
  const size_t off_stats = total;
  if (cell_stats) total = align256(total + sizeof(camp_cell_stats) * n);
  const size_t off_order = total;
  if (order) total = align256(total + 4 * n);
  char* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(solve buffers)");
  for (auto& p : parts)
    if (p.bytes) {
      e = hipMemcpy(d + p.off, p.src, p.bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) { hipFree(d); return hip_fail(e, "hipMemcpy H2D"); }
    }
  camp_env denv{(const double*)(d + parts[1].off), (const double*)(d + parts[2].off),
                parts[3].bytes ? (const double*)(d + parts[3].off) : nullptr,
                parts[4].bytes ? (const double*)(d + parts[4].off) : nullptr,
                parts[5].bytes ? (const double*)(d + parts[5].off) : nullptr,
                parts[6].bytes ? (const double*)(d + parts[6].off) : nullptr};
  int* d_status = (int*)(d + off_status);
  camp_cell_stats* d_stats = cell_stats ? (camp_cell_stats*)(d + off_stats) : nullptr;
  camp_opts dopts{};
  if (opts) dopts = *opts;
  if (order) {
    e = hipMemcpy(d + off_order, order, 4 * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(d); return hip_fail(e, "hipMemcpy H2D"); }
    dopts.cell_order = (const int*)(d + off_order);
  }
  rc = camp_solve_device(mh, n_cells, (double*)(d + parts[0].off), &denv, dt, rtol, atol,
                         opts ? &dopts : nullptr, d_status, d_stats, nullptr);
  if (rc == CAMP_OK) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e, "solve");
  }
  std::vector<int> st(n);
  if (rc == CAMP_OK) {
    e = hipMemcpy(state, d + parts[0].off, bytes_state, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(st.data(), d_status, 4 * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && cell_stats)
      e = hipMemcpy(cell_stats, d_stats, sizeof(camp_cell_stats) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy D2H");
  }
  hipFree(d);
  if (rc != CAMP_OK) return rc;
  if (cell_status) std::copy(st.begin(), st.end(), cell_status);
  for (int s : st)
    if (s != 0) {
      set_error("one or more cells failed; see cell_status");
      return CAMP_ESOLVE;
    }
  return CAMP_OK;
}

int camp_rate_constants_device(camp_mech* mh, int n_cells, const camp_env* d_env, double* d_k,
                               void* stream) {
  if (!mh || !d_env || n_cells < 0 || (n_cells > 0 && (!d_k || !d_env->T_K || !d_env->P_Pa))) {
    set_error("bad argument");
    return CAMP_EINVAL;
  }
  if (n_cells == 0) return CAMP_OK;
  const DevMech* dm = nullptr;
  int rc = resident(mh, &dm);
  if (rc != CAMP_OK) return rc;
  hipError_t e = launch_rates_step(*dm, make_env(d_env), n_cells, d_k, (hipStream_t)stream);
  return e == hipSuccess ? CAMP_OK : hip_fail(e, "rate constants");
}

static int step_common(camp_mech* mh, int n_cells, int op, const double* kin, const double* yin,
                       double* out, double gamma, void* stream) {
  if (!mh || n_cells < 0 || (n_cells > 0 && !out)) { set_error("bad argument"); return CAMP_EINVAL; }
  if (n_cells == 0) return CAMP_OK;
  const DevMech* dm = nullptr;
  int rc = resident(mh, &dm);
  if (rc != CAMP_OK) return rc;
  if (!dm->stage || (dm->N + kWave - 1) / kWave > 9 || wave_cell_bytes(*dm) > kLdsBytes) {
    set_error("single-step kernels support at most 576 state variables per cell");
    return CAMP_EINVAL;
  }
  hipError_t e = launch_wave_step(*dm, op, n_cells, kin, yin, out, gamma, (hipStream_t)stream);
  return e == hipSuccess ? CAMP_OK : hip_fail(e, "step kernel");
}

int camp_forcing_device(camp_mech* mh, int n_cells, const double* d_k, const double* d_y, double* d_f,
                        void* stream) {
  if (n_cells > 0 && (!d_k || !d_y)) { set_error("bad argument"); return CAMP_EINVAL; }
  return step_common(mh, n_cells, 0, d_k, d_y, d_f, 0.0, stream);
}

int camp_newton_matrix_device(camp_mech* mh, int n_cells, const double* d_k, const double* d_y,
                              double gamma, double* d_m, void* stream) {
  if (n_cells > 0 && (!d_k || !d_y)) { set_error("bad argument"); return CAMP_EINVAL; }
  return step_common(mh, n_cells, 1, d_k, d_y, d_m, gamma, stream);
}

int camp_lu_factor_device(camp_mech* mh, int n_cells, double* d_m, void* stream) {
  return step_common(mh, n_cells, 2, nullptr, nullptr, d_m, 0.0, stream);
}

int camp_lu_solve_device(camp_mech* mh, int n_cells, const double* d_lu, double* d_b, void* stream) {
  if (n_cells > 0 && !d_lu) { set_error("bad argument"); return CAMP_EINVAL; }
  return step_common(mh, n_cells, 3, d_lu, nullptr, d_b, 0.0, stream);
}

int camp_count_failed(int n_cells, const int* d_status, int* n_failed, void* stream) {
  if (n_cells < 0 || !n_failed || (n_cells > 0 && !d_status)) { set_error("bad argument"); return CAMP_EINVAL; }
  *n_failed = 0;
  if (n_cells == 0) return CAMP_OK;
  int* d = nullptr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMallocAsync((void**)&d, 256, s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
  e = launch_count_failed(n_cells, d_status, d, s);
  if (e == hipSuccess) e = hipMemcpyAsync(n_failed, d, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFreeAsync(d, s);
  return e == hipSuccess ? CAMP_OK : hip_fail(e, "count failed");
}

}  // extern "C"
