// Fused persistent engine, host side: launch shapes, LDS sizes and the dispatch of a launch
// to the kernel instantiation for its species per lane, group size and launch mode; and the
// single-step kernels behind the step entry points.
#include "engine_wave.hpp"
#include "runtime.hpp"

namespace camp {

int wave_lanes_ok(int n_state, int lanes) {
  if (lanes == 64) return (n_state + 63) / 64 <= 9;
  if (lanes == 128) return n_state > 64 && (n_state + 127) / 128 <= 5;
  if (lanes == 256) return n_state > 128 && (n_state + 255) / 256 <= 3;
  return 0;
}

int wave_max_waves(int n_state, int mode, int lanes) {
  if (lanes != 64) return 1;
  const int npl = (n_state + kWave - 1) / kWave;
  return (npl <= 2 && kc_global(mode)) ? 12 : npl <= 3 ? 8 : 4;
}

int wave_resident_cells_per_cu(int n_state, int mode, int lanes) {
  if (lanes == 64) return wave_max_waves(n_state, mode, 64);
  const int npl = (n_state + lanes - 1) / lanes;   // see min_waves_per_simd
  const int per_simd = (lanes == 128 && npl <= 2 && kc_global(mode)) ? 3 : npl <= 3 ? 2 : 1;
  return 4 * per_simd / (lanes / 64);
}

int wave_effective_mode(const DevMech& m, int mode) { return m.n_param ? kParamMode : mode; }

size_t wave_cell_bytes(const DevMech& m) { return sizeof(double) * cell_doubles(m, 0); }

size_t wave_lds_bytes(const DevMech& m) { return wave_cell_bytes(m); }

// LDS bytes of a workgroup of `waves` cells in launch mode `mode` (0..4), with `lanes` per
// cell (which picks the table layout).
size_t wave_wg_lds_bytes(const DevMech& m, int waves, int mode, int lanes) {
  mode = wave_effective_mode(m, mode);
  return (size_t)staged_bytes(m.sv[lanes / 128], mode) +
         (size_t)waves * sizeof(double) * cell_doubles(m, mode);
}

hipError_t launch_bdf_wave(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                           const SolveParams& sp, int* status, camp_cell_stats* stats, int* queue,
                           double* kc_glob, int grid, int waves, int stage, int lanes,
                           bool attr_only, hipStream_t stream) {
  if (!wave_lanes_ok(m.N, lanes)) return hipErrorInvalidValue;
  if (stage < 0 || (stage > 4 && stage != kParamMode)) return hipErrorInvalidValue;
  stage = wave_effective_mode(m, stage);
  if (stage == kParamMode && !m.n_param) return hipErrorInvalidValue;
  const StageView& view = m.sv[lanes / 128];
  if (!view.base || view.wave_lists != lanes / kWave) return hipErrorInvalidValue;
  if (waves < 1 || waves > wave_max_waves(m.N, stage, lanes)) return hipErrorInvalidValue;
  if (!attr_only && kc_global(stage) && (!queue || !kc_glob)) return hipErrorInvalidValue;
  const WaveParams p{m,     env,   state, n_cells, sp,
                     status, stats, queue, kc_glob, grid,
                     waves, wave_wg_lds_bytes(m, waves, stage, lanes), attr_only, stream};
  const int npl = (m.N + lanes - 1) / lanes;
  if (lanes == 128) return wave_run_128(p, npl, stage);
  if (lanes == 256) return wave_run_256(p, npl, stage);
  if (npl <= 3) return wave_run_64_a(p, npl, stage);
  if (npl <= 6) return wave_run_64_b(p, npl, stage);
  return wave_run_64_c(p, npl, stage);
}

namespace {

// ---------------------------------------------------------------- single-step kernels
// One wavefront per cell; the same device code as the fused engine (tables read from
// global memory), on row-major [cells][...] arrays in user state order.

template <int NPL, bool kPar>
__global__ __launch_bounds__(kWave) void wave_step_kernel(DevMech m, int op, int n_cells,
                                                          const double* kin, const double* yin,
                                                          double* out, double gamma) {
  extern __shared__ double lds[];
  const int np = m.n_part > m.R ? m.n_part : m.R;
  const char* g = reinterpret_cast<const char*>(m.sv[3].base);
  double* yl = lds + m.Z;
  double* xl = yl + m.N;
  double* P = xl + m.N;
  const WaveCell<NPL, kWave, kPar> W{m, Tabs{g, g, m.sv[3]}, lds, yl, xl, P, P + np + 8, P + np,
                                     (int)threadIdx.x};
  const int cell = blockIdx.x;
  if (cell >= n_cells) return;
  const int lane = threadIdx.x;
  if (op == 0 || op == 1) {  // forcing / Newton matrix from k and y
    for (int k = lane; k < m.R; k += kWave) W.kc[k] = kin[(size_t)cell * m.R + k];
    for (int t = lane; t < m.N; t += kWave) W.yl[t] = yin[(size_t)cell * m.N + m.perm[t]];
    wave_sync();
    if (op == 0) {
      double f[NPL];
      W.forcing(f);
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        const int t = lane + kWave * i;
        if (t < m.N) out[(size_t)cell * m.N + m.perm[t]] = f[i];
      }
    } else {
      W.newton_matrix(gamma);
      for (int s = lane; s < m.Z; s += kWave) out[(size_t)cell * m.Z + s] = W.M[s];
    }
  } else if (op == 2) {      // LU in place on out
    for (int s = lane; s < m.Z; s += kWave) W.M[s] = out[(size_t)cell * m.Z + s];
    wave_sync();
    W.lu();
    W.factors_to_conventional();
    for (int s = lane; s < m.Z; s += kWave) out[(size_t)cell * m.Z + s] = W.M[s];
  } else {                   // solve: kin = LU, out = b -> x
    for (int s = lane; s < m.Z; s += kWave) W.M[s] = kin[(size_t)cell * m.Z + s];
    for (int t = lane; t < m.N; t += kWave) W.xl[t] = out[(size_t)cell * m.N + m.perm[t]];
    wave_sync();
    W.factors_from_conventional();
    W.solve();
    for (int t = lane; t < m.N; t += kWave) out[(size_t)cell * m.N + m.perm[t]] = W.xl[t];
  }
}

// seen[0..n) starts at zero; *bad becomes nonzero unless order is a permutation of 0..n-1
// (n entries, each in range and none repeated).
__global__ void check_order_kernel(const int* order, int n, int* seen, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = order[i];
  if (c < 0 || c >= n || atomicAdd(seen + c, 1) != 0) atomicOr(bad, 1);
}

__global__ void rates_step_kernel(DevMech m, DevEnv env, int n_cells, double* k_out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n_cells * m.R) return;
  const int cell = (int)(idx / m.R), r = (int)(idx % m.R);
  const double* rad = env.radius ? env.radius + (size_t)cell * m.n_inst : nullptr;
  const double* mas = env.mass ? env.mass + (size_t)cell * m.n_inst : nullptr;
  const double* ovr = env.override_ ? env.override_ + (size_t)cell * m.n_ext : nullptr;
  k_out[idx] = rate_constant(m, r, env.T[cell], env.P[cell], env.cos_sza ? env.cos_sza[cell] : 1.0,
                             rad, mas, ovr);
}

}  // namespace

hipError_t launch_check_order(const int* order, int n, int* seen, int* bad, hipStream_t stream) {
  hipError_t e = launch_fill_int(seen, n, 0, stream);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(check_order_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, order, n,
                     seen, bad);
  return hipGetLastError();
}

hipError_t launch_rates_step(const DevMech& m, const DevEnv& env, int n_cells, double* k_out,
                             hipStream_t stream) {
  const long long n = (long long)n_cells * m.R;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(rates_step_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, m,
                     env, n_cells, k_out);
  return hipGetLastError();
}

hipError_t launch_wave_step(const DevMech& m, int op, int n_cells, const double* kin,
                            const double* yin, double* out, double gamma, hipStream_t stream) {
  const size_t lds = wave_cell_bytes(m);
  const int npl = (m.N + kWave - 1) / kWave;
  if (n_cells == 0) return hipSuccess;
#define CAMP_STEP_CASE(K)                                                                      \
  case K: {                                                                                    \
    const void* fn = m.n_param ? (const void*)wave_step_kernel<K, true>                       \
                                : (const void*)wave_step_kernel<K, false>;                     \
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e != hipSuccess) return e;                                                             \
    if (m.n_param)                                                                            \
      hipLaunchKernelGGL((wave_step_kernel<K, true>), dim3(n_cells), dim3(kWave), lds, stream, \
                         m, op, n_cells, kin, yin, out, gamma);                                \
    else                                                                                       \
      hipLaunchKernelGGL((wave_step_kernel<K, false>), dim3(n_cells), dim3(kWave), lds, stream, \
                         m, op, n_cells, kin, yin, out, gamma);                                \
    return hipGetLastError();                                                                  \
  }
  switch (npl) {
    CAMP_STEP_CASE(1)
    CAMP_STEP_CASE(2)
    CAMP_STEP_CASE(3)
    CAMP_STEP_CASE(4)
    CAMP_STEP_CASE(5)
    CAMP_STEP_CASE(6)
    CAMP_STEP_CASE(7)
    CAMP_STEP_CASE(8)
    CAMP_STEP_CASE(9)
    default:
      return hipErrorInvalidValue;
  }
#undef CAMP_STEP_CASE
}

}  // namespace camp
