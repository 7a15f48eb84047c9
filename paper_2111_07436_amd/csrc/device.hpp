// Device-side view of a compiled mechanism and helpers shared by every engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace camp {

constexpr int kWave = 64;
constexpr int kMaxOrder = 5;
constexpr int kHist = kMaxOrder + 3;   // backward differences D[0..q+2]

// Level-scheduled task (see mech.hpp Task).
struct alignas(16) DTask {
  int dst, diag, pbeg, pend;
};

// One layout of the compact table block: device address, sizes and byte offsets.
struct StageView {
  const uint8_t* base;
  int bytes;        // whole block
  int core_bytes;   // core prefix (index tables of the sparse steps)
  int so_rx, so_diag, so_sf, so_sf_lp, so_sb, so_sb_lp, so_lt, so_lt_lp, so_lf, so_lf_lp, so_us;
  int n_sf_lev, n_sb_lev, n_us;
  int so_ft, so_ft_coef, so_jt, so_jt_coef, n_ft, n_jt, so_ft_lp, so_jt_lp;
  int wave_lists;   // per-wavefront term lists per level (1, 2 or 4)
  int n_lu_lev;     // factorization levels of this layout
  int tail_k, tail_s, so_tail, so_tail_lp, n_tail;   // dense tail (tail_k = 0: none)
  int so_tail_rs;
};

// Device copies of the compiled tables; passed to kernels by value.
struct DevMech {
  int N, R, Z, n_inst, n_ext, n_part, n_gas;
  int lu_levels, fwd_levels, bwd_levels;
  // rate constants
  const int* rs_kind;
  const int* rs_ext;
  const int* rs_inst;
  const int* rs_nr;
  const double* rs_v;          // [R * 12]
  // reactions
  const int* rx_react;         // [R * 3], -1 padded, elimination positions
  const int* rx_pofs;          // [R + 1]
  // reactions with Parameters: records {k, flags, d, dN, dV, dL, s_1 .. s_m} and their
  // weights at the same positions, see Compiled
  const int* param_ptr;        // [n_param + 1]
  const int* param;
  const double* param_w;
  int n_param;
  // forcing terms per species
  const int* term_ptr;
  const int* term_rxn;
  const double* term_coef;
  // Jacobian contributions per slot
  const int* jc_ptr;
  const int* jc_part;
  const double* jc_coef;
  const uint8_t* is_diag;      // [Z]
  const int* diag;             // [N]
  const int* perm;             // [N] user state index at elimination position t
  // sequential (level-ordered) tasks
  const DTask* lu_task;  int n_lu_task;
  const DTask* fwd_task; int n_fwd_task;
  const DTask* bwd_task; int n_bwd_task;
  const int2* lu_pair;         // (pa, pb)
  const int2* fwd_pair;
  const int2* bwd_pair;
  // compact tables of the wavefront engine (see StageBlock), one layout per group size:
  // sv[0] one wavefront per cell, sv[1] two, sv[2] four wavefronts (a workgroup) per cell;
  // sv[3] one wavefront without the dense tail (single-step kernels)
  StageView sv[4];
  const uint8_t* stage;   // sv[0].base, null when the mechanism exceeds the 16-bit layout
};

// Per-cell environment (device pointers, row-major [cells] / [cells][n_inst]).
struct DevEnv {
  const double* T;
  const double* P;
  const double* cos_sza;       // may be null
  const double* radius;        // may be null when n_inst == 0
  const double* mass;
  const double* override_;     // may be null
};

struct SolveParams {
  double dt, rtol, atol, h_min, h_init, newton_tol;
  double lu_drift;    // refactor when gamma drifts by more than this fraction
  int lu_max_age;     // ... or after this many accepted steps
  double atol_call;   // the caller's atol (a retry attempt may tighten atol)
  int max_order, max_steps, newton_maxit;
  int full_newton;   // 1: full Newton from the start (no Jacobian reuse)
  // Persistent wavefront launches: queue position -> cell, used unless *order_bad != 0
  // (both null: index order).
  const int* order;
  const int* order_bad;
};

// BDF coefficients: gamma_q = sum_{j=1}^{q} 1/j; local error constant 1/(q+1).
__device__ __forceinline__ double bdf_gamma(int q) {
  return q <= 1 ? 1.0 : q == 2 ? 1.5 : q == 3 ? 11.0 / 6.0 : q == 4 ? 25.0 / 12.0 : 137.0 / 60.0;
}

constexpr double kGasConstant = 8.314462618;  // J mol^-1 K^-1
constexpr double kAtmPa = 101325.0;
constexpr double kPi = 3.14159265358979323846;

constexpr double kBoltzmann = 1.380649e-23;   // J K^-1

// A exp(-Ea/T) (T/300)^B: the Arrhenius form with D = 300 K and E = 0 that the fall-off
// and custom forms are built from.
__device__ __forceinline__ double arrhenius300(const double* a, double T) {
  double k = a[0] * exp(-a[1] / T);
  if (a[2] != 0.0) k *= pow(T / 300.0, a[2]);
  return k;
}

// Rate constant of expanded reaction `r` for one cell (paper tables of Process classes).
// Phase-instance rates are zero when the instance has no mass.
__device__ inline double rate_constant(const DevMech& m, int r, double T, double P, double cosz,
                                       const double* radius, const double* mass,
                                       const double* ovr) {
  const int kind = m.rs_kind[r];
  const double* v = m.rs_v + (size_t)r * 12;
  // number density of air, molecule cm^-3
  const double air = P / (kBoltzmann * T) * 1.0e-6;
  switch (kind) {
    case 10: {  // Troe fall-off
      const double k0m = arrhenius300(v, T) * air, kinf = arrhenius300(v + 3, T);
      const double lg = log10(k0m / kinf);
      const double k = k0m / (1.0 + k0m / kinf) * pow(v[6], 1.0 / (1.0 + lg * lg / v[7]));
      return k * v[9];
    }
    case 11:    // HO2 self-reaction: k1 + k2 [M]
      return (arrhenius300(v, T) + arrhenius300(v + 3, T) * air) * v[9];
    case 12: {  // OH + HNO3: k0 + k3[M] / (1 + k3[M] / k2)
      const double k3m = arrhenius300(v + 6, T) * air;
      return (arrhenius300(v, T) + k3m / (1.0 + k3m / arrhenius300(v + 3, T))) * v[9];
    }
    case 13:    // tunneling: A exp(-B/T) exp(C/T^3)
      return v[0] * exp(-v[1] / T) * exp(v[2] / (T * T * T)) * v[9];
    default:
      break;
  }
  switch (kind) {
    case 1: {  // Arrhenius, already scaled to mol m^-3 units
      double k = v[0] * exp(-v[1] / T);
      if (v[2] != 0.0) k *= pow(T / v[3], v[2]);
      if (v[4] != 0.0) k *= 1.0 + v[4] * P;
      return k;
    }
    case 2: {  // photolysis
      int e = m.rs_ext[r];
      if (ovr) return ovr[e];
      return v[1] != 0.0 ? v[0] * fmax(0.0, cosz) : v[0];
    }
    case 3:
    case 4: {  // emission, first-order loss
      int e = m.rs_ext[r];
      return ovr ? ovr[e] : v[0];
    }
    default:
      break;
  }
  const int g = m.rs_inst[r];
  const double ms = mass[g];
  if (ms == 0.0) return 0.0;
  if (kind == 17) return ms / v[4];  // absorbing moles of the instance
  if (kind == 19) return ms / v[3];  // particle core volume per volume of air
  if (kind == 14 || kind == 15) {  // aqueous reversible: forward K k_r, reverse k_r, on molarities
    const int nr = m.rs_nr[r];
    const double vol = ms / v[3];
    double k = v[2];
    if (kind == 14) k *= v[0] * exp(v[1] * (1.0 / T - 1.0 / 298.0));
    if (nr != 1) k *= pow(1000.0 * vol, (double)(1 - nr));
    return k;
  }
  if (kind == 5) {  // condensed-phase Arrhenius
    double k = v[0] * exp(-v[1] / T);
    if (v[2] != 0.0) k *= pow(T / v[3], v[2]);
    if (v[4] != 0.0) k *= 1.0 + v[4] * P;
    if (v[5] != 0.0) {
      const int nr = m.rs_nr[r];
      const double vol = ms / v[6];          // phase volume per air volume
      if (nr != 1) k *= pow(1000.0 * vol, (double)(1 - nr));
    }
    return k;
  }
  // phase transfer: v = {D_g, MW_g, alpha, density, mw_abs, p0..p3}
  const double rad = radius[g];
  const double Dg = v[0], mw = v[1], alpha = v[2], rho = v[3];
  const double c_bar = sqrt(8.0 * kGasConstant * T / (kPi * mw));
  if (kind == 20) return 3.0 * Dg / c_bar;   // mean free path
  const double Kn = 3.0 * Dg / c_bar / rad;
  const double ffs = 0.75 * alpha * (1.0 + Kn) / (Kn * Kn + Kn + 0.283 * Kn * alpha + 0.75 * alpha);
  const double n_part = ms / (rho * (4.0 / 3.0) * kPi * rad * rad * rad);
  if (kind == 18) return n_part;             // particle number concentration
  const double kc = 4.0 * kPi * rad * Dg * ffs * n_part;
  if (kind == 6 || kind == 8) return kc;
  if (kind == 7) {  // Henry evaporation
    const double H = v[5] * exp(v[6] * (1.0 / T - 1.0 / 298.0));
    return kc / (H * 1000.0 * (ms / rho) * kGasConstant * T);
  }
  // SIMPOL evaporation; with the full Raoult mole fraction (kind 16) the rate's parameter
  // divides by the instance's total condensed moles instead of n_abs
  const double p0 = exp10(v[5] / T + v[6] + v[7] * T + v[8] * log(T));
  if (kind == 16) return kc * p0 * kAtmPa / (kGasConstant * T);
  const double n_abs = ms / v[4];
  return kc * p0 * kAtmPa / (kGasConstant * T * n_abs);
}

// Fuchs-Sutugin factor F(Kn) and its derivative.
__device__ __forceinline__ void fuchs_sutugin(double Kn, double alpha, double& f, double& df) {
  const double num = 0.75 * alpha * (1.0 + Kn);
  const double den = Kn * Kn + Kn + 0.283 * Kn * alpha + 0.75 * alpha;
  const double dden = 2.0 * Kn + 1.0 + 0.283 * alpha;
  f = num / den;
  df = (0.75 * alpha * den - num * dden) / (den * den);
}

// The Parameters of record q (reaction k = its first entry): the rate factor phi (1/p and
// psi multiplied), and the chain-rule factors inv_p = 1/p and g = dln(psi)/dr /
// (4 pi N_p r^2) (see Compiled::param). Sums run in record order.
struct ParamEval {
  int k, flags;
  double phi, inv_p, g;
};
template <class Kc, class Y>
__device__ __forceinline__ ParamEval parameter_eval(const DevMech& m, int q, Kc kc, Y y) {
  const int b = m.param_ptr[q], e = m.param_ptr[q + 1];
  ParamEval r;
  r.k = m.param[b];
  r.flags = m.param[b + 1];
  r.phi = 1.0;
  r.inv_p = 0.0;
  r.g = 0.0;
  if (r.flags & 1) {
    double s = 0.0;
    for (int i = b + 6; i < e; ++i) s += y(m.param[i]);
    const double p = kc(m.param[b + 2]) + s;
    r.inv_p = p != 0.0 ? 1.0 / p : 0.0;
    r.phi = r.inv_p;
  }
  if (r.flags & 2) {
    const double np = kc(m.param[b + 3]);
    if (np == 0.0) {
      r.phi = 0.0;
    } else {
      double s = 0.0;
      for (int i = b + 6; i < e; ++i) s += m.param_w[i] * y(m.param[i]);
      const double v0 = kc(m.param[b + 4]), lam = kc(m.param[b + 5]), alpha = m.param_w[b + 1];
      const double scale = 3.0 / (4.0 * kPi * np);
      const double rad = cbrt(scale * (v0 + s)), rad0 = cbrt(scale * v0);
      double f, df, f0, df0;
      fuchs_sutugin(lam / rad, alpha, f, df);
      fuchs_sutugin(lam / rad0, alpha, f0, df0);
      r.phi *= rad * f / (rad0 * f0);
      r.g = (f - (lam / rad) * df) / (rad * f) / (4.0 * kPi * np * rad * rad);
    }
  }
  return r;
}

// Moves a double between lanes with one DPP pattern (both 32-bit halves).
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, kCtrl, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The value of `v` held by lane `l` (a compile-time constant), as a wavefront-uniform value.
template <int l>
__device__ __forceinline__ double lane_value(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The value of `v` held by lane `l` (wavefront-uniform; l need not be a constant).
__device__ __forceinline__ double lane_double(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// DPP patterns inside each row of 16 lanes.
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141; // lane i <-> 7 - i within 8 lanes
constexpr int kDppRowMirror = 0x140;     // lane i <-> 15 - i within 16 lanes

// Sum over the 64 lanes of a wavefront, the same value in every lane. All 64 lanes must
// be active. Row sums by DPP moves, then the four row sums in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<kDppQuadXor1>(v);
  v += dpp_move<kDppQuadXor2>(v);
  v += dpp_move<kDppRowHalfMirror>(v);
  v += dpp_move<kDppRowMirror>(v);
  return (lane_value<0>(v) + lane_value<16>(v)) + (lane_value<32>(v) + lane_value<48>(v));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<kDppQuadXor1>(v));
  v = fmax(v, dpp_move<kDppQuadXor2>(v));
  v = fmax(v, dpp_move<kDppRowHalfMirror>(v));
  v = fmax(v, dpp_move<kDppRowMirror>(v));
  return fmax(fmax(lane_value<0>(v), lane_value<16>(v)), fmax(lane_value<32>(v), lane_value<48>(v)));
}

// Nonzero in any active lane.
__device__ __forceinline__ int wave_or(int v) { return __ballot(v != 0) != 0ull; }

// Cell-interleaved slab addressing: element x (of X per cell) of cell c lives at
// ((c / 64) * X + x) * 64 + c % 64, so the 64 lanes of a wavefront touching the same x of
// 64 consecutive cells read one contiguous 512-byte line.
__device__ __forceinline__ size_t slab(int c, int X) {
  return ((size_t)(c >> 6) * X) * kWave + (c & 63);
}

}  // namespace camp
