// Host-side compiled mechanism: expansion, elimination order, symbolic fill and the
// level-scheduled tables that every device engine reads. Pure C++ (no HIP types), so the
// compiler can be built and checked on a machine without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "camp.h"

namespace camp {

// Kind of rate constant carried by one expanded (generalized mass-action) reaction.
enum RateKind : int {
  KR_ARRHENIUS = 1,
  KR_PHOTOLYSIS = 2,
  KR_EMISSION = 3,
  KR_LOSS = 4,
  KR_CONDENSED = 5,
  KR_HENRY_COND = 6,
  KR_HENRY_EVAP = 7,
  KR_SIMPOL_COND = 8,
  KR_SIMPOL_EVAP = 9,
  KR_TROE = 10,
  KR_H2O2 = 11,
  KR_OHHNO3 = 12,
  KR_TUNNEL = 13,
  KR_AQREV_FWD = 14,
  KR_AQREV_REV = 15,
  KR_SIMPOL_EVAP_RAOULT = 16,
  KR_ABSORBER = 17,
  KR_NUMBER = 18,
  KR_CORE_VOLUME = 19,
  KR_MEAN_PATH = 20
};

// Parameter flags of a reaction (Sect. 2.2.2), and the fixed head of its record.
constexpr int kParamRaoult = 1;   // rate divided by p = kc[d] + sum of y over the set
constexpr int kParamRadius = 2;   // transfer rate at the radius grown by the set's volume
constexpr int kParamHead = 6;     // {k, flags, d, dN, dV, dL}
inline int n_param_partials(int flags) {
  return ((flags & kParamRaoult) ? 1 : 0) + ((flags & kParamRadius) ? 1 : 0);
}

constexpr int kRateParams = 12;

// Parameter block of one expanded reaction, laid out for the rate-constant kernel.
//   ARRHENIUS : v = {A * (N_A 1e-6)^(n_r-1), Ea/kb, B, D, E}
//   PHOTOLYSIS: v = {J0, sza_flag}
//   EMISSION  : v = {E};  LOSS: v = {k}
//   CONDENSED : v = {A, Ea/kb, B, D, E, aqueous, density}
//   *_COND/*_EVAP: v = {D_g, MW_g, alpha, density, mw_absorber, p0..p3}
//                  Henry p = {H298, C}, SIMPOL p = {B1, B2, B3, B4}
//   TROE, H2O2, OHHNO3, TUNNEL: v[0..8] = the process parameters p[0..8], v[9] = the unit
//                  factor (N_A 1e-6)^(n_r-1) from molecule cm^-3 to mol m^-3
//   AQREV_FWD/REV: v = {A, C, k_r, density}
//   SIMPOL_EVAP_RAOULT: as *_EVAP; its rate constant omits the absorber amount, which the
//                  rate's parameter supplies (the instance's total condensed moles)
//   ABSORBER  : v[3] = density, v[4] = mw_absorber; no reactants or products, rate
//                  constant m / mw_absorber (the absorbing moles of one phase instance)
//   NUMBER, CORE_VOLUME, MEAN_PATH: carriers of a phase whose radius follows the state:
//                  particle number concentration m / (rho 4/3 pi r^3), core volume m / rho,
//                  the gas species' mean free path 3 D_g / c_bar (v[0] = D_g, v[1] = MW_g)
struct RateSpec {
  int kind;
  int ext;    // column of rate_override, or -1
  int inst;   // global phase-instance index, or -1
  int nr;     // reactant occurrences
  double v[kRateParams];
};

// One unit of level-scheduled work shared by the LU factorization and the triangular
// solves: value[dst] = (value[dst] - sum_{q in [pbeg, pend)} A[pa[q]] * B[pb[q]]) / A[diag]
// (no division when diag < 0).
struct Task {
  int dst, diag, pbeg, pend;
};

struct Compiled {
  // sizes
  int n_state = 0, n_gas = 0, n_inst = 0, n_rxn = 0, n_ext = 0;
  int nnz0 = 0, nnz = 0;
  long long lu_pairs = 0;
  // Size of the dense trailing block of the filled pattern (0: none). The last tail_k
  // elimination positions form a fully stored block, so the wavefront engine can replace
  // their factorization and triangular solves by the explicit inverse of their Schur
  // complement (see StageBlock).
  int tail_k = 0;
  int nnz_lu = 0;   // entries of the symbolic LU fill (before the dense tail is added)

  // phase instance -> phase, first state index (user order)
  std::vector<int> inst_phase, inst_base;
  // elimination order: perm[t] = user state index at position t; iperm is its inverse
  std::vector<int> perm, iperm;

  // expanded reactions (device state indices, i.e. elimination positions)
  std::vector<RateSpec> rate;           // [R]
  std::vector<int> rx_react;            // [R * 3], pad -1
  std::vector<int> rx_nr;               // [R]
  std::vector<int> rx_pofs;             // [R + 1] partial offsets
  int n_partials = 0;
  // Reactions with Parameters (Sect. 2.2.2), one record per reaction: `param` in
  // [param_ptr[q], param_ptr[q+1]) holds {k, flags, d, dN, dV, dL, s_1 .. s_m} (state
  // indices as elimination positions) and `param_w` at the same positions holds the
  // accommodation coefficient (at the flags slot) and the weights w_j = MW_j / rho (at the
  // s_j slots). Reaction k's rate is multiplied by
  //   1 / p, p = kc[d] + sum_j y[s_j]           (kParamRaoult; 0 when p = 0), and
  //   psi = r F(kc[dL] / r) / (r0 F(kc[dL] / r0)), r = (3 V / (4 pi kc[dN]))^(1/3),
  //   V = kc[dV] + sum_j w_j y[s_j], r0 the radius at V = kc[dV]   (kParamRadius; F the
  //   Fuchs-Sutugin factor; 0 when kc[dN] = 0).
  // Partials: P[rx_pofs[k]] = kc[k] psi / p for the reactant occurrence, then -r / p and
  // r dln(psi)/dr / (4 pi kc[dN] r^2), one per Parameter in that order.
  std::vector<int> param_ptr{0}, param;
  std::vector<double> param_w;

  // forcing: f_t = sum_q term_coef[q] * r[term_rxn[q]], q in [term_ptr[t], term_ptr[t+1])
  std::vector<int> term_ptr, term_rxn;
  std::vector<double> term_coef;

  // filled pattern, CSR in elimination order
  std::vector<int> row_ptr, col, diag;
  std::vector<char> pattern0;

  // Jacobian: J[s] = sum_q jc_coef[q] * P[jc_part[q]], q in [jc_ptr[s], jc_ptr[s+1])
  std::vector<int> jc_ptr, jc_part;
  std::vector<double> jc_coef;

  // LU (Crout, one task per computed entry) and solves, in level order
  std::vector<Task> lu_tasks, fwd_tasks, bwd_tasks;
  std::vector<int> lu_level_ptr, fwd_level_ptr, bwd_level_ptr;
  std::vector<int> lu_pa, lu_pb;        // LU pairs: M[pa] * M[pb]
  std::vector<int> fwd_pa, fwd_pb;      // forward pairs: M[pa] * x[pb]
  std::vector<int> bwd_pa, bwd_pb;      // backward pairs: M[pa] * x[pb]

  int lu_levels() const { return (int)lu_level_ptr.size() - 1; }
  int fwd_levels() const { return (int)fwd_level_ptr.size() - 1; }
  int bwd_levels() const { return (int)bwd_level_ptr.size() - 1; }
};

// Compact copies of the tables the wavefront engine reads at every step, in one byte block
// laid out so a workgroup can copy it into LDS with 16-byte loads. 16-bit indices: requires
// N < 1023 (10-bit reactant fields) and Z <= 65535.
//
// The sparse LU and triangular solves are stored as term lists, level by level: every
// term is one product subtracted from one entry, so all terms of a level run in parallel.
//   LU level l:  M[dst] -= M[pa] * M[pb] for its terms; then its finalize entries:
//                M[dst] *= M[piv] for L entries (M[piv] holds the pivot's reciprocal),
//                M[dst] = 1 / M[dst] for pivots. Finalize segment 0 (before level 0)
//                inverts the pivots no elimination step touches. After the last level the
//                strict upper entries of each row are scaled by that row's reciprocal
//                pivot, so both triangular factors have a unit diagonal.
//   forward:     x[dst] -= M[slot] * x[src] (unit lower)
//   diagonal:    x[t] *= M[diag[t]]
//   backward:    x[dst] -= M[slot] * x[src] (row-scaled upper, unit diagonal)
// Layout: rx u32 [R]; diag u16 [N]; sf/sb terms uint2 {dst | src << 16, slot}; LU terms
// uint2 {dst | pa << 16, pb}; finalize u32 {dst | piv << 16} (piv 0xFFFF: invert) with
// pointers u32 [levels + 2]; row scaling u32 {slot | piv << 16}.
// The product terms of each level (and the forcing / Jacobian lists) are stored as W
// per-wavefront lists (W = wave_lists: 1 for one wavefront per cell, 2 or 4 for a
// workgroup per cell); all terms of one destination are in one list, so the order in
// which they accumulate is fixed. Pointers u32 [W * levels + 1]: list a of level l spans
// [ptr[W l + a], ptr[W l + a + 1]).
// Dense tail (tail_k = K > 0, s = N - K): the trailing K x K block is stored in full. The
// LU levels then compute, for entries of that block, only the Schur complement
//   S_ij = M_ij - sum_{k < s} L_ik U_kj
// (no pivot division, no pivot inversion), and after the levels the block is inverted in
// place by Gauss-Jordan elimination (K steps), leaving S^-1. Rows below s are factored as
// usual. A solve is then: forward sweep over the head rows and the tail rows' L entries in
// head columns; t = S^-1 x[s..N) (the tail terms {slot | i << 16 | j << 24}: t[i] +=
// M[slot] x[s + j]); head rows scaled by their reciprocal pivots, x[s + i] = t[i]; backward
// sweep over the head rows. This replaces the tail's chain of one-row sweep levels by one
// level. The tail terms are stored as W per-wavefront lists, whole rows per list, with
// pointers u32 [W + 1]; the tail row i's columns are the slots rs[i] .. rs[i] + K - 1
// (u16 [K]); LU levels of the layout: n_lu_lev.
//
// The block has a core part (the above) followed by an extension with the forcing terms
// (u32 {species | reaction << 16}, coef f64) and the Jacobian contributions
// (u32 {slot | partial << 16}, coef f64), W lists each with pointers u32 [W + 1], so a
// workgroup may stage only the core when the whole block does not fit. Every list is
// interleaved by destination (see interleave_by_dst).
struct StageBlock {
  std::vector<uint8_t> bytes;
  int core_bytes = 0;
  int off_rx = 0, off_diag = 0;
  int off_sf = 0, off_sf_lp = 0, off_sb = 0, off_sb_lp = 0;
  int off_lt = 0, off_lt_lp = 0, off_lf = 0, off_lf_lp = 0, off_us = 0;
  int n_sf_lev = 0, n_sb_lev = 0, n_us = 0;
  int off_ft = 0, off_ft_coef = 0, off_jt = 0, off_jt_coef = 0, n_ft = 0, n_jt = 0;
  int off_ft_lp = 0, off_jt_lp = 0;
  int wave_lists = 1;
  int n_lu_lev = 0;
  int tail_k = 0, tail_s = 0, off_tail = 0, off_tail_lp = 0, n_tail = 0;
  int off_tail_rs = 0;   // u16 [K]: slot of the first tail column of tail row i
  bool ok = false;   // false when the mechanism exceeds the 16-bit index ranges
};

// Largest dense tail a layout supports. Gauss-Jordan gives wavefront w of W the rows
// i = w, w + W, ...; its lanes are split into max(1, 64 / K) groups of K lanes, lane j of a
// group owning column j of every group-th row; a lane holds at most kTailPerLane entries.
// It also needs 4K doubles of scratch.
// Measured: 4 entries per lane (C5 on four wavefronts: a 27 x 27 tail, two lane groups of 27)
// run 10 % faster than 10, from the registers and unrolled slots the tail loops no longer take.
constexpr int kTailPerLane = 4;
constexpr int kTailPerLaneOneWave = 4;
int max_tail(int wave_lists);

// wave_lists: per-wavefront term lists per level, 1 (one wavefront per cell), 2 or 4 (one
// workgroup of that many wavefronts per cell). use_tail: apply the dense tail (C.tail_k,
// limited to max_tail(wave_lists)); false builds the plain LU and solve tables.
StageBlock build_stage_block(const Compiled& C, int wave_lists, bool use_tail);

// Host emulation of a stage block's table program, level by level, for validation:
// factors m[Z] (a Newton matrix in slot order) in place, then solves the system for
// x[N] (elimination order) in place. Returns false if a pivot is zero or not finite.
bool emulate_factor_solve(const Compiled& C, const StageBlock& sb, double* m, double* x);

// A mechanism description read from JSON (see mech_json.cpp): the arrays camp_mech_load takes.
struct MechDescription {
  struct Species {
    std::string name;
    int phase = -1;
    double mw = 0.1, diff = 1e-5, accom = 0.1;
  };
  struct Phase {
    std::string name;
    std::vector<int> species;
    int n_instances = 1;
    double density = 1000.0, mw_absorber = 0.2;
    int radius_from_state = 0;
  };
  std::vector<Species> species;
  std::vector<Phase> phases;
  std::vector<camp_reaction> reactions;
};
// Empty string on success, else the error (with the offending element).
std::string parse_mechanism_json(const char* text, size_t len, MechDescription& out);

// Packed compiled mechanism (see mech_pack.cpp); stage points to the four table blocks.
std::vector<uint8_t> pack_compiled(const Compiled& C, const StageBlock* stage);
std::string unpack_compiled(const uint8_t* buf, size_t size, Compiled& C, StageBlock* stage);

// Returns an empty string on success, else the validation/compile error.
std::string compile_mechanism(const camp_reaction* rxns, int n_rxn, const camp_species* sp,
                              int n_sp, const camp_phase* ph, int n_ph, Compiled& out);

}  // namespace camp
