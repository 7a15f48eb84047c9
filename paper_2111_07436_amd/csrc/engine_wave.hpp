// Fused persistent engine: device code shared by the translation units that instantiate it
// (engine_wave.hip, engine_wave_k*.hip).
//
// Every cell's whole integration over the host step (rate constants, then BDF steps with
// forcing, Newton matrix, sparse LU and triangular solves, error test and step/order
// control) runs inside one kernel. A group of G lanes owns one cell at a time: one
// wavefront (G = 64, several cells per workgroup) or a whole workgroup of 2 or 4
// wavefronts (G = 128, 256). The cell's Newton matrix, state, right-hand side, rates and
// partial derivatives live in LDS; its BDF history lives in registers, species t on group
// lane t % G. Sparse work runs as term lists built on the host, level by level: every
// product term of a level is one lane's work, accumulated into LDS, and levels are
// separated by a group barrier. Control decisions use group reductions, so every lane of
// the group takes the same path.
//
// The wavefronts of a workgroup share one LDS copy of the tables they stage (launch modes
// 1, 2, 4). When a cell is done the group takes the next one from a device-side queue
// (persistent grid) or from the grid index.
//
// Forcing and Jacobian (paper Sect. 2.4.2): f_i = sum_k S_ik r_k and
// J_ij = sum_k S_ik dr_k/dy_j, with r_k = k_k prod y over reactant occurrences.
#pragma once

#include "bdf_common.hpp"
#include "camp.h"
#include "mech.hpp"

namespace camp {

// Arguments of one fused-kernel launch.
struct WaveParams {
  const DevMech& m;
  const DevEnv& env;
  double* state;
  int n_cells;
  const SolveParams& sp;
  int* status;
  camp_cell_stats* stats;
  int* queue;
  double* kc_glob;
  int grid, waves;
  size_t lds;
  bool attr_only;   // set the launch attributes only
  hipStream_t stream;
};

namespace {

// Orders LDS traffic of one wavefront: LDS instructions of a wavefront execute in order,
// so a release/acquire fence at wavefront scope is all that lanes need to see each
// other's writes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront-uniform copy of a value every lane holds.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// LDS accumulation: several lanes of one instruction may target the same entry.
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// The lanes that integrate one cell: one wavefront (G = 64, several cells per workgroup),
// or a whole workgroup of G / 64 wavefronts (G = 128 or 256, one cell per workgroup).
// Control decisions come from group-wide reductions, so every lane of the group takes the
// same path.
template <int G>
struct Group {
  static_assert(G == 64 || G == 128 || G == 256, "lanes per cell");
  static constexpr int kWaves = G / kWave;
  // Orders the LDS (and global scratch) traffic of the group's lanes.
  __device__ static void sync() {
    if constexpr (G == kWave) wave_sync();
    else __syncthreads();
  }
  // Sum over the group, the same value in every lane. red: kWaves doubles of LDS.
  __device__ static double sum(double v, double* red) {
    v = wave_sum(v);
    if constexpr (G == kWave) {
      return v;
    } else {
      if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
      __syncthreads();
      double t = red[0];
#pragma unroll
      for (int k = 1; k < kWaves; ++k) t += red[k];
      __syncthreads();
      return t;
    }
  }
  // Nonzero in any lane of the group.
  __device__ static int any(int v, double* red) {
    const int a = wave_or(v);
    if constexpr (G == kWave) {
      return a;
    } else {
      if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = a ? 1.0 : 0.0;
      __syncthreads();
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < kWaves; ++k) t += red[k];
      __syncthreads();
      return t != 0.0;
    }
  }
};

// One update of a term loop: add `v` to entry `dst`.
struct TermUpdate {
  int dst;
  double v;
};

// Runs the terms i = lo + lane, lo + lane + G, ... < hi of a term list (G lanes) in groups
// of kU: the loads of a group (gather) are all issued before any of its updates (scatter),
// so their latencies overlap. Only valid where no term of the list reads what another
// writes.
template <int kU, int G, class Gather, class Scatter>
__device__ __forceinline__ void for_terms(int lo, int hi, int lane, Gather gather, Scatter scatter) {
  int i = lo + lane;
  for (; i + (kU - 1) * G < hi; i += kU * G) {
    TermUpdate it[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) it[u] = gather(i + u * G);
#pragma unroll
    for (int u = 0; u < kU; ++u) scatter(it[u]);
  }
  for (; i < hi; i += G) scatter(gather(i));
}

// A table entry of a term loop as loaded: packed indices, a second index word and a
// coefficient (fields a loop does not use stay 0).
struct TermEntry {
  uint32_t e;
  uint32_t x;
  double c;
};

// for_terms in three phases per group, each closed by a scheduling barrier: the table
// entries of the group are loaded (entry), then one LDS datum per entry (load), then the
// updates are formed (make) and applied (scatter). Without the barriers the compiler,
// short of registers, chains each entry load to its data read and each data read to its
// use; with them a group costs one table round trip and one LDS round trip.
// One group of kU terms i, i + G, ... of for_terms_split.
template <int kU, int G, class Entry, class Load, class Make, class Scatter>
__device__ __forceinline__ void term_group(int i, Entry entry, Load load, Make make,
                                           Scatter scatter) {
  TermEntry e[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) e[u] = entry(i + u * G);
  __builtin_amdgcn_sched_barrier(0);
  double d[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) d[u] = load(e[u]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kU; ++u) scatter(make(e[u], d[u]));
}

// The remainder after the groups of kU runs as groups of 2, then single terms.
template <int kU, int G, class Entry, class Load, class Make, class Scatter>
__device__ __forceinline__ void for_terms_split(int lo, int hi, int lane, Entry entry, Load load,
                                                Make make, Scatter scatter) {
  int i = lo + lane;
  for (; i + (kU - 1) * G < hi; i += kU * G) term_group<kU, G>(i, entry, load, make, scatter);
  for (; i + G < hi; i += 2 * G) term_group<2, G>(i, entry, load, make, scatter);
  for (; i < hi; i += G) term_group<1, G>(i, entry, load, make, scatter);
}

constexpr int kTermBatch = 4;

// Product terms i = lo + lane, lo + lane + 64, ... < hi of one wavefront's list, in groups of
// kU per lane: the table entries of a group first, then the two LDS operands of each
// (operands(e) -> double2), then the updates (apply(e, operands)), phases held apart by
// scheduling barriers so a group costs one table and one LDS round trip. Only valid where
// no term of the list reads what another writes.
template <int kU, class Entry, class Operands, class Apply>
__device__ __forceinline__ void product_group(int i, Entry entry, Operands operands, Apply apply) {
  uint2 e[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) e[u] = entry(i + u * kWave);
  __builtin_amdgcn_sched_barrier(0);
  double2 v[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) v[u] = operands(e[u]);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < kU; ++u) apply(e[u], v[u]);
}
template <int kU, class Entry, class Operands, class Apply>
__device__ __forceinline__ void for_products(int lo, int hi, int lane, Entry entry, Operands operands,
                                             Apply apply) {
  int i = lo + lane;
  for (; i + (kU - 1) * kWave < hi; i += kU * kWave) product_group<kU>(i, entry, operands, apply);
  for (; i + kWave < hi; i += 2 * kWave) product_group<2>(i, entry, operands, apply);
  for (; i < hi; i += kWave) product_group<1>(i, entry, operands, apply);
}

// Level pointers of a term list held in registers: lane k holds entry k and entry k + 64,
// so reading the bounds of a level is a lane read instead of an LDS round trip. Lists of
// more than 127 levels read the rest from the table.
struct LevelPtrs {
  int a, b;
};

// Loads entries 0..nlev of a level-pointer table (ptr(l) reads entry l); entry 0 is 0.
template <class Ptr>
__device__ __forceinline__ LevelPtrs load_levels(int nlev, Ptr ptr) {
  const int lane = threadIdx.x % kWave;
  LevelPtrs p{0, 0};
  if (lane <= nlev) p.a = ptr(lane);
  if (lane + kWave <= nlev) p.b = ptr(lane + kWave);
  return p;
}

template <class Ptr>
__device__ __forceinline__ int level_ptr(const LevelPtrs& p, int l, Ptr ptr) {
  if (l < kWave) return __builtin_amdgcn_readlane(p.a, l);
  if (l < 2 * kWave) return __builtin_amdgcn_readlane(p.b, l - kWave);
  return uniform(ptr(l));
}

// Bounds of one wavefront's term list in each level of a table with kW lists per level
// (list a of level l spans [ptr(kW l + a), ptr(kW l + a + 1))), held in registers like
// LevelPtrs: lane k holds the bounds of levels k and k + 64.
struct LevelRange {
  int s0, e0, s1, e1;
};

template <int kW, class Ptr>
__device__ __forceinline__ LevelRange load_ranges(int nlev, int wid, Ptr ptr) {
  const int l = threadIdx.x % kWave;
  LevelRange r{0, 0, 0, 0};
  if (l < nlev) {
    r.s0 = ptr(kW * l + wid);
    r.e0 = ptr(kW * l + wid + 1);
  }
  if (l + kWave < nlev) {
    r.s1 = ptr(kW * (l + kWave) + wid);
    r.e1 = ptr(kW * (l + kWave) + wid + 1);
  }
  return r;
}

template <int kW, class Ptr>
__device__ __forceinline__ int2 level_range(const LevelRange& r, int l, int wid, Ptr ptr) {
  if (l < kWave)
    return make_int2(__builtin_amdgcn_readlane(r.s0, l), __builtin_amdgcn_readlane(r.e0, l));
  if (l < 2 * kWave)
    return make_int2(__builtin_amdgcn_readlane(r.s1, l - kWave),
                     __builtin_amdgcn_readlane(r.e1, l - kWave));
  return make_int2(uniform(ptr(kW * l + wid)), uniform(ptr(kW * l + wid + 1)));
}

// Accessors of the compact table block: the core tables through `b`, the forcing-term and
// Jacobian-contribution extension through `e`; each base is LDS (staged) or global memory.
struct Tabs {
  const char* b;
  const char* e;
  const StageView& v;
  __device__ uint32_t ft(int i) const { return reinterpret_cast<const uint32_t*>(e + v.so_ft)[i]; }
  __device__ double ft_coef(int i) const { return reinterpret_cast<const double*>(e + v.so_ft_coef)[i]; }
  __device__ uint32_t jt(int i) const { return reinterpret_cast<const uint32_t*>(e + v.so_jt)[i]; }
  __device__ int ft_lp(int a) const { return (int)reinterpret_cast<const uint32_t*>(e + v.so_ft_lp)[a]; }
  __device__ int jt_lp(int a) const { return (int)reinterpret_cast<const uint32_t*>(e + v.so_jt_lp)[a]; }
  __device__ double jt_coef(int i) const { return reinterpret_cast<const double*>(e + v.so_jt_coef)[i]; }
  __device__ uint32_t rx(int k) const { return reinterpret_cast<const uint32_t*>(b + v.so_rx)[k]; }
  __device__ int dg(int t) const { return reinterpret_cast<const uint16_t*>(b + v.so_diag)[t]; }
  __device__ uint2 sf(int i) const { return reinterpret_cast<const uint2*>(b + v.so_sf)[i]; }
  __device__ int sf_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + v.so_sf_lp)[l]; }
  __device__ uint2 sb(int i) const { return reinterpret_cast<const uint2*>(b + v.so_sb)[i]; }
  __device__ int sb_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + v.so_sb_lp)[l]; }
  __device__ uint2 lt(int i) const { return reinterpret_cast<const uint2*>(b + v.so_lt)[i]; }
  __device__ int lt_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + v.so_lt_lp)[l]; }
  __device__ uint32_t lf(int i) const { return reinterpret_cast<const uint32_t*>(b + v.so_lf)[i]; }
  __device__ int lf_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + v.so_lf_lp)[l]; }
  __device__ uint32_t us(int i) const { return reinterpret_cast<const uint32_t*>(b + v.so_us)[i]; }
  __device__ uint32_t tl(int i) const { return reinterpret_cast<const uint32_t*>(b + v.so_tail)[i]; }
  __device__ int tl_lp(int a) const { return (int)reinterpret_cast<const uint32_t*>(b + v.so_tail_lp)[a]; }
  __device__ int tl_rs(int i) const { return reinterpret_cast<const uint16_t*>(b + v.so_tail_rs)[i]; }
};

template <int NPL, int G, bool kPar = false>
struct WaveCell {
  // Terms per lane issued together in the LU and sweep levels: levels of large mechanisms
  // hold several terms per lane, small ones rarely more than one.
  static constexpr int kLevelBatch = NPL >= 4 ? 4 : 1;
  // Levels whose first table entries are read together (sweeps, LU). Measured: the
  // one-wavefront kernels of up to three species per lane and the four-wavefront kernels
  // are fastest with short windows (registers are tight there), the others with 8.
  static constexpr int kWindow = (G == kWave && NPL <= 3) ? 2 : G == 4 * kWave ? 3 : 8;
  // Dense-tail entries per lane (see tail_invert; max_tail bounds K to fit).
  static constexpr int kTail = G == kWave ? kTailPerLaneOneWave : kTailPerLane;
  // Product terms per lane issued together beyond a level's first. Measured: 2 where
  // registers are tightest (the one-wavefront kernels of at most three species per lane,
  // 2 % faster than 4 on 192 state variables, and the four-wavefront kernels, 2 % faster
  // on 520 state variables, where 1 and 8 are slower); kTermBatch elsewhere.
  static constexpr int kProdBatch = ((G == kWave && NPL <= 3) || G == 4 * kWave) ? 2 : kTermBatch;
  const DevMech& m;
  Tabs tb;
  double* M;
  double* yl;
  double* xl;
  double* P;
  double* kc;
  double* red;   // reduction scratch of the group (8 doubles of LDS)
  int lane;      // 0 .. G-1
  static constexpr int kW = G / kWave;   // wavefronts per cell = term lists per level
  __device__ static int wlane() { return threadIdx.x % kWave; }
  __device__ static int wid() { return (threadIdx.x % G) / kWave; }

  __device__ __forceinline__ void sync() const { Group<G>::sync(); }
  __device__ __forceinline__ int any(int v) const { return Group<G>::any(v, red); }

  __device__ __forceinline__ double wrms(const double (&v)[NPL], const double (&w)[NPL]) const {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i)
      if (lane + G * i < m.N) {
        double a = v[i] * w[i];
        s += a * a;
      }
    return sqrt(Group<G>::sum(s, red) / m.N);
  }

  // Concentration factors of reaction entry t (packed reactant slots, 0x3FF = absent):
  // the three LDS reads are issued unconditionally (an absent slot reads y[0]); yfac then
  // turns an absent reactant's factor into 1, which leaves a product bit for bit unchanged.
  __device__ __forceinline__ void yload(uint32_t e, double (&y)[3]) const {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int a = (e >> (10 * j)) & 0x3FF;
      y[j] = yl[a != 0x3FF ? a : 0];
    }
  }
  __device__ __forceinline__ static double yfac(uint32_t e, int j, double v) {
    return ((e >> (10 * j)) & 0x3FF) != 0x3FF ? v : 1.0;
  }

  // Reactions k = lane, lane + G, ... in groups of kTermBatch per lane: table entries of a
  // group (entry), then its concentration reads, then use(entry, factors), with scheduling
  // barriers between the phases as in for_terms_split.
  template <int kU, class Entry, class Use>
  __device__ __forceinline__ void reaction_group(int k, Entry entry, Use use) const {
    TermEntry e[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) e[u] = entry(k + u * G);
    __builtin_amdgcn_sched_barrier(0);
    double y[kU][3];
#pragma unroll
    for (int u = 0; u < kU; ++u) yload(e[u].e, y[u]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kU; ++u) use(e[u], y[u]);
  }
  template <class Entry, class Use>
  __device__ __forceinline__ void for_reactions(Entry entry, Use use) const {
    int k = lane;
    for (; k + (kTermBatch - 1) * G < m.R; k += kTermBatch * G)
      reaction_group<kTermBatch>(k, entry, use);
    for (; k + G < m.R; k += 2 * G) reaction_group<2>(k, entry, use);
    for (; k < m.R; k += G) reaction_group<1>(k, entry, use);
  }

  // P[k] = r_k from yl; then f for owned species, accumulated term by term (one term per
  // lane) in xl, which no caller holds live across this call. yl must be visible to all
  // lanes.
  __device__ __forceinline__ void forcing(double (&f)[NPL]) const {
    for_reactions([&](int k) { return TermEntry{tb.rx(k), (uint32_t)k, kc[k]}; },
                  [&](const TermEntry& t, const double (&y)[3]) {
                    P[t.x] = t.c * yfac(t.e, 0, y[0]) * yfac(t.e, 1, y[1]) * yfac(t.e, 2, y[2]);
                  });
    if constexpr (kPar) {   // rates with Parameters: r = kc prod(y) phi(y)
      sync();
      for (int q = lane; q < m.n_param; q += G) {
        const ParamEval pe = parameter_eval(m, q, [&](int d) { return kc[d]; },
                                            [&](int j) { return yl[j]; });
        P[pe.k] *= pe.phi;
      }
    }
    for (int t = lane; t < m.N; t += G) xl[t] = 0.0;
    sync();
    for_terms_split<kTermBatch, kWave>(
        uniform(tb.ft_lp(wid())), uniform(tb.ft_lp(wid() + 1)), wlane(),
        [&](int i) { return TermEntry{tb.ft(i), 0u, tb.ft_coef(i)}; },
        [&](const TermEntry& t) { return P[t.e >> 16]; },
        [&](const TermEntry& t, double p) { return TermUpdate{(int)(t.e & 0xFFFF), t.c * p}; },
        [&](const TermUpdate& u) { lds_add(&xl[u.dst], u.v); });
    sync();
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int t = lane + G * i;
      f[i] = t < m.N ? xl[t] : 0.0;
    }
    sync();
  }

  // M = I - c J(yl) in the filled pattern (fill slots 0 off the diagonal), accumulated
  // contribution by contribution (one per lane).
  __device__ __forceinline__ void newton_matrix(double c) const {
    // partials of each reaction's rate with respect to each reactant occurrence
    for_reactions([&](int k) { return TermEntry{tb.rx(k), (uint32_t)m.rx_pofs[k], kc[k]}; },
                  [&](const TermEntry& t, const double (&y)[3]) {
                    const double ya = yfac(t.e, 0, y[0]), yb = yfac(t.e, 1, y[1]),
                                 yc = yfac(t.e, 2, y[2]);
                    if ((t.e & 0x3FF) != 0x3FF) P[t.x] = t.c * yb * yc;
                    if (((t.e >> 10) & 0x3FF) != 0x3FF) P[t.x + 1] = t.c * ya * yc;
                    if (((t.e >> 20) & 0x3FF) != 0x3FF) P[t.x + 2] = t.c * ya * yb;
                  });
    for (int s = lane; s < m.Z; s += G) M[s] = 0.0;
    sync();
    if constexpr (kPar) {   // chain rule through the Parameters (one reactant each)
      for (int q = lane; q < m.n_param; q += G) {
        const ParamEval pe = parameter_eval(m, q, [&](int d) { return kc[d]; },
                                            [&](int j) { return yl[j]; });
        int o = m.rx_pofs[pe.k];
        const double r = kc[pe.k] * yl[m.rx_react[3 * pe.k]] * pe.phi;
        P[o++] = kc[pe.k] * pe.phi;
        if (pe.flags & 1) P[o++] = -r * pe.inv_p;
        if (pe.flags & 2) P[o] = r * pe.g;
      }
      sync();
    }
    const double mc = -c;
    for_terms_split<kTermBatch, kWave>(
        uniform(tb.jt_lp(wid())), uniform(tb.jt_lp(wid() + 1)), wlane(),
        [&](int i) { return TermEntry{tb.jt(i), 0u, tb.jt_coef(i)}; },
        [&](const TermEntry& t) { return P[t.e >> 16]; },
        [&](const TermEntry& t, double p) { return TermUpdate{(int)(t.e & 0xFFFF), mc * t.c * p}; },
        [&](const TermUpdate& u) { lds_add(&M[u.dst], u.v); });
    sync();
    for (int t = lane; t < m.N; t += G) M[tb.dg(t)] += 1.0;
    sync();
  }

  // In-place Crout LU of M, one dependency level at a time: the level's product terms in
  // parallel (one per lane), then its finalize entries (L entries times the reciprocal
  // pivot, pivots inverted). Leaves the unit-diagonal factors: L strictly below the
  // diagonal, reciprocal pivots on it, and U / diag(U) strictly above. Returns 0 if a
  // pivot is not a finite nonzero.
  __device__ __forceinline__ int lu() const {
    const int L = tb.v.n_lu_lev;
    auto ltp = [&](int k) { return tb.lt_lp(k); };
    const LevelRange tr = load_ranges<kW>(L, wid(), ltp);
    const LevelPtrs fp = load_levels(L + 1, [&](int l) { return tb.lf_lp(l); });
    int fhi = level_ptr(fp, 1, [&](int l) { return tb.lf_lp(l); });
    for (int i = lane; i < fhi; i += G) {
      const int d = tb.lf(i) & 0xFFFF;
      M[d] = 1.0 / M[d];
    }
    sync();
    if constexpr (kLevelBatch == 1) {
      // Windows of kWin levels as in sweep(): a lane's first product-term entry and first
      // finalize entry of every level of the window are read up front (an empty slot
      // reads entry 0 and is not used).
      constexpr int kWin = kWindow;
      auto prod = [&](const uint2& e) { lds_add(&M[e.x & 0xFFFF], -(M[e.x >> 16] * M[e.y])); };
      auto fin = [&](uint32_t e) {
        const int dst = e & 0xFFFF, pv = e >> 16;
        M[dst] = pv == 0xFFFF ? 1.0 / M[dst] : M[dst] * M[pv];
      };
      for (int l0 = 0; l0 < L; l0 += kWin) {
        int2 r[kWin];
        int fb[kWin + 1];
        uint2 e[kWin];
        uint32_t fe[kWin];
        fb[0] = fhi;
#pragma unroll
        for (int u = 0; u < kWin; ++u) {
          const bool on = l0 + u < L;
          r[u] = on ? level_range<kW>(tr, l0 + u, wid(), ltp) : make_int2(0, 0);
          fb[u + 1] = on ? level_ptr(fp, l0 + u + 2, [&](int k) { return tb.lf_lp(k); }) : fb[u];
          const int i = r[u].x + wlane(), j = fb[u] + lane;
          e[u] = tb.lt(i < r[u].y ? i : 0);
          fe[u] = tb.lf(j < fb[u + 1] ? j : 0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kWin; ++u) {
          if (l0 + u >= L) break;
          const int i = r[u].x + wlane();
          if (i < r[u].y) prod(e[u]);
          for_products<kProdBatch>(
              r[u].x + kWave, r[u].y, wlane(), [&](int k) { return tb.lt(k); },
              [&](const uint2& t) { return make_double2(M[t.x >> 16], M[t.y]); },
              [&](const uint2& t, const double2& v) { lds_add(&M[t.x & 0xFFFF], -(v.x * v.y)); });
          sync();
          if (fb[u] == fb[u + 1]) continue;
          const int j = fb[u] + lane;
          if (j < fb[u + 1]) fin(fe[u]);
          for (int k = j + G; k < fb[u + 1]; k += G) fin(tb.lf(k));
          sync();
        }
        fhi = fb[kWin];
      }
    } else {
      for (int l = 0; l < L; ++l) {
        const int2 r = level_range<kW>(tr, l, wid(), ltp);
        for_terms<kLevelBatch, kWave>(
            r.x, r.y, wlane(),
            [&](int i) {
              const uint2 e = tb.lt(i);
              return TermUpdate{(int)(e.x & 0xFFFF), M[e.x >> 16] * M[e.y]};
            },
            [&](const TermUpdate& u) { lds_add(&M[u.dst], -u.v); });
        sync();
        const int flo = fhi;
        fhi = level_ptr(fp, l + 2, [&](int k) { return tb.lf_lp(k); });
        if (flo == fhi) continue;
        for (int i = flo + lane; i < fhi; i += G) {
          const uint32_t e = tb.lf(i);
          const int dst = e & 0xFFFF, pv = e >> 16;
          M[dst] = pv == 0xFFFF ? 1.0 / M[dst] : M[dst] * M[pv];
        }
        sync();
      }
    }
    for (int i = lane; i < tb.v.n_us; i += G) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] *= M[e >> 16];
    }
    int bad = tb.v.tail_k ? tail_invert() : 0;
    for (int t = lane; t < tb.v.tail_s; t += G) {
      const double r = M[tb.dg(t)];
      if (!(fabs(r) > 0.0) || !isfinite(r)) bad = 1;
    }
    sync();
    return !any(bad);
  }

  // Dense tail: inverts the trailing K x K block in place (it holds the Schur complement S
  // after the levels) by Gauss-Jordan elimination without pivoting, one group barrier per
  // step. Wavefront w of the group owns the block rows i = w, w + kW, ...; its lanes form
  // max(1, 64 / K) groups of K, lane j of group g holding column j of the wavefront's rows
  // g, g + groups, ... in registers for all K steps. Step p needs row p and column p of the
  // current matrix: a copy of each sits in LDS (P, two sets alternating), and the lanes whose
  // new values form row and column p + 1 write them to the other set. With one lane group,
  // the column values of the wavefront's rows are read once and passed by lane reads.
  // Returns nonzero if a pivot is zero or not finite.
  __device__ __forceinline__ int tail_invert() const {
    const int K = tb.v.tail_k;
    const int w = wid(), l = wlane();
    const int groups = K <= kWave / 2 ? kWave / K : 1;
    const int g = l / K, j = l - g * K;
    const int rows = (K - w + kW - 1) / kW;             // rows of this wavefront
    const int n_t = g < groups ? (rows - g + groups - 1) / groups : 0;   // entries of this lane
    // block row of the lane's entry t
    auto row = [&](int t) { return w + kW * (g + groups * t); };
    double a[kTail];
#pragma unroll
    for (int t = 0; t < kTail; ++t) a[t] = t < n_t ? M[tb.tl_rs(row(t)) + j] : 0.0;
    // row 0 and column 0 of S into set 0
#pragma unroll
    for (int t = 0; t < kTail; ++t) {
      if (t >= n_t) continue;
      if (row(t) == 0) P[j] = a[t];
      if (j == 0) P[K + row(t)] = a[t];
    }
    sync();
    int bad = 0;
    for (int p = 0; p < K; ++p) {
      const double* rp = P + (p & 1) * 2 * K;          // row p
      const double* cp = rp + K;                       // column p
      double* rn = P + ((p + 1) & 1) * 2 * K;          // row p + 1 (next set)
      double* cn = rn + K;                             // column p + 1
      const double piv = rp[p];
      const double rj = rp[n_t > 0 ? j : 0];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) bad = 1;
      const double r = 1.0 / piv;
      // every entry slot is updated (fully unrolled, registers indexed by constants); slots
      // beyond the lane's entries hold unused values
      auto update = [&](int t, double ci) {
        const int i = row(t);
        const double off = i == p ? rj * r : a[t] - ci * rj * r;
        a[t] = j == p ? (i == p ? r : -ci * r) : off;
      };
      if (groups == 1) {
        const double cr = cp[l < rows ? w + kW * l : 0];
#pragma unroll
        for (int t = 0; t < kTail; ++t) update(t, lane_double(cr, t));
      } else {
#pragma unroll
        for (int t = 0; t < kTail; ++t) update(t, cp[t < n_t ? row(t) : 0]);
      }
      // row p + 1: at most one entry of this lane; column p + 1: lane j = p + 1's entries
      double vr = 0.0;
      int wr = 0;
#pragma unroll
      for (int t = 0; t < kTail; ++t)
        if (t < n_t && row(t) == p + 1) {
          vr = a[t];
          wr = 1;
        }
      if (wr) rn[j] = vr;
      if (j == p + 1) {
#pragma unroll
        for (int t = 0; t < kTail; ++t)
          if (t < n_t) cn[row(t)] = a[t];
      }
      sync();
    }
#pragma unroll
    for (int t = 0; t < kTail; ++t)
      if (t < n_t) M[tb.tl_rs(row(t)) + j] = a[t];
    return bad;
  }

  __device__ __forceinline__ int newton_matrix_lu(double c) const {
    newton_matrix(c);
    return lu();
  }

  // Conversions between the factor form lu() leaves and the conventional one (unit L
  // strictly below the diagonal, U on and above it).
  __device__ __forceinline__ void factors_to_conventional() const {
    for (int i = lane; i < tb.v.n_us; i += G) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] /= M[e >> 16];
    }
    sync();
    for (int t = lane; t < m.N; t += G) M[tb.dg(t)] = 1.0 / M[tb.dg(t)];
    sync();
  }
  __device__ __forceinline__ void factors_from_conventional() const {
    for (int t = lane; t < m.N; t += G) M[tb.dg(t)] = 1.0 / M[tb.dg(t)];
    sync();
    for (int i = lane; i < tb.v.n_us; i += G) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] *= M[e >> 16];
    }
    sync();
  }

  // One triangular sweep over the unit-diagonal factor: x[dst] -= M[slot] * x[src] for
  // the terms of each level, one term per lane.
  template <bool kForward>
  __device__ __forceinline__ void sweep() const {
    const int nlev = kForward ? tb.v.n_sf_lev : tb.v.n_sb_lev;
    auto lp = [&](int l) { return kForward ? tb.sf_lp(l) : tb.sb_lp(l); };
    const LevelRange p = load_ranges<kW>(nlev, wid(), lp);
    if constexpr (kLevelBatch == 1) {
      // Levels of about one term per lane, in windows of kWin levels: a lane's first table
      // entry of every level of the window is read up front (one round trip per window;
      // an empty slot reads entry 0 and is not used), so a level then costs one LDS round
      // trip for its data. Tables are read-only, and each level's data reads still follow
      // the previous level's updates.
      constexpr int kWin = kWindow;
      auto ent = [&](int i) { return kForward ? tb.sf(i) : tb.sb(i); };
      auto term = [&](const uint2& e) { lds_add(&xl[e.x & 0xFFFF], -(M[e.y] * xl[e.x >> 16])); };
      for (int l0 = 0; l0 < nlev; l0 += kWin) {
        int2 r[kWin];
        uint2 e[kWin];
#pragma unroll
        for (int u = 0; u < kWin; ++u) {
          r[u] = l0 + u < nlev ? level_range<kW>(p, l0 + u, wid(), lp) : make_int2(0, 0);
          const int i = r[u].x + wlane();
          e[u] = ent(i < r[u].y ? i : 0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kWin; ++u) {
          if (l0 + u >= nlev) break;
          const int i = r[u].x + wlane();
          if (i < r[u].y) term(e[u]);
          for_products<kProdBatch>(
              r[u].x + kWave, r[u].y, wlane(), ent,
              [&](const uint2& t) { return make_double2(M[t.y], xl[t.x >> 16]); },
              [&](const uint2& t, const double2& v) { lds_add(&xl[t.x & 0xFFFF], -(v.x * v.y)); });
          sync();
        }
      }
      return;
    }
    for (int l = 0; l < nlev; ++l) {
      const int2 r = level_range<kW>(p, l, wid(), lp);
      for_terms<kLevelBatch, kWave>(
          r.x, r.y, wlane(),
          [&](int i) {
            const uint2 e = kForward ? tb.sf(i) : tb.sb(i);
            return TermUpdate{(int)(e.x & 0xFFFF), M[e.y] * xl[e.x >> 16]};
          },
          [&](const TermUpdate& u) { lds_add(&xl[u.dst], -u.v); });
      sync();
    }
  }

  // xl <- (LU)^-1 xl from the factors lu() leaves: forward sweep, diagonal scaling,
  // backward sweep.
  // With a dense tail the block's unknowns come from t = S^-1 x[s..N) between the sweeps
  // (accumulated in P, whole rows per wavefront so each sum has a fixed order).
  __device__ __forceinline__ void solve() const {
    const int K = tb.v.tail_k, ts = tb.v.tail_s;
    for (int i = lane; i < K; i += G) P[i] = 0.0;
    if (K && tb.v.n_sf_lev == 0) sync();
    sweep<true>();
    if (K) {
      for_terms<kTermBatch, kWave>(
          uniform(tb.tl_lp(wid())), uniform(tb.tl_lp(wid() + 1)), wlane(),
          [&](int i) {
            const uint32_t e = tb.tl(i);
            return TermUpdate{(int)((e >> 16) & 0xFF), M[e & 0xFFFF] * xl[ts + (e >> 24)]};
          },
          [&](const TermUpdate& u) { lds_add(&P[u.dst], u.v); });
      sync();
    }
    for (int t = lane; t < m.N; t += G) xl[t] = t < ts ? xl[t] * M[tb.dg(t)] : P[t - ts];
    sync();
    sweep<false>();
  }
};

// Step change by rho: D[1..q] become the backward differences at the new spacing of the
// polynomial interpolating the history (rescale_point / rescale_differences).
template <int NPL>
__device__ __forceinline__ void rescale_hist(double (&D)[kHist][NPL], int q, double rho) {
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    double a[kMaxOrder + 1];
#pragma unroll
    for (int mm = 0; mm <= kMaxOrder; ++mm) {
      double acc = 0.0;
#pragma unroll
      for (int k = kMaxOrder; k >= 1; --k)
        if (k <= q) acc = rescale_coef(k, mm, rho) * (D[k][i] + acc);
      a[mm] = D[0][i] + acc;
    }
#pragma unroll
    for (int lev = 1; lev <= kMaxOrder; ++lev) {
#pragma unroll
      for (int mm = 0; mm + lev <= kMaxOrder; ++mm) a[mm] -= a[mm + 1];
      if (lev <= q) D[lev][i] = a[0];
    }
  }
}

// Integrates one cell over the host step from its input row (rate constants already in
// LDS; `bad` flags a non-finite rate constant on this lane). full != 0: full Newton, with a
// fresh Jacobian and LU at every iteration; else Newton with Jacobian reuse. On success
// the state row is overwritten; on failure it is left as it was.
template <int NPL, int G, bool kPar>
__device__ __forceinline__ int integrate(const DevMech& m, double* yrow, const SolveParams& sp, int bad, int full,
                         camp_cell_stats& cs, const WaveCell<NPL, G, kPar>& W) {
  const int lane = W.lane;
  const int N = m.N;
  int status = ST_OK;

  // ---- initial state ----
  double D[kHist][NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int t = lane + G * i;
    const double v = t < N ? start_value(yrow[m.perm[t]], sp.rtol, sp.atol_call) : 0.0;
    if (t < N) {
      W.yl[t] = v;
      if (!isfinite(v)) bad = 1;
    }
    D[0][i] = v;
#pragma unroll
    for (int j = 1; j < kHist; ++j) D[j][i] = 0.0;
  }
  W.sync();
  if (W.any(bad)) status = ST_NONFINITE;

  const double span = sp.dt;
  double w[NPL], f0[NPL], d[NPL];
  if (status == ST_OK) {
    W.forcing(f0);
    cs.n_f++;
    int nf = 0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      if (!isfinite(f0[i])) nf = 1;
      const double s = sp.atol + sp.rtol * fabs(D[0][i]);
      w[i] = s > 0.0 ? 1.0 / s : 0.0;
    }
    if (W.any(nf)) status = ST_NONFINITE;
  }
  double h = 0.0;
  if (status == ST_OK) {
    // starting step
    const double d0 = W.wrms(D[0], w), d1 = W.wrms(f0, w);
    const double h0 = starting_step_h0(d0, d1, span);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int t = lane + G * i;
      if (t < N) W.yl[t] = D[0][i] + h0 * f0[i];
    }
    W.sync();
    double f1[NPL];
    W.forcing(f1);
    cs.n_f++;
#pragma unroll
    for (int i = 0; i < NPL; ++i) f1[i] -= f0[i];
    const double d2 = W.wrms(f1, w) / h0;
    h = sp.h_init > 0.0 ? fmin(sp.h_init, span) : starting_step(h0, d1, d2, span);
#pragma unroll
    for (int i = 0; i < NPL; ++i) D[1][i] = h * f0[i];
  }

  int q = 1, n_equal = 0, attempts = 0, lu_valid = 0, lu_age = 0;
  double t = 0.0, c_lu = 0.0, crate = 1.0, err = 0.0;
  while (status == ST_OK && t < span) {
    if (span - (t + h) <= 1e-12 * span) {
      const double rho = (span - t) / h;
      if (rho != 1.0) {
        rescale_hist(D, q, rho);
        h = span - t;
        n_equal = 0;
      }
    }
    int nfw = 0;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      w[i] = 1.0 / (sp.rtol * fabs(D[0][i]) + sp.atol);
      if (lane + G * i < N && !isfinite(w[i])) nfw = 1;
    }
    if (W.any(nfw)) {
      status = ST_NONFINITE;
      break;
    }
    int consec_err = 0, consec_nf = 0, force_lu = 0;
    bool accepted = false;
    while (true) {
      if (++attempts > sp.max_steps) { status = ST_MAX_STEPS; break; }
      if (step_collapsed(h, t, sp.h_min)) { status = ST_H_MIN; break; }
      const double gq = bdf_gamma(q);
      const double c = h / gq, inv_gq = 1.0 / gq;
      double psi[NPL], yv[NPL];
#pragma unroll
      for (int i = 0; i < NPL; ++i) {
        double s = D[0][i], ps = 0.0, g = 0.0;
#pragma unroll
        for (int j = 1; j <= kMaxOrder; ++j) {
          g += 1.0 / j;
          if (j <= q) {
            s += D[j][i];
            ps += g * D[j][i];
          }
        }
        psi[i] = ps * inv_gq;
        yv[i] = s;
        d[i] = 0.0;
        const int tt = lane + G * i;
        if (tt < N) W.yl[tt] = s;
      }
      W.sync();
      int fresh = 0, lu_ok = 1;
      if (force_lu || !lu_valid || fabs(c / c_lu - 1.0) > sp.lu_drift || lu_age >= sp.lu_max_age) {
        lu_ok = W.newton_matrix_lu(c);
        cs.n_jac++;
        cs.n_lu++;
        lu_valid = lu_ok;
        c_lu = c;
        lu_age = 0;
        crate = 1.0;
        fresh = 1;
      }
      bool conv = false;
      int nonfin = 0;
      if (lu_ok) {
        double dn_old = 0.0;
        for (int it = 0; it < sp.newton_maxit; ++it) {
          if (it > 0) {
#pragma unroll
            for (int i = 0; i < NPL; ++i) {
              const int tt = lane + G * i;
              if (tt < N) W.yl[tt] = yv[i];
            }
            W.sync();
          }
          if (full && (it > 0 || !fresh)) {
            lu_ok = W.newton_matrix_lu(c);   // Jacobian at the current iterate
            cs.n_jac++;
            cs.n_lu++;
            lu_valid = lu_ok;
            c_lu = c;
            lu_age = 0;
            crate = 1.0;
            fresh = 1;
            if (!lu_ok) break;
          }
          const double scale = (c == c_lu) ? 1.0 : 2.0 / (1.0 + c / c_lu);
          double f[NPL];
          W.forcing(f);
          cs.n_f++;
          int nf = 0;
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            const int tt = lane + G * i;
            if (tt < N) {
              if (!isfinite(f[i])) nf = 1;
              W.xl[tt] = c * f[i] - psi[i] - d[i];
            }
          }
          if (W.any(nf)) { nonfin = 1; break; }
          W.sync();
          W.solve();
          double dl[NPL];
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            const int tt = lane + G * i;
            dl[i] = tt < N ? W.xl[tt] * scale : 0.0;
          }
          W.sync();
          const double dn = W.wrms(dl, w);
          cs.newton_iters++;
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            yv[i] += dl[i];
            d[i] += dl[i];
          }
          if (!isfinite(dn)) break;
          if (it > 0) crate = fmax(0.3 * crate, dn / dn_old);
          const double dcon = dn * fmin(1.0, crate) / sp.newton_tol;
          if (dcon <= 1.0) { conv = true; break; }
          if (it > 0 && dn > kNewtonDiverge * dn_old) break;
          dn_old = dn;
        }
      }
      if (nonfin) { status = ST_NONFINITE; break; }
      if (!conv) {
        if (!fresh && lu_ok) { force_lu = 1; continue; }
        cs.newton_fail++;
        if (++consec_nf >= kMaxConsecFail) { status = ST_NEWTON_FAIL; break; }
        rescale_hist(D, q, 0.25);
        h *= 0.25;
        n_equal = 0;
        force_lu = 0;
        continue;
      }
      force_lu = 0;
      // positivity constraint: a converged solution more than one tolerance unit below
      // zero is rejected and retried with a smaller step (values are never clipped)
      int neg = 0;
#pragma unroll
      for (int i = 0; i < NPL; ++i)
        if (lane + G * i < N && yv[i] * w[i] < -1.0) neg = 1;
      if (W.any(neg)) {
        // a component that starts negative only counts if it is also more than one
        // tolerance unit below its start value (read back from the input row, which holds
        // the input until the cell finishes)
        neg = 0;
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          const int tt = lane + G * i;
          if (tt < N && yv[i] * w[i] < -1.0 &&
              (yv[i] - fmin(0.0, start_value(yrow[m.perm[tt]], sp.rtol, sp.atol_call))) * w[i] <
                  -1.0)
            neg = 1;
        }
      }
      if (W.any(neg)) {
        cs.rejected++;
        rescale_hist(D, q, kConstraintFactor);
        h *= kConstraintFactor;
        n_equal = 0;
        continue;
      }
      double dq1[NPL];
      const double inv_q1 = 1.0 / (q + 1);
#pragma unroll
      for (int i = 0; i < NPL; ++i) dq1[i] = d[i] * inv_q1;
      err = W.wrms(dq1, w);
      if (err > 1.0) {
        cs.rejected++;
        if (++consec_err >= kMaxConsecFail) { status = ST_ERR_FAIL; break; }
        n_equal = 0;
        if (consec_err >= kErrRestart) {
          // restart at order 1 from y_n with a much smaller step: D[1] = h f(y_n)
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            const int tt = lane + G * i;
            if (tt < N) W.yl[tt] = D[0][i];
          }
          W.sync();
          double fn[NPL];
          W.forcing(fn);
          cs.n_f++;
          h *= kRestartFactor;
          q = 1;
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            D[1][i] = h * fn[i];
#pragma unroll
            for (int j = 2; j < kHist; ++j) D[j][i] = 0.0;
          }
          continue;
        }
        double rho = fmax(kMinFactor, kSafety * pow(err, -1.0 / (q + 1)));
        if (consec_err >= 2) rho = fmin(rho, kMinFactor);
        rescale_hist(D, q, rho);
        h *= rho;
        continue;
      }
      accepted = true;
      break;
    }
    if (!accepted) break;

    // ---- accept: advance time and update the differences ----
    cs.steps++;
    lu_age++;
    t = (span - (t + h) <= 1e-12 * span) ? span : t + h;
    n_equal++;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      double old_q1 = 0.0;
#pragma unroll
      for (int j = 1; j < kHist; ++j)
        if (j == q + 1) old_q1 = D[j][i];
      double s = d[i];
#pragma unroll
      for (int j = kMaxOrder; j >= 0; --j)
        if (j <= q) {
          s += D[j][i];
          D[j][i] = s;
        }
#pragma unroll
      for (int j = 1; j < kHist; ++j) {
        if (j == q + 1) D[j][i] = d[i];
        if (j == q + 2) D[j][i] = d[i] - old_q1;
      }
    }
    if (t >= span) break;
    if (n_equal < q + 1) continue;
    double vm[NPL], vp[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      vm[i] = 0.0;
      vp[i] = 0.0;
#pragma unroll
      for (int j = 1; j < kHist; ++j) {
        if (j == q) vm[i] = D[j][i];
        if (j == q + 2) vp[i] = D[j][i];
      }
    }
    const double err_m = q > 1 ? W.wrms(vm, w) / q : 0.0;
    const double err_p = q < sp.max_order ? W.wrms(vp, w) / (q + 2) : 0.0;
    double rho;
    q = choose_order(q, sp.max_order, err, err_m, err_p, &rho);
    rescale_hist(D, q, rho);
    h *= rho;
    n_equal = 0;
  }

  if (status == ST_OK) {
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int tt = lane + G * i;
      if (tt < N) yrow[m.perm[tt]] = D[0][i];
    }
  }
  cs.order = q;
  return status;
}

// Rate constants, then the integration; a cell whose integration fails (too many steps,
// step below the minimum, repeated error-test or Newton failures) is integrated again from
// its input: with full Newton, then with full Newton and a tighter absolute tolerance.
template <int NPL, int G, bool kPar>
__device__ __forceinline__ void solve_one_cell(const DevMech& m, const DevEnv& env, double* state, int cell,
                               const SolveParams& sp, int* status_out, camp_cell_stats* stats_out,
                               const WaveCell<NPL, G, kPar>& W) {
  const int lane = W.lane;
  camp_cell_stats cs = {0, 0, 0, 0, 0, 0, 0, 0};
  const double Tk = env.T[cell], Pp = env.P[cell];
  const double cz = env.cos_sza ? env.cos_sza[cell] : 1.0;
  const double* rad = env.radius ? env.radius + (size_t)cell * m.n_inst : nullptr;
  const double* mas = env.mass ? env.mass + (size_t)cell * m.n_inst : nullptr;
  const double* ovr = env.override_ ? env.override_ + (size_t)cell * m.n_ext : nullptr;
  int bad = 0;
  for (int k = lane; k < m.R; k += G) {
    const double v = rate_constant(m, k, Tk, Pp, cz, rad, mas, ovr);
    W.kc[k] = v;
    if (!isfinite(v)) bad = 1;
  }
  __threadfence_block();   // rate constants (LDS or global scratch) visible to all lanes
  double* yrow = state + (size_t)cell * m.N;
  int status = ST_OK;
  for (int attempt = sp.full_newton ? 1 : 0; attempt < kAttempts; ++attempt) {
    SolveParams spa = sp;
    if (attempt == 2) spa.atol *= kRetryAtolFactor;
    status = integrate(m, yrow, spa, bad, attempt > 0, cs, W);
    if (status < ST_MAX_STEPS || status > ST_NEWTON_FAIL) break;
  }
  if (lane == 0) {
    status_out[cell] = status;
    if (stats_out) stats_out[cell] = cs;
  }
  W.sync();
}

// Launch modes of the wavefront engine (table staging and where rate constants live):
//   0  tables read from global memory, rate constants in LDS
//   1  core index tables staged in LDS
//   2  whole table block staged in LDS
//   3  tables from global memory and rate constants in a global per-wavefront scratch
//      (persistent launches only), for mechanisms whose per-cell LDS is the occupancy limit
//   4  core index tables staged in LDS and rate constants in the global scratch
//   5  as 3, for mechanisms with Parameters (rates divided by a state-dependent amount):
//      the only mode such mechanisms run in, so the kernels of the other modes carry no
//      parameter code
// In modes 3 and 4, cells of at most two species per lane (up to 128 state variables on one
// wavefront, up to 256 on two) run a kernel built for three wavefronts per SIMD (at most 168
// registers): up to 12 one-wavefront cells per workgroup, or six two-wavefront cells per CU.
constexpr int kParamMode = 5;
// The table staging of a launch mode (mode 5 stages as mode 3).
__host__ __device__ constexpr int table_mode(int mode) { return mode == kParamMode ? 3 : mode; }
__host__ __device__ constexpr bool kc_global(int mode) { return table_mode(mode) >= 3; }

// LDS doubles of one cell: M [Z], y [N], x [N], partials/rates, 8 doubles of group
// scratch, and the rate constants unless they live in global scratch (modes 3, 4).
__host__ __device__ inline size_t cell_doubles(const DevMech& m, int mode) {
  const int np = m.n_part > m.R ? m.n_part : m.R;
  return (size_t)m.Z + 2 * (size_t)m.N + np + 8 + (kc_global(mode) ? 0 : m.R);
}

// Bytes of the table block staged in LDS in launch mode `mode`.
__host__ __device__ inline int staged_bytes(const StageView& v, int mode) {
  mode = table_mode(mode);
  return mode == 2 ? v.bytes : (mode == 1 || mode == 4) ? v.core_bytes : 0;
}

// Copies the staged part of the table block into LDS (16-byte units).
template <int kStage>
__device__ __forceinline__ Tabs stage_tables(const StageView& v, double* lds) {
  const char* g = reinterpret_cast<const char*>(v.base);
  if (table_mode(kStage) == 0 || table_mode(kStage) == 3) return Tabs{g, g, v};
  const uint4* src = reinterpret_cast<const uint4*>(v.base);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  const int n16 = staged_bytes(v, kStage) / 16;
  for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  const char* l = reinterpret_cast<const char*>(lds);
  return Tabs{l, table_mode(kStage) == 2 ? l : g, v};
}


// One wavefront per cell (G = 64): up to 3 species per lane the kernel fits 256 VGPRs (two
// wavefronts per SIMD, workgroups of up to 8 cells); larger states get 512 VGPRs
// (workgroups of up to 4 cells). In modes 3 and 4, up to 2 species per lane the kernel is
// built for 168 registers (three wavefronts per SIMD, workgroups of up to 12 cells).
// One workgroup per cell (G = 128 or 256): at most 256 VGPRs (two wavefronts per SIMD) up
// to 3 species per lane, 512 beyond; with G = 128 in modes 3 and 4, up to 2 species per
// lane, 168 registers (three wavefronts per SIMD, six cells per CU).
template <int NPL, int kMode, int G>
constexpr bool occ3() { return (G == kWave || G == 2 * kWave) && NPL <= 2 && kc_global(kMode); }
template <int NPL, int kMode, int G>
constexpr int max_threads() {
  return G > kWave ? G : kWave * (occ3<NPL, kMode, G>() ? 12 : NPL <= 3 ? 8 : 4);
}
template <int NPL, int kMode, int G>
constexpr int min_waves_per_simd() {
  return occ3<NPL, kMode, G>() ? 3 : G > kWave ? (NPL <= 3 ? 2 : 1) : 1;
}

// G = 64: blockDim.x = 64 * W, W wavefronts, one cell each; G > 64: blockDim.x = G, one
// cell per workgroup. queue != nullptr: persistent grid pulling cells from the counter;
// else cell = blockIdx.x * W + wavefront. Modes 3 and 4 keep the rate constants at
// kc_glob + (blockIdx.x * W + wavefront) * R and need the queue.
template <int NPL, int kStage, int G>
__global__ __launch_bounds__((max_threads<NPL, kStage, G>()),
                             (min_waves_per_simd<NPL, kStage, G>())) void bdf_wave_kernel(
    DevMech m, DevEnv env, double* state, int n_cells, SolveParams sp, int* status,
    camp_cell_stats* stats, int* queue, double* kc_glob) {
  extern __shared__ double lds[];
  const StageView& view = m.sv[G / 128];
  const Tabs tab = stage_tables<kStage>(view, lds);
  const int W = G == kWave ? blockDim.x / kWave : 1;
  const int wid = G == kWave ? threadIdx.x / kWave : 0;
  const int lane = threadIdx.x % G;
  double* base = lds + staged_bytes(view, kStage) / 8 + wid * cell_doubles(m, kStage);
  const int np = m.n_part > m.R ? m.n_part : m.R;
  double* yl = base + m.Z;
  double* xl = yl + m.N;
  double* P = xl + m.N;
  double* red = P + np;
  double* kc = kc_global(kStage) ? kc_glob + (size_t)(blockIdx.x * W + wid) * m.R : red + 8;
  const WaveCell<NPL, G, kStage == kParamMode> Wc{m, tab, base, yl, xl, P, kc, red, lane};
  if (!queue) {
    const int cell = blockIdx.x * W + wid;
    if (cell < n_cells) solve_one_cell(m, env, state, cell, sp, status, stats, Wc);
    return;
  }
  while (true) {
    int cell = 0;
    if constexpr (G == kWave) {
      if (lane == 0) cell = atomicAdd(queue, 1);
      cell = uniform(cell);
    } else {
      int* slot = reinterpret_cast<int*>(red + 4);
      if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
      __syncthreads();
      cell = *slot;
      __syncthreads();
    }
    if (cell >= n_cells) break;
    if (sp.order && *sp.order_bad == 0) cell = sp.order[cell];
    solve_one_cell(m, env, state, cell, sp, status, stats, Wc);
  }
}

template <int NPL, int kStage, int G>
hipError_t launch_wave_npl(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                           const SolveParams& sp, int* status, camp_cell_stats* stats, int* queue,
                           double* kc_glob, int grid, int waves, size_t lds, bool attr_only,
                           hipStream_t stream) {
  hipError_t e = hipFuncSetAttribute((const void*)bdf_wave_kernel<NPL, kStage, G>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess || attr_only) return e;
  const int threads = G == kWave ? kWave * waves : G;
  hipLaunchKernelGGL((bdf_wave_kernel<NPL, kStage, G>), dim3(grid), dim3(threads), lds, stream,
                     m, env, state, n_cells, sp, status, stats, queue, kc_glob);
  return hipGetLastError();
}

template <int NPL, int G>
hipError_t run_wave(const WaveParams& p, int stage) {
  switch (stage) {
    case 0: return launch_wave_npl<NPL, 0, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    case 1: return launch_wave_npl<NPL, 1, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    case 2: return launch_wave_npl<NPL, 2, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    case 3: return launch_wave_npl<NPL, 3, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    case 4: return launch_wave_npl<NPL, 4, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    case kParamMode: return launch_wave_npl<NPL, kParamMode, G>(p.m, p.env, p.state, p.n_cells, p.sp, p.status, p.stats, p.queue, p.kc_glob, p.grid, p.waves, p.lds, p.attr_only, p.stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Instantiations of the fused kernel are spread over several translation units (compiled
// in parallel), each covering a range of species per lane for one group size.
hipError_t wave_run_64_a(const WaveParams& p, int npl, int stage);    // NPL 1..3
hipError_t wave_run_64_b(const WaveParams& p, int npl, int stage);    // NPL 4..6
hipError_t wave_run_64_c(const WaveParams& p, int npl, int stage);    // NPL 7..9
hipError_t wave_run_128(const WaveParams& p, int npl, int stage);     // NPL 1..5
hipError_t wave_run_256(const WaveParams& p, int npl, int stage);     // NPL 1..3

}  // namespace camp
