// Fused persistent engine, one wavefront per cell.
//
// Every cell's whole integration over the host step (rate constants, then BDF steps with
// forcing, Newton matrix, sparse LU and triangular solves, error test and step/order
// control) runs inside one kernel. A wavefront owns one cell at a time: its Newton matrix,
// state, right-hand side, rates and partial derivatives live in LDS, and its BDF history
// lives in registers with species t held by lane t % 64. Sparse work is spread over the
// 64 lanes by the level-scheduled tables built on the host: every task of one dependency
// level runs in parallel, levels are separated by a wavefront-scoped barrier. Control
// decisions use wavefront reductions, so they are uniform and need no masking.
//
// A workgroup holds several wavefronts (cells) that share one LDS copy of the
// latency-critical index tables (reactants, CSR pattern with level-ordered solve rows,
// Crout LU tasks and pairs), staged once per workgroup. When a cell is done the wavefront
// takes the next one from a device-side queue (persistent grid) or from the grid index.
//
// Forcing and Jacobian (paper Sect. 2.4.2): f_i = sum_k S_ik r_k and
// J_ij = sum_k S_ik dr_k/dy_j, with r_k = k_k prod y over reactant occurrences.
#include "bdf_common.hpp"
#include "camp.h"

namespace camp {

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

// One update of a term loop: add `v` to entry `dst`.
struct TermUpdate {
  int dst;
  double v;
};

// Runs the terms i = lo + lane, lo + lane + 64, ... < hi of a term list in groups of kU:
// the loads of a group (gather) are all issued before any of its updates (scatter), so
// their latencies overlap. Only valid where no term of the list reads what another writes.
template <int kU, class Gather, class Scatter>
__device__ __forceinline__ void for_terms(int lo, int hi, int lane, Gather gather, Scatter scatter) {
  int i = lo + lane;
  for (; i + (kU - 1) * kWave < hi; i += kU * kWave) {
    TermUpdate it[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) it[u] = gather(i + u * kWave);
#pragma unroll
    for (int u = 0; u < kU; ++u) scatter(it[u]);
  }
  for (; i < hi; i += kWave) scatter(gather(i));
}

constexpr int kTermBatch = 4;

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

// Accessors of the compact table block: the core tables through `b`, the forcing-term and
// Jacobian-contribution extension through `e`; each base is LDS (staged) or global memory.
struct Tabs {
  const char* b;
  const char* e;
  const DevMech& m;
  __device__ uint32_t ft(int i) const { return reinterpret_cast<const uint32_t*>(e + m.so_ft)[i]; }
  __device__ double ft_coef(int i) const { return reinterpret_cast<const double*>(e + m.so_ft_coef)[i]; }
  __device__ uint32_t jt(int i) const { return reinterpret_cast<const uint32_t*>(e + m.so_jt)[i]; }
  __device__ double jt_coef(int i) const { return reinterpret_cast<const double*>(e + m.so_jt_coef)[i]; }
  __device__ uint32_t rx(int k) const { return reinterpret_cast<const uint32_t*>(b + m.so_rx)[k]; }
  __device__ int dg(int t) const { return reinterpret_cast<const uint16_t*>(b + m.so_diag)[t]; }
  __device__ uint2 sf(int i) const { return reinterpret_cast<const uint2*>(b + m.so_sf)[i]; }
  __device__ int sf_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + m.so_sf_lp)[l]; }
  __device__ uint2 sb(int i) const { return reinterpret_cast<const uint2*>(b + m.so_sb)[i]; }
  __device__ int sb_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + m.so_sb_lp)[l]; }
  __device__ uint2 lt(int i) const { return reinterpret_cast<const uint2*>(b + m.so_lt)[i]; }
  __device__ int lt_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + m.so_lt_lp)[l]; }
  __device__ uint32_t lf(int i) const { return reinterpret_cast<const uint32_t*>(b + m.so_lf)[i]; }
  __device__ int lf_lp(int l) const { return (int)reinterpret_cast<const uint32_t*>(b + m.so_lf_lp)[l]; }
  __device__ uint32_t us(int i) const { return reinterpret_cast<const uint32_t*>(b + m.so_us)[i]; }
};

template <int NPL>
struct WaveCell {
  // Terms per lane issued together in the LU and sweep levels: levels of large mechanisms
  // hold several terms per lane, small ones rarely more than one.
  static constexpr int kLevelBatch = NPL >= 4 ? 4 : 1;
  const DevMech& m;
  Tabs tb;
  double* M;
  double* yl;
  double* xl;
  double* P;
  double* kc;
  int lane;

  __device__ double wrms(const double (&v)[NPL], const double (&w)[NPL]) const {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NPL; ++i)
      if (lane + kWave * i < m.N) {
        double a = v[i] * w[i];
        s += a * a;
      }
    return sqrt(wave_sum(s) / m.N);
  }

  // P[k] = r_k from yl; then f for owned species, accumulated term by term (one term per
  // lane) in xl, which no caller holds live across this call. yl must be visible to all
  // lanes.
  __device__ void forcing(double (&f)[NPL]) const {
    for (int k = lane; k < m.R; k += kWave) {
      const uint32_t v = tb.rx(k);
      const int a = v & 0x3FF, b = (v >> 10) & 0x3FF, c = (v >> 20) & 0x3FF;
      double r = kc[k];
      if (a != 0x3FF) r *= yl[a];
      if (b != 0x3FF) r *= yl[b];
      if (c != 0x3FF) r *= yl[c];
      P[k] = r;
    }
    for (int t = lane; t < m.N; t += kWave) xl[t] = 0.0;
    wave_sync();
    for_terms<kTermBatch>(
        0, m.n_ft, lane,
        [&](int i) {
          const uint32_t e = tb.ft(i);
          return TermUpdate{(int)(e & 0xFFFF), tb.ft_coef(i) * P[e >> 16]};
        },
        [&](const TermUpdate& u) { lds_add(&xl[u.dst], u.v); });
    wave_sync();
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int t = lane + kWave * i;
      f[i] = t < m.N ? xl[t] : 0.0;
    }
    wave_sync();
  }

  // M = I - c J(yl) in the filled pattern (fill slots 0 off the diagonal), accumulated
  // contribution by contribution (one per lane).
  __device__ void newton_matrix(double c) const {
    for (int k = lane; k < m.R; k += kWave) {
      const uint32_t v = tb.rx(k);
      const int a = v & 0x3FF, b = (v >> 10) & 0x3FF, cc = (v >> 20) & 0x3FF;
      const double kk = kc[k];
      const int base = m.rx_pofs[k];
      const double ya = a != 0x3FF ? yl[a] : 1.0, yb = b != 0x3FF ? yl[b] : 1.0,
                   yc = cc != 0x3FF ? yl[cc] : 1.0;
      if (a != 0x3FF) P[base] = kk * yb * yc;
      if (b != 0x3FF) P[base + 1] = kk * ya * yc;
      if (cc != 0x3FF) P[base + 2] = kk * ya * yb;
    }
    for (int s = lane; s < m.Z; s += kWave) M[s] = 0.0;
    wave_sync();
    const double mc = -c;
    for_terms<kTermBatch>(
        0, m.n_jt, lane,
        [&](int i) {
          const uint32_t e = tb.jt(i);
          return TermUpdate{(int)(e & 0xFFFF), mc * tb.jt_coef(i) * P[e >> 16]};
        },
        [&](const TermUpdate& u) { lds_add(&M[u.dst], u.v); });
    wave_sync();
    for (int t = lane; t < m.N; t += kWave) M[tb.dg(t)] += 1.0;
    wave_sync();
  }

  // In-place Crout LU of M, one dependency level at a time: the level's product terms in
  // parallel (one per lane), then its finalize entries (L entries times the reciprocal
  // pivot, pivots inverted). Leaves the unit-diagonal factors: L strictly below the
  // diagonal, reciprocal pivots on it, and U / diag(U) strictly above. Returns 0 if a
  // pivot is not a finite nonzero.
  __device__ int lu() const {
    const int L = m.lu_levels;
    const LevelPtrs tp = load_levels(L, [&](int l) { return tb.lt_lp(l); });
    const LevelPtrs fp = load_levels(L + 1, [&](int l) { return tb.lf_lp(l); });
    int fhi = level_ptr(fp, 1, [&](int l) { return tb.lf_lp(l); });
    for (int i = lane; i < fhi; i += kWave) {
      const int d = tb.lf(i) & 0xFFFF;
      M[d] = 1.0 / M[d];
    }
    wave_sync();
    int tlo = 0;
    for (int l = 0; l < L; ++l) {
      const int thi = level_ptr(tp, l + 1, [&](int k) { return tb.lt_lp(k); });
      for_terms<kLevelBatch>(
          tlo, thi, lane,
          [&](int i) {
            const uint2 e = tb.lt(i);
            return TermUpdate{(int)(e.x & 0xFFFF), M[e.x >> 16] * M[e.y]};
          },
          [&](const TermUpdate& u) { lds_add(&M[u.dst], -u.v); });
      tlo = thi;
      wave_sync();
      const int flo = fhi;
      fhi = level_ptr(fp, l + 2, [&](int k) { return tb.lf_lp(k); });
      if (flo == fhi) continue;
      for (int i = flo + lane; i < fhi; i += kWave) {
        const uint32_t e = tb.lf(i);
        const int dst = e & 0xFFFF, pv = e >> 16;
        M[dst] = pv == 0xFFFF ? 1.0 / M[dst] : M[dst] * M[pv];
      }
      wave_sync();
    }
    for (int i = lane; i < m.n_us; i += kWave) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] *= M[e >> 16];
    }
    int bad = 0;
    for (int t = lane; t < m.N; t += kWave) {
      const double r = M[tb.dg(t)];
      if (!(fabs(r) > 0.0) || !isfinite(r)) bad = 1;
    }
    wave_sync();
    return !wave_or(bad);
  }

  __device__ int newton_matrix_lu(double c) const {
    newton_matrix(c);
    return lu();
  }

  // Conversions between the factor form lu() leaves and the conventional one (unit L
  // strictly below the diagonal, U on and above it).
  __device__ void factors_to_conventional() const {
    for (int i = lane; i < m.n_us; i += kWave) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] /= M[e >> 16];
    }
    wave_sync();
    for (int t = lane; t < m.N; t += kWave) M[tb.dg(t)] = 1.0 / M[tb.dg(t)];
    wave_sync();
  }
  __device__ void factors_from_conventional() const {
    for (int t = lane; t < m.N; t += kWave) M[tb.dg(t)] = 1.0 / M[tb.dg(t)];
    wave_sync();
    for (int i = lane; i < m.n_us; i += kWave) {
      const uint32_t e = tb.us(i);
      M[e & 0xFFFF] *= M[e >> 16];
    }
    wave_sync();
  }

  // One triangular sweep over the unit-diagonal factor: x[dst] -= M[slot] * x[src] for
  // the terms of each level, one term per lane.
  template <bool kForward>
  __device__ void sweep() const {
    const int nlev = kForward ? m.n_sf_lev : m.n_sb_lev;
    auto lp = [&](int l) { return kForward ? tb.sf_lp(l) : tb.sb_lp(l); };
    const LevelPtrs p = load_levels(nlev, lp);
    int lo = 0;
    for (int l = 0; l < nlev; ++l) {
      const int hi = level_ptr(p, l + 1, lp);
      for_terms<kLevelBatch>(
          lo, hi, lane,
          [&](int i) {
            const uint2 e = kForward ? tb.sf(i) : tb.sb(i);
            return TermUpdate{(int)(e.x & 0xFFFF), M[e.y] * xl[e.x >> 16]};
          },
          [&](const TermUpdate& u) { lds_add(&xl[u.dst], -u.v); });
      lo = hi;
      wave_sync();
    }
  }

  // xl <- (LU)^-1 xl from the factors lu() leaves: forward sweep, diagonal scaling,
  // backward sweep.
  __device__ void solve() const {
    sweep<true>();
    for (int t = lane; t < m.N; t += kWave) xl[t] *= M[tb.dg(t)];
    wave_sync();
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
template <int NPL>
__device__ __forceinline__ int integrate(const DevMech& m, double* yrow, const SolveParams& sp, int bad, int full,
                         camp_cell_stats& cs, const WaveCell<NPL>& W) {
  const int lane = W.lane;
  const int N = m.N;
  int status = ST_OK;

  // ---- initial state ----
  double D[kHist][NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int t = lane + kWave * i;
    const double v = t < N ? yrow[m.perm[t]] : 0.0;
    if (t < N) {
      W.yl[t] = v;
      if (!isfinite(v)) bad = 1;
    }
    D[0][i] = v;
#pragma unroll
    for (int j = 1; j < kHist; ++j) D[j][i] = 0.0;
  }
  wave_sync();
  if (wave_or(bad)) status = ST_NONFINITE;

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
    if (wave_or(nf)) status = ST_NONFINITE;
  }
  double h = 0.0;
  if (status == ST_OK) {
    // starting step
    const double d0 = W.wrms(D[0], w), d1 = W.wrms(f0, w);
    const double h0 = starting_step_h0(d0, d1, span);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int t = lane + kWave * i;
      if (t < N) W.yl[t] = D[0][i] + h0 * f0[i];
    }
    wave_sync();
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
      if (lane + kWave * i < N && !isfinite(w[i])) nfw = 1;
    }
    if (wave_or(nfw)) {
      status = ST_NONFINITE;
      break;
    }
    int consec_err = 0, consec_nf = 0, force_lu = 0;
    bool accepted = false;
    while (true) {
      if (++attempts > sp.max_steps) { status = ST_MAX_STEPS; break; }
      if (h < sp.h_min) { status = ST_H_MIN; break; }
      const double gq = bdf_gamma(q);
      const double c = h / gq;
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
        psi[i] = ps / gq;
        yv[i] = s;
        d[i] = 0.0;
        const int tt = lane + kWave * i;
        if (tt < N) W.yl[tt] = s;
      }
      wave_sync();
      int fresh = 0, lu_ok = 1;
      if (force_lu || !lu_valid || fabs(c / c_lu - 1.0) > kLuGammaDrift || lu_age >= kLuMaxAge) {
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
              const int tt = lane + kWave * i;
              if (tt < N) W.yl[tt] = yv[i];
            }
            wave_sync();
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
            const int tt = lane + kWave * i;
            if (tt < N) {
              if (!isfinite(f[i])) nf = 1;
              W.xl[tt] = c * f[i] - psi[i] - d[i];
            }
          }
          if (wave_or(nf)) { nonfin = 1; break; }
          wave_sync();
          W.solve();
          double dl[NPL];
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            const int tt = lane + kWave * i;
            dl[i] = tt < N ? W.xl[tt] * scale : 0.0;
          }
          wave_sync();
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
        if (lane + kWave * i < N && yv[i] * w[i] < -1.0) neg = 1;
      if (wave_or(neg)) {
        cs.rejected++;
        rescale_hist(D, q, kConstraintFactor);
        h *= kConstraintFactor;
        n_equal = 0;
        continue;
      }
      double dq1[NPL];
#pragma unroll
      for (int i = 0; i < NPL; ++i) dq1[i] = d[i] / (q + 1);
      err = W.wrms(dq1, w);
      if (err > 1.0) {
        cs.rejected++;
        if (++consec_err >= kMaxConsecFail) { status = ST_ERR_FAIL; break; }
        n_equal = 0;
        if (consec_err >= kErrRestart) {
          // restart at order 1 from y_n with a much smaller step: D[1] = h f(y_n)
#pragma unroll
          for (int i = 0; i < NPL; ++i) {
            const int tt = lane + kWave * i;
            if (tt < N) W.yl[tt] = D[0][i];
          }
          wave_sync();
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
      const int tt = lane + kWave * i;
      if (tt < N) yrow[m.perm[tt]] = D[0][i];
    }
  }
  cs.order = q;
  return status;
}

// Rate constants, then the integration; a cell whose integration fails (too many steps,
// step below the minimum, repeated error-test or Newton failures) is integrated again from
// its input: with full Newton, then with full Newton and a tighter absolute tolerance.
template <int NPL>
__device__ void solve_one_cell(const DevMech& m, const DevEnv& env, double* state, int cell,
                               const SolveParams& sp, int* status_out, camp_cell_stats* stats_out,
                               const WaveCell<NPL>& W) {
  const int lane = W.lane;
  camp_cell_stats cs = {0, 0, 0, 0, 0, 0, 0, 0};
  const double Tk = env.T[cell], Pp = env.P[cell];
  const double cz = env.cos_sza ? env.cos_sza[cell] : 1.0;
  const double* rad = env.radius ? env.radius + (size_t)cell * m.n_inst : nullptr;
  const double* mas = env.mass ? env.mass + (size_t)cell * m.n_inst : nullptr;
  const double* ovr = env.override_ ? env.override_ + (size_t)cell * m.n_ext : nullptr;
  int bad = 0;
  for (int k = lane; k < m.R; k += kWave) {
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
    status = integrate<NPL>(m, yrow, spa, bad, attempt > 0, cs, W);
    if (status < ST_MAX_STEPS || status > ST_NEWTON_FAIL) break;
  }
  if (lane == 0) {
    status_out[cell] = status;
    if (stats_out) stats_out[cell] = cs;
  }
  wave_sync();
}

// Launch modes of the wavefront engine (table staging and where rate constants live):
//   0  tables read from global memory, rate constants in LDS
//   1  core index tables staged in LDS
//   2  whole table block staged in LDS
//   3  tables from global memory and rate constants in a global per-wavefront scratch
//      (persistent launches only), for mechanisms whose per-cell LDS is the occupancy limit
//   4  core index tables staged in LDS and rate constants in the global scratch
// In modes 3 and 4 a mechanism of at most 128 state variables runs a kernel built for
// three wavefronts per SIMD (at most 168 registers), with up to 12 cells per workgroup.
__host__ __device__ constexpr bool kc_global(int mode) { return mode >= 3; }

// LDS doubles of one cell: M, y, x, partials/rates, and the rate constants unless mode 3.
__host__ __device__ inline size_t cell_doubles(const DevMech& m, int mode) {
  const int np = m.n_part > m.R ? m.n_part : m.R;
  return (size_t)m.Z + 2 * (size_t)m.N + np + (kc_global(mode) ? 0 : m.R);
}

// Bytes of the table block staged in LDS in launch mode `mode`.
__host__ __device__ inline int staged_bytes(const DevMech& m, int mode) {
  return mode == 2 ? m.stage_bytes : (mode == 1 || mode == 4) ? m.stage_core_bytes : 0;
}

// Copies the staged part of the table block into LDS (16-byte units).
template <int kStage>
__device__ __forceinline__ Tabs stage_tables(const DevMech& m, double* lds) {
  const char* g = reinterpret_cast<const char*>(m.stage);
  if (kStage == 0 || kStage == 3) return Tabs{g, g, m};
  const uint4* src = reinterpret_cast<const uint4*>(m.stage);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  const int n16 = staged_bytes(m, kStage) / 16;
  for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  const char* l = reinterpret_cast<const char*>(lds);
  return Tabs{l, kStage == 2 ? l : g, m};
}

}  // namespace

// Up to 3 species per lane the kernel fits 256 VGPRs (two wavefronts per SIMD, workgroups
// of up to 8 wavefronts); larger states get 512 VGPRs (workgroups of up to 4 wavefronts).
// In modes 3 and 4, up to 2 species per lane the kernel is built for 168 registers (three
// wavefronts per SIMD, workgroups of up to 12 wavefronts).
template <int NPL, int kMode>
constexpr bool occ3() { return NPL <= 2 && kc_global(kMode); }
template <int NPL, int kMode>
constexpr int max_waves_per_wg() { return occ3<NPL, kMode>() ? 12 : NPL <= 3 ? 8 : 4; }
template <int NPL, int kMode>
constexpr int min_waves_per_simd() { return occ3<NPL, kMode>() ? 3 : 1; }
int wave_max_waves(int n_state, int mode) {
  const int npl = (n_state + kWave - 1) / kWave;
  return (npl <= 2 && kc_global(mode)) ? 12 : npl <= 3 ? 8 : 4;
}

// blockDim.x = 64 * W: W wavefronts, one cell each. queue != nullptr: persistent grid
// pulling cells from the counter; else cell = blockIdx.x * W + wavefront. Mode 3 keeps the
// rate constants at kc_glob + (blockIdx.x * W + wavefront) * R and needs the queue.
template <int NPL, int kStage>
__global__ __launch_bounds__((kWave * max_waves_per_wg<NPL, kStage>()),
                             (min_waves_per_simd<NPL, kStage>())) void bdf_wave_kernel(
    DevMech m, DevEnv env, double* state, int n_cells, SolveParams sp, int* status,
    camp_cell_stats* stats, int* queue, double* kc_glob) {
  extern __shared__ double lds[];
  const Tabs tab = stage_tables<kStage>(m, lds);
  const int W = blockDim.x / kWave, wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* base = lds + staged_bytes(m, kStage) / 8 + wid * cell_doubles(m, kStage);
  const int np = m.n_part > m.R ? m.n_part : m.R;
  double* kc = kc_global(kStage) ? kc_glob + (size_t)(blockIdx.x * W + wid) * m.R
                                       : base + m.Z + 2 * m.N + np;
  const WaveCell<NPL> Wc{m, tab, base, base + m.Z, base + m.Z + m.N, base + m.Z + 2 * m.N, kc, lane};
  if (!queue) {
    const int cell = blockIdx.x * W + wid;
    if (cell < n_cells) solve_one_cell<NPL>(m, env, state, cell, sp, status, stats, Wc);
    return;
  }
  while (true) {
    int cell = 0;
    if (lane == 0) cell = atomicAdd(queue, 1);
    cell = uniform(cell);
    if (cell >= n_cells) break;
    solve_one_cell<NPL>(m, env, state, cell, sp, status, stats, Wc);
  }
}

size_t wave_cell_bytes(const DevMech& m) { return sizeof(double) * cell_doubles(m, 0); }

size_t wave_lds_bytes(const DevMech& m) { return wave_cell_bytes(m); }

// LDS bytes of a workgroup of `waves` cells in launch mode `mode` (0..3).
size_t wave_wg_lds_bytes(const DevMech& m, int waves, int mode) {
  return (size_t)staged_bytes(m, mode) + (size_t)waves * sizeof(double) * cell_doubles(m, mode);
}

template <int NPL, int kStage>
hipError_t launch_wave_npl(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                           const SolveParams& sp, int* status, camp_cell_stats* stats, int* queue,
                           double* kc_glob, int grid, int waves, size_t lds, hipStream_t stream) {
  hipError_t e = hipFuncSetAttribute((const void*)bdf_wave_kernel<NPL, kStage>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((bdf_wave_kernel<NPL, kStage>), dim3(grid), dim3(kWave * waves), lds, stream,
                     m, env, state, n_cells, sp, status, stats, queue, kc_glob);
  return hipGetLastError();
}

template <int NPL>
hipError_t launch_wave_stage(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                             const SolveParams& sp, int* status, camp_cell_stats* stats,
                             int* queue, double* kc_glob, int grid, int waves, int stage,
                             size_t lds, hipStream_t stream) {
  switch (stage) {
    case 0: return launch_wave_npl<NPL, 0>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, lds, stream);
    case 1: return launch_wave_npl<NPL, 1>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, lds, stream);
    case 2: return launch_wave_npl<NPL, 2>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, lds, stream);
    case 3: return launch_wave_npl<NPL, 3>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, lds, stream);
    case 4: return launch_wave_npl<NPL, 4>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bdf_wave(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                           const SolveParams& sp, int* status, camp_cell_stats* stats, int* queue,
                           double* kc_glob, int grid, int waves, int stage, hipStream_t stream) {
  const size_t lds = wave_wg_lds_bytes(m, waves, stage);
  const int npl = (m.N + kWave - 1) / kWave;
  if (stage < 0 || stage > 4 || !m.stage) return hipErrorInvalidValue;
  if (waves < 1 || waves > wave_max_waves(m.N, stage)) return hipErrorInvalidValue;
  if (kc_global(stage) && (!queue || !kc_glob)) return hipErrorInvalidValue;
  switch (npl) {
    case 1: return launch_wave_stage<1>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 2: return launch_wave_stage<2>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 3: return launch_wave_stage<3>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 4: return launch_wave_stage<4>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 5: return launch_wave_stage<5>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 6: return launch_wave_stage<6>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 7: return launch_wave_stage<7>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 8: return launch_wave_stage<8>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    case 9: return launch_wave_stage<9>(m, env, state, n_cells, sp, status, stats, queue, kc_glob, grid, waves, stage, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- single-step kernels
// One wavefront per cell; the same device code as the fused engine (tables read from
// global memory), on row-major [cells][...] arrays in user state order.

template <int NPL>
__global__ __launch_bounds__(kWave) void wave_step_kernel(DevMech m, int op, int n_cells,
                                                          const double* kin, const double* yin,
                                                          double* out, double gamma) {
  extern __shared__ double lds[];
  const int np = m.n_part > m.R ? m.n_part : m.R;
  const char* g = reinterpret_cast<const char*>(m.stage);
  const WaveCell<NPL> W{m, Tabs{g, g, m}, lds, lds + m.Z,
                        lds + m.Z + m.N, lds + m.Z + 2 * m.N, lds + m.Z + 2 * m.N + np,
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
    hipError_t e = hipFuncSetAttribute((const void*)wave_step_kernel<K>,                       \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    if (e != hipSuccess) return e;                                                             \
    hipLaunchKernelGGL(wave_step_kernel<K>, dim3(n_cells), dim3(kWave), lds, stream, m, op,     \
                       n_cells, kin, yin, out, gamma);                                         \
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
