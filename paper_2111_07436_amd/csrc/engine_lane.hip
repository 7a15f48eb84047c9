// Lane-per-cell engines: one lane integrates one cell; all of a cell's vectors and its
// Newton matrix live in cell-interleaved slabs in HBM (element x of cell c at
// ((c/64)*X + x)*64 + c%64), so each table-driven access of a wavefront is one coalesced
// 512-byte line, and the mechanism tables are read with wavefront-uniform (scalar) loads.
//
// The BDF step is split into phase functions (init, predict, Newton matrix + LU, one Newton
// iteration, finish). The plain engine launches one kernel per phase per step attempt
// with per-cell masks; the fused engine runs the same phases in one persistent kernel
// where each lane loops over its own cells.
#include "bdf_common.hpp"
#include "camp.h"

namespace camp {

// Per-slot control state (SoA, [slots]).
struct LaneState {
  double *t, *h, *c_lu, *crate, *err, *dn_old;
  int *q, *n_equal, *attempts, *lu_valid, *lu_age, *consec_err, *consec_nf, *force_lu;
  int *phase, *it, *fresh, *lu_ok, *cell, *full;
  camp_cell_stats* st;
};

enum LanePhase : int { PH_IDLE = 0, PH_NEWTON = 1, PH_FINISH = 2, PH_DONE = 3 };

struct LaneSlabs {
  double *kc, *P, *M, *y, *x, *D, *d, *psi, *w, *f;
};

struct LaneCtx {
  DevMech m;
  DevEnv env;
  SolveParams sp;
  LaneSlabs s;
  LaneState st;
  double* state;     // user [cells][N]
  int* status;       // user [cells]
  camp_cell_stats* stats_out;
  int n_cells;
};

namespace {

struct Lane {
  const LaneCtx& C;
  int slot;
  size_t bR, bP, bZ, bN, bD;
  __device__ Lane(const LaneCtx& c, int s) : C(c), slot(s) {
    const int np = c.m.n_part > c.m.R ? c.m.n_part : c.m.R;
    bR = slab(s, c.m.R);
    bP = slab(s, np);
    bZ = slab(s, c.m.Z);
    bN = slab(s, c.m.N);
    bD = slab(s, kHist * c.m.N);
  }
  __device__ double& kc(int k) const { return C.s.kc[bR + (size_t)k * kWave]; }
  __device__ double& P(int k) const { return C.s.P[bP + (size_t)k * kWave]; }
  __device__ double& M(int z) const { return C.s.M[bZ + (size_t)z * kWave]; }
  __device__ double& y(int i) const { return C.s.y[bN + (size_t)i * kWave]; }
  __device__ double& x(int i) const { return C.s.x[bN + (size_t)i * kWave]; }
  __device__ double& d(int i) const { return C.s.d[bN + (size_t)i * kWave]; }
  __device__ double& psi(int i) const { return C.s.psi[bN + (size_t)i * kWave]; }
  __device__ double& w(int i) const { return C.s.w[bN + (size_t)i * kWave]; }
  __device__ double& f(int i) const { return C.s.f[bN + (size_t)i * kWave]; }
  __device__ double& D(int j, int i) const { return C.s.D[bD + ((size_t)j * C.m.N + i) * kWave]; }

  // f(y) into f(); returns 0 if non-finite
  __device__ int forcing() const {
    const DevMech& m = C.m;
    for (int k = 0; k < m.R; ++k) {
      const int a = m.rx_react[3 * k], b = m.rx_react[3 * k + 1], c = m.rx_react[3 * k + 2];
      double r = kc(k);
      if (a >= 0) r *= y(a);
      if (b >= 0) r *= y(b);
      if (c >= 0) r *= y(c);
      P(k) = r;
    }
    for (int q = 0; q < m.n_param; ++q) {   // rates with Parameters: r = kc prod(y) phi(y)
      const ParamEval pe = parameter_eval(m, q, [&](int d) { return kc(d); },
                                          [&](int j) { return y(j); });
      P(pe.k) *= pe.phi;
    }
    int ok = 1;
    for (int t = 0; t < m.N; ++t) {
      double acc = 0.0;
      for (int q = m.term_ptr[t]; q < m.term_ptr[t + 1]; ++q) acc += m.term_coef[q] * P(m.term_rxn[q]);
      f(t) = acc;
      if (!isfinite(acc)) ok = 0;
    }
    return ok;
  }

  __device__ void newton_matrix(double c) const {
    const DevMech& m = C.m;
    for (int k = 0; k < m.R; ++k) {
      const int a = m.rx_react[3 * k], b = m.rx_react[3 * k + 1], cc = m.rx_react[3 * k + 2];
      const double kk = kc(k);
      const int base = m.rx_pofs[k];
      const double ya = a >= 0 ? y(a) : 1.0, yb = b >= 0 ? y(b) : 1.0, yc = cc >= 0 ? y(cc) : 1.0;
      if (a >= 0) P(base) = kk * yb * yc;
      if (b >= 0) P(base + 1) = kk * ya * yc;
      if (cc >= 0) P(base + 2) = kk * ya * yb;
    }
    for (int q = 0; q < m.n_param; ++q) {   // chain rule through the Parameters
      const ParamEval pe = parameter_eval(m, q, [&](int d) { return kc(d); },
                                          [&](int j) { return y(j); });
      int o = m.rx_pofs[pe.k];
      const double r = kc(pe.k) * y(m.rx_react[3 * pe.k]) * pe.phi;
      P(o++) = kc(pe.k) * pe.phi;
      if (pe.flags & 1) P(o++) = -r * pe.inv_p;
      if (pe.flags & 2) P(o) = r * pe.g;
    }
    for (int s = 0; s < m.Z; ++s) {
      double acc = 0.0;
      for (int q = m.jc_ptr[s]; q < m.jc_ptr[s + 1]; ++q) acc += m.jc_coef[q] * P(m.jc_part[q]);
      M(s) = (m.is_diag[s] ? 1.0 : 0.0) - c * acc;
    }
  }

  // returns 1 if every pivot is a finite nonzero
  __device__ int lu() const {
    const DevMech& m = C.m;
    for (int i = 0; i < m.n_lu_task; ++i) {
      const DTask t = m.lu_task[i];
      double acc = M(t.dst);
      for (int q = t.pbeg; q < t.pend; ++q) {
        const int2 pr = m.lu_pair[q];
        acc -= M(pr.x) * M(pr.y);
      }
      if (t.diag >= 0) acc /= M(t.diag);
      M(t.dst) = acc;
    }
    int ok = 1;
    for (int t = 0; t < m.N; ++t) {
      const double u = M(m.diag[t]);
      if (!(fabs(u) > 0.0) || !isfinite(u)) ok = 0;
    }
    return ok;
  }

  __device__ void solve() const {
    const DevMech& m = C.m;
    for (int i = 0; i < m.n_fwd_task; ++i) {
      const DTask t = m.fwd_task[i];
      double acc = x(t.dst);
      for (int q = t.pbeg; q < t.pend; ++q) {
        const int2 pr = m.fwd_pair[q];
        acc -= M(pr.x) * x(pr.y);
      }
      x(t.dst) = acc;
    }
    for (int i = 0; i < m.n_bwd_task; ++i) {
      const DTask t = m.bwd_task[i];
      double acc = x(t.dst);
      for (int q = t.pbeg; q < t.pend; ++q) {
        const int2 pr = m.bwd_pair[q];
        acc -= M(pr.x) * x(pr.y);
      }
      x(t.dst) = acc / M(t.diag);
    }
  }

  // Step change by rho (see rescale_coef): evaluate the interpolant at the new points, then
  // difference.
  __device__ void rescale(int q, double rho) const {
    for (int i = 0; i < C.m.N; ++i) {
      double old[kMaxOrder + 1], a[kMaxOrder + 1];
#pragma unroll
      for (int k = 0; k <= kMaxOrder; ++k) old[k] = k <= q ? D(k, i) : 0.0;
#pragma unroll
      for (int mm = 0; mm <= kMaxOrder; ++mm) {
        double acc = 0.0;
#pragma unroll
        for (int k = kMaxOrder; k >= 1; --k)
          if (k <= q) acc = rescale_coef(k, mm, rho) * (old[k] + acc);
        a[mm] = old[0] + acc;
      }
#pragma unroll
      for (int lev = 1; lev <= kMaxOrder; ++lev) {
#pragma unroll
        for (int mm = 0; mm + lev <= kMaxOrder; ++mm) a[mm] -= a[mm + 1];
        if (lev <= q) D(lev, i) = a[0];
      }
    }
  }
};

__device__ inline double lane_wrms_d_w(const Lane& L, double scale) {
  double s = 0.0;
  for (int i = 0; i < L.C.m.N; ++i) {
    const double a = L.d(i) * scale * L.w(i);
    s += a * a;
  }
  return sqrt(s / L.C.m.N);
}

// ---------------------------------------------------------------- phase functions

// Absolute tolerance of the slot's current attempt.
__device__ inline double slot_atol(const LaneCtx& C, int slot) {
  return C.st.full[slot] >= 2 ? C.sp.atol * kRetryAtolFactor : C.sp.atol;
}

// Rate constants, initial state, starting step. Leaves the slot in PH_IDLE (ready to
// predict) or PH_DONE (failed). attempt (see kAttempts): 0 Newton with Jacobian reuse,
// 1 full Newton, 2 full Newton with a tighter atol; a retry keeps the counters of the
// earlier attempts.
__device__ void lane_init(const LaneCtx& C, int slot, int cell, int attempt, bool retry) {
  const Lane L(C, slot);
  const DevMech& m = C.m;
  const LaneState& S = C.st;
  S.cell[slot] = cell;
  S.full[slot] = attempt;
  camp_cell_stats cs = {0, 0, 0, 0, 0, 0, 0, 1};
  if (retry) cs = S.st[slot];
  const double Tk = C.env.T[cell], Pp = C.env.P[cell];
  const double cz = C.env.cos_sza ? C.env.cos_sza[cell] : 1.0;
  const double* rad = C.env.radius ? C.env.radius + (size_t)cell * m.n_inst : nullptr;
  const double* mas = C.env.mass ? C.env.mass + (size_t)cell * m.n_inst : nullptr;
  const double* ovr = C.env.override_ ? C.env.override_ + (size_t)cell * m.n_ext : nullptr;
  int ok = 1;
  for (int k = 0; k < m.R; ++k) {
    const double v = rate_constant(m, k, Tk, Pp, cz, rad, mas, ovr);
    L.kc(k) = v;
    if (!isfinite(v)) ok = 0;
  }
  const double* yrow = C.state + (size_t)cell * m.N;
  for (int t = 0; t < m.N; ++t) {
    const double v = start_value(yrow[m.perm[t]], C.sp.rtol, C.sp.atol_call);
    if (!isfinite(v)) ok = 0;
    L.y(t) = v;
    L.D(0, t) = v;
    for (int j = 1; j < kHist; ++j) L.D(j, t) = 0.0;
  }
  if (ok) {
    ok = L.forcing();
    cs.n_f++;
  }
  double h = 0.0;
  if (ok) {
    const double span = C.sp.dt;
    double s0 = 0.0, s1 = 0.0;
    for (int t = 0; t < m.N; ++t) {
      const double sc = slot_atol(C, slot) + C.sp.rtol * fabs(L.D(0, t));
      const double wt = sc > 0.0 ? 1.0 / sc : 0.0;
      L.w(t) = wt;
      L.x(t) = L.f(t);   // keep f0
      const double a = L.D(0, t) * wt, b = L.f(t) * wt;
      s0 += a * a;
      s1 += b * b;
    }
    const double d0 = sqrt(s0 / m.N), d1 = sqrt(s1 / m.N);
    const double h0 = starting_step_h0(d0, d1, span);
    for (int t = 0; t < m.N; ++t) L.y(t) = L.D(0, t) + h0 * L.f(t);
    L.forcing();
    cs.n_f++;
    double s2 = 0.0;
    for (int t = 0; t < m.N; ++t) {
      const double a = (L.f(t) - L.x(t)) * L.w(t);
      s2 += a * a;
    }
    const double d2 = sqrt(s2 / m.N) / h0;
    h = C.sp.h_init > 0.0 ? fmin(C.sp.h_init, span) : starting_step(h0, d1, d2, span);
    for (int t = 0; t < m.N; ++t) L.D(1, t) = h * L.x(t);
  }
  S.t[slot] = 0.0;
  S.h[slot] = h;
  S.q[slot] = 1;
  S.n_equal[slot] = 0;
  S.attempts[slot] = 0;
  S.lu_valid[slot] = 0;
  S.lu_age[slot] = 0;
  S.c_lu[slot] = 0.0;
  S.crate[slot] = 1.0;
  S.force_lu[slot] = 0;
  S.consec_err[slot] = 0;
  S.consec_nf[slot] = 0;
  S.st[slot] = cs;
  S.phase[slot] = ok ? PH_IDLE : PH_DONE;
  if (!ok) C.status[cell] = ST_NONFINITE;
}

// Start a step attempt: clip to the end of the host step, weights, predictor, decide on a
// new Newton matrix. Sets PH_NEWTON, or PH_DONE on failure.
__device__ void lane_predict(const LaneCtx& C, int slot, int new_step) {
  const Lane L(C, slot);
  const DevMech& m = C.m;
  const LaneState& S = C.st;
  const int cell = S.cell[slot];
  const double span = C.sp.dt;
  double t = S.t[slot], h = S.h[slot];
  int q = S.q[slot];
  if (new_step) {
    if (span - (t + h) <= 1e-12 * span) {
      const double rho = (span - t) / h;
      if (rho != 1.0) {
        L.rescale(q, rho);
        h = span - t;
        S.n_equal[slot] = 0;
      }
    }
    int ok = 1;
    for (int i = 0; i < m.N; ++i) {
      const double wt = 1.0 / (C.sp.rtol * fabs(L.D(0, i)) + slot_atol(C, slot));
      L.w(i) = wt;
      if (!isfinite(wt)) ok = 0;
    }
    S.consec_err[slot] = 0;
    S.consec_nf[slot] = 0;
    if (!ok) {
      S.phase[slot] = PH_DONE;
      C.status[cell] = ST_NONFINITE;
      return;
    }
  }
  const int att = ++S.attempts[slot];
  if (att > C.sp.max_steps || step_collapsed(h, t, C.sp.h_min)) {
    S.phase[slot] = PH_DONE;
    C.status[cell] = att > C.sp.max_steps ? ST_MAX_STEPS : ST_H_MIN;
    return;
  }
  S.h[slot] = h;
  const double gq = bdf_gamma(q);
  const double c = h / gq;
  for (int i = 0; i < m.N; ++i) {
    double s = L.D(0, i), ps = 0.0, g = 0.0;
#pragma unroll
    for (int j = 1; j <= kMaxOrder; ++j) {
      g += 1.0 / j;
      if (j <= q) {
        const double dj = L.D(j, i);
        s += dj;
        ps += g * dj;
      }
    }
    L.y(i) = s;
    L.psi(i) = ps / gq;
    L.d(i) = 0.0;
  }
  const double c_lu = S.c_lu[slot];
  const int need = S.full[slot] || S.force_lu[slot] || !S.lu_valid[slot] ||
                   fabs(c / c_lu - 1.0) > C.sp.lu_drift ||
                   S.lu_age[slot] >= C.sp.lu_max_age;
  S.fresh[slot] = need;
  S.lu_ok[slot] = 1;
  S.it[slot] = 0;
  S.phase[slot] = PH_NEWTON;
}

__device__ void lane_lu(const LaneCtx& C, int slot) {
  const LaneState& S = C.st;
  if (!S.fresh[slot]) return;
  const Lane L(C, slot);
  const double c = S.h[slot] / bdf_gamma(S.q[slot]);
  L.newton_matrix(c);
  const int ok = L.lu();
  S.st[slot].n_jac++;
  S.st[slot].n_lu++;
  S.lu_valid[slot] = ok;
  S.lu_ok[slot] = ok;
  S.c_lu[slot] = c;
  S.lu_age[slot] = 0;
  S.crate[slot] = 1.0;
  if (!ok) S.phase[slot] = PH_FINISH;
}

// One Newton iteration. Moves to PH_FINISH when converged, failed or out of iterations.
__device__ void lane_newton(const LaneCtx& C, int slot) {
  const Lane L(C, slot);
  const DevMech& m = C.m;
  const LaneState& S = C.st;
  const int it = S.it[slot];
  const double c = S.h[slot] / bdf_gamma(S.q[slot]);
  if (S.full[slot] && it > 0) {
    // full Newton: Jacobian and LU at the current iterate
    L.newton_matrix(c);
    const int lok = L.lu();
    S.st[slot].n_jac++;
    S.st[slot].n_lu++;
    S.lu_valid[slot] = lok;
    S.lu_ok[slot] = lok;
    S.c_lu[slot] = c;
    S.lu_age[slot] = 0;
    S.crate[slot] = 1.0;
    S.fresh[slot] = 1;
    if (!lok) {
      S.phase[slot] = PH_FINISH;
      return;
    }
  }
  const double c_lu = S.c_lu[slot];
  const double scale = (c == c_lu) ? 1.0 : 2.0 / (1.0 + c / c_lu);
  const int ok = L.forcing();
  S.st[slot].n_f++;
  if (!ok) {
    S.phase[slot] = PH_DONE;
    C.status[S.cell[slot]] = ST_NONFINITE;
    return;
  }
  for (int i = 0; i < m.N; ++i) L.x(i) = c * L.f(i) - L.psi(i) - L.d(i);
  L.solve();
  double s = 0.0;
  for (int i = 0; i < m.N; ++i) {
    const double dl = L.x(i) * scale;
    const double a = dl * L.w(i);
    s += a * a;
    L.y(i) += dl;
    L.d(i) += dl;
  }
  const double dn = sqrt(s / m.N);
  S.st[slot].newton_iters++;
  S.it[slot] = it + 1;
  if (!isfinite(dn)) {
    S.phase[slot] = PH_FINISH;   // not converged
    return;
  }
  double crate = S.crate[slot];
  const double dn_old = S.dn_old[slot];
  if (it > 0) crate = fmax(0.3 * crate, dn / dn_old);
  S.crate[slot] = crate;
  const double dcon = dn * fmin(1.0, crate) / C.sp.newton_tol;
  if (dcon <= 1.0) {
    S.lu_ok[slot] = 2;            // converged marker
    S.phase[slot] = PH_FINISH;
    return;
  }
  if ((it > 0 && dn > kNewtonDiverge * dn_old) || it + 1 >= C.sp.newton_maxit) {
    S.phase[slot] = PH_FINISH;
    return;
  }
  S.dn_old[slot] = dn;
}

// Error test, accept/reject, history update, order and step choice. Returns with the slot
// in PH_IDLE (next attempt or step), or PH_DONE (end of the host step or failure; the
// result or the failure status is then written).
__device__ void lane_finish(const LaneCtx& C, int slot, int* new_step) {
  const Lane L(C, slot);
  const DevMech& m = C.m;
  const LaneState& S = C.st;
  const int cell = S.cell[slot];
  int q = S.q[slot];
  double h = S.h[slot];
  const int conv = S.lu_ok[slot] == 2;
  *new_step = 0;
  if (!conv) {
    if (!S.fresh[slot] && S.lu_ok[slot]) {
      S.force_lu[slot] = 1;
      S.phase[slot] = PH_IDLE;
      return;
    }
    S.st[slot].newton_fail++;
    if (++S.consec_nf[slot] >= kMaxConsecFail) {
      S.phase[slot] = PH_DONE;
      C.status[cell] = ST_NEWTON_FAIL;
      return;
    }
    L.rescale(q, 0.25);
    S.h[slot] = h * 0.25;
    S.n_equal[slot] = 0;
    S.force_lu[slot] = 0;
    S.phase[slot] = PH_IDLE;
    return;
  }
  S.force_lu[slot] = 0;
  // positivity constraint (see kConstraintFactor): reject, never clip
  int neg = 0;
  for (int i = 0; i < m.N; ++i)
    if (L.y(i) * L.w(i) < -1.0) neg = 1;
  if (neg) {
    // a component that starts negative only counts if it is also more than one tolerance
    // unit below its start value (the input row is unchanged until the cell ends)
    const double* yin = C.state + (size_t)cell * m.N;
    neg = 0;
    for (int i = 0; i < m.N; ++i) {
      const double lo = fmin(0.0, start_value(yin[m.perm[i]], C.sp.rtol, C.sp.atol_call));
      if (L.y(i) * L.w(i) < -1.0 && (L.y(i) - lo) * L.w(i) < -1.0) neg = 1;
    }
  }
  if (neg) {
    S.st[slot].rejected++;
    L.rescale(q, kConstraintFactor);
    S.h[slot] = h * kConstraintFactor;
    S.n_equal[slot] = 0;
    S.phase[slot] = PH_IDLE;
    return;
  }
  const double err = lane_wrms_d_w(L, 1.0 / (q + 1));
  if (err > 1.0) {
    S.st[slot].rejected++;
    const int ce = ++S.consec_err[slot];
    if (ce >= kMaxConsecFail) {
      S.phase[slot] = PH_DONE;
      C.status[cell] = ST_ERR_FAIL;
      return;
    }
    S.n_equal[slot] = 0;
    S.phase[slot] = PH_IDLE;
    if (ce >= kErrRestart) {
      // restart at order 1 from y_n with a much smaller step: D[1] = h f(y_n)
      for (int i = 0; i < m.N; ++i) L.y(i) = L.D(0, i);
      L.forcing();
      S.st[slot].n_f++;
      h *= kRestartFactor;
      for (int i = 0; i < m.N; ++i) {
        L.D(1, i) = h * L.f(i);
        for (int j = 2; j < kHist; ++j) L.D(j, i) = 0.0;
      }
      S.h[slot] = h;
      S.q[slot] = 1;
      return;
    }
    double rho = fmax(kMinFactor, kSafety * pow(err, -1.0 / (q + 1)));
    if (ce >= 2) rho = fmin(rho, kMinFactor);
    L.rescale(q, rho);
    S.h[slot] = h * rho;
    return;
  }
  // accept
  *new_step = 1;
  S.st[slot].steps++;
  S.lu_age[slot]++;
  const double span = C.sp.dt;
  double t = S.t[slot];
  t = (span - (t + h) <= 1e-12 * span) ? span : t + h;
  S.t[slot] = t;
  int n_equal = S.n_equal[slot] + 1;
  for (int i = 0; i < m.N; ++i) {
    const double di = L.d(i);
    const double old_q1 = L.D(q + 1, i);
    double s = di;
    for (int j = q; j >= 0; --j) {
      s += L.D(j, i);
      L.D(j, i) = s;
    }
    L.D(q + 1, i) = di;
    L.D(q + 2, i) = di - old_q1;
  }
  if (t >= span) {
    double* yrow = C.state + (size_t)cell * m.N;
    for (int i = 0; i < m.N; ++i) yrow[m.perm[i]] = L.D(0, i);
    C.status[cell] = ST_OK;
    S.phase[slot] = PH_DONE;
    return;
  }
  if (n_equal >= q + 1) {
    double sm = 0.0, sp2 = 0.0;
    for (int i = 0; i < m.N; ++i) {
      const double wi = L.w(i);
      const double a = L.D(q, i) * wi, b = L.D(q + 2, i) * wi;
      sm += a * a;
      sp2 += b * b;
    }
    const double err_m = q > 1 ? sqrt(sm / m.N) / q : 0.0;
    const double err_p = q < C.sp.max_order ? sqrt(sp2 / m.N) / (q + 2) : 0.0;
    double rho;
    q = choose_order(q, C.sp.max_order, err, err_m, err_p, &rho);
    L.rescale(q, rho);
    S.h[slot] = h * rho;
    S.q[slot] = q;
    n_equal = 0;
  }
  S.n_equal[slot] = n_equal;
  S.phase[slot] = PH_IDLE;
}

__device__ inline void lane_store_stats(const LaneCtx& C, int slot) {
  const int cell = C.st.cell[slot];
  if (C.stats_out) {
    camp_cell_stats cs = C.st.st[slot];
    cs.order = C.st.q[slot];
    C.stats_out[cell] = cs;
  }
}

}  // namespace

// ------------------------------------------------------------------ plain engine kernels
// slot == cell. `active_count` accumulates the cells still integrating.

__device__ inline bool retry_status(int s) { return s >= ST_MAX_STEPS && s <= ST_NEWTON_FAIL; }

// First attempt: start every cell; later attempts restart only the cells whose previous
// attempt failed (the others stay done).
__global__ __launch_bounds__(256) void plain_init_kernel(LaneCtx C, int attempt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells) return;
  const bool retry = attempt > C.sp.full_newton;
  if (retry && !retry_status(C.status[c])) return;
  C.status[c] = -1;
  lane_init(C, c, c, attempt, retry);
  C.st.it[c] = 1;   // "new step" flag for the first predict
}

__global__ __launch_bounds__(256) void plain_predict_kernel(LaneCtx C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells || C.st.phase[c] != PH_IDLE) return;
  lane_predict(C, c, C.st.it[c]);
}

__global__ __launch_bounds__(256) void plain_lu_kernel(LaneCtx C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells || C.st.phase[c] != PH_NEWTON) return;
  lane_lu(C, c);
}

__global__ __launch_bounds__(256) void plain_newton_kernel(LaneCtx C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells || C.st.phase[c] != PH_NEWTON) return;
  lane_newton(C, c);
}

__global__ __launch_bounds__(256) void plain_finish_kernel(LaneCtx C, int* active_count) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells) return;
  int ph = C.st.phase[c];
  if (ph == PH_NEWTON) ph = PH_FINISH;   // iterations exhausted
  if (ph == PH_FINISH) {
    int ns = 0;
    lane_finish(C, c, &ns);
    C.st.it[c] = ns;                    // next predict starts a new step?
    ph = C.st.phase[c];
  } else if (ph == PH_DONE) {
    return;
  }
  if (ph != PH_DONE) atomicAdd(active_count, 1);
}

// finish for cells that failed during init/predict (status already set)
__global__ __launch_bounds__(256) void plain_stats_kernel(LaneCtx C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n_cells) return;
  lane_store_stats(C, c);
}

// ------------------------------------------------------------------ fused lane engine
// Persistent: slot = global thread id; cells come from `queue`.
__global__ __launch_bounds__(256) void fused_lane_kernel(LaneCtx C, int n_slots, int* queue) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  while (true) {
    const int cell = atomicAdd(queue, 1);
    if (cell >= C.n_cells) break;
    for (int attempt = C.sp.full_newton; attempt < kAttempts; ++attempt) {
      C.status[cell] = -1;
      lane_init(C, slot, cell, attempt, attempt > C.sp.full_newton);
      int new_step = 1;
      while (C.st.phase[slot] != PH_DONE) {
        lane_predict(C, slot, new_step);
        if (C.st.phase[slot] != PH_NEWTON) break;
        lane_lu(C, slot);
        while (C.st.phase[slot] == PH_NEWTON) lane_newton(C, slot);
        if (C.st.phase[slot] == PH_DONE) break;
        lane_finish(C, slot, &new_step);
      }
      if (!retry_status(C.status[cell])) break;
    }
    lane_store_stats(C, slot);
  }
}

}  // namespace camp

// ------------------------------------------------------------------ host side

#include "runtime.hpp"

namespace camp {

namespace {

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void count_failed_kernel(int n, const int* status, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int bad = (i < n && status[i] != 0) ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) bad += __shfl_xor(bad, o, kWave);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(out, bad);
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves the lane-engine workspace for n_slots (multiple of 64) out of one allocation.
struct LaneLayout {
  size_t bytes = 0;
  size_t off_kc, off_P, off_M, off_y, off_x, off_D, off_d, off_psi, off_w, off_f;
  size_t off_dbl[6], off_int[14], off_stats, off_counter;
  LaneLayout(const DevMech& m, size_t slots) {
    const size_t np = (size_t)(m.n_part > m.R ? m.n_part : m.R);
    size_t o = 0;
    auto take = [&](size_t b) {
      size_t r = o;
      o = align_up(o + b, 256);
      return r;
    };
    off_kc = take(8 * slots * m.R);
    off_P = take(8 * slots * np);
    off_M = take(8 * slots * m.Z);
    off_y = take(8 * slots * m.N);
    off_x = take(8 * slots * m.N);
    off_D = take(8 * slots * kHist * m.N);
    off_d = take(8 * slots * m.N);
    off_psi = take(8 * slots * m.N);
    off_w = take(8 * slots * m.N);
    off_f = take(8 * slots * m.N);
    for (auto& v : off_dbl) v = take(8 * slots);
    for (auto& v : off_int) v = take(4 * slots);
    off_stats = take(sizeof(camp_cell_stats) * slots);
    off_counter = take(64);
    bytes = o;
  }
};

}  // namespace

namespace {
// Cell slots of a launch: one per cell for the plain engine (n_slots == 0), else the fused
// engine's resident slots, at most one per cell.
size_t lane_slots(int n_cells, int n_slots) {
  return n_slots == 0 ? align_up((size_t)n_cells, kWave)
                      : align_up((size_t)(n_slots < n_cells ? n_slots : n_cells), 256);
}
}  // namespace

size_t lane_scratch_bytes(const DevMech& m, int n_cells, int n_slots) {
  return n_cells > 0 ? LaneLayout(m, lane_slots(n_cells, n_slots)).bytes : 0;
}

namespace {

void bind(LaneCtx& C, char* base, const LaneLayout& L) {
  auto D = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
  auto I = [&](size_t o) { return reinterpret_cast<int*>(base + o); };
  C.s = LaneSlabs{D(L.off_kc), D(L.off_P), D(L.off_M), D(L.off_y), D(L.off_x),
                  D(L.off_D), D(L.off_d), D(L.off_psi), D(L.off_w), D(L.off_f)};
  LaneState& S = C.st;
  S.t = D(L.off_dbl[0]);
  S.h = D(L.off_dbl[1]);
  S.c_lu = D(L.off_dbl[2]);
  S.crate = D(L.off_dbl[3]);
  S.err = D(L.off_dbl[4]);
  S.dn_old = D(L.off_dbl[5]);
  int** ints[14] = {&S.q,     &S.n_equal, &S.attempts, &S.lu_valid, &S.lu_age,
                    &S.consec_err, &S.consec_nf, &S.force_lu, &S.phase, &S.it,
                    &S.fresh, &S.lu_ok, &S.cell, &S.full};
  for (int i = 0; i < 14; ++i) *ints[i] = I(L.off_int[i]);
  S.st = reinterpret_cast<camp_cell_stats*>(base + L.off_stats);
}

int* g_pinned_counter() {
  thread_local int* p = nullptr;
  if (!p) {
    if (hipHostMalloc((void**)&p, 64, hipHostMallocDefault) != hipSuccess) p = nullptr;
  }
  return p;
}

}  // namespace

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_count_failed(int n, const int* status, int* out, hipStream_t stream) {
  hipError_t e = launch_fill_int(out, 1, 0, stream);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(count_failed_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, status, out);
  return hipGetLastError();
}

hipError_t run_plain(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                     const SolveParams& sp, int* status, camp_cell_stats* stats, int use_graph,
                     hipStream_t stream) {
  if (n_cells <= 0) return hipSuccess;
  const size_t slots = lane_slots(n_cells, 0);
  LaneLayout lay(m, slots);
  char* base = nullptr;
  hipError_t e = hipMallocAsync((void**)&base, lay.bytes, stream);
  if (e != hipSuccess) return e;
  LaneCtx C{};
  C.m = m;
  C.env = env;
  C.sp = sp;
  C.state = state;
  C.status = status;
  C.stats_out = stats;
  C.n_cells = n_cells;
  bind(C, base, lay);
  int* counter = reinterpret_cast<int*>(base + lay.off_counter);
  int* host_counter = g_pinned_counter();
  const dim3 grid((n_cells + 255) / 256), block(256);
  constexpr int kChunk = 4;
  auto enqueue_chunk = [&]() {
    for (int a = 0; a < kChunk; ++a) {
      hipLaunchKernelGGL(plain_predict_kernel, grid, block, 0, stream, C);
      hipLaunchKernelGGL(plain_lu_kernel, grid, block, 0, stream, C);
      for (int it = 0; it < sp.newton_maxit; ++it)
        hipLaunchKernelGGL(plain_newton_kernel, grid, block, 0, stream, C);
      hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, stream, counter, 1, 0);
      hipLaunchKernelGGL(plain_finish_kernel, grid, block, 0, stream, C, counter);
    }
  };
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph && stream != nullptr) {
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      enqueue_chunk();
      e = hipStreamEndCapture(stream, &graph);
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      hipFreeAsync(base, stream);
      return e;
    }
  }
  // The first pass integrates every cell; each later pass restarts the cells whose previous
  // attempt failed (full Newton, then also a tighter atol). Each chunk runs kChunk step
  // attempts for every active cell; a pass stops when no cell is active.
  const long long max_chunks = (long long)sp.max_steps / kChunk + 2;
  for (int pass = sp.full_newton ? 1 : 0; pass < kAttempts && e == hipSuccess; ++pass) {
    hipLaunchKernelGGL(plain_init_kernel, grid, block, 0, stream, C, pass);
    for (long long ch = 0; ch < max_chunks; ++ch) {
      if (exec) {
        e = hipGraphLaunch(exec, stream);
      } else {
        enqueue_chunk();
        e = hipGetLastError();
      }
      if (e != hipSuccess) break;
      if (host_counter) {
        e = hipMemcpyAsync(host_counter, counter, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) break;
        if (*host_counter == 0) break;
      } else {
        int hc = 0;
        e = hipMemcpy(&hc, counter, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess || hc == 0) break;
      }
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(plain_stats_kernel, grid, block, 0, stream, C);
    e = hipGetLastError();
  }
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  hipError_t e2 = hipFreeAsync(base, stream);
  return e != hipSuccess ? e : e2;
}

hipError_t run_fused_lane(const DevMech& m, const DevEnv& env, double* state, int n_cells,
                          const SolveParams& sp, int* status, camp_cell_stats* stats, int n_slots,
                          hipStream_t stream) {
  if (n_cells <= 0) return hipSuccess;
  size_t slots = lane_slots(n_cells, n_slots);
  LaneLayout lay(m, slots);
  char* base = nullptr;
  hipError_t e = hipMallocAsync((void**)&base, lay.bytes, stream);
  if (e != hipSuccess) return e;
  LaneCtx C{};
  C.m = m;
  C.env = env;
  C.sp = sp;
  C.state = state;
  C.status = status;
  C.stats_out = stats;
  C.n_cells = n_cells;
  bind(C, base, lay);
  int* queue = reinterpret_cast<int*>(base + lay.off_counter);
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, stream, queue, 1, 0);
  hipLaunchKernelGGL(fused_lane_kernel, dim3((unsigned)(slots / 256)), dim3(256), 0, stream, C,
                     (int)slots, queue);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(base, stream);
  return e != hipSuccess ? e : e2;
}

}  // namespace camp
