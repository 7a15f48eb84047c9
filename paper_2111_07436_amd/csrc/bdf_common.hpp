// Scalar BDF control shared by the engines: constants, starting step, step/order choice.
//
// The integrator is variable-order (1..5), variable-step BDF in backward-difference form
// (Shampine & Reichelt 1997, kappa = 0) with a modified Newton iteration: the Newton
// matrix I - c J (c = h / gamma_q) is factored once and reused until c drifts by more than
// 30 % or 20 steps pass, and a correction computed with a stale c is scaled by
// 2 / (1 + c / c_lu) (Brown, Byrne & Hindmarsh 1989). Convergence uses the estimated
// contraction rate (Newton tolerance 0.1 of the local error tolerance, CVODE's published
// default). The paper specifies only that CVODE's variable-order, variable-step BDF with
// Newton iteration and error control is used (Sect. 2.4.1).
#pragma once

#include "device.hpp"

namespace camp {

constexpr double kSafety = 0.9;
constexpr double kMinFactor = 0.2;
constexpr double kMaxFactor = 5.0;
constexpr double kLuGammaDrift = 0.3;
constexpr int kLuMaxAge = 20;
constexpr double kNewtonTol = 0.1;     // Newton convergence bound in the weighted norm
constexpr int kMaxConsecFail = 10;
constexpr double kNewtonDiverge = 2.0;
// Repeated local-error failures at one step (CVODE's published recovery): from the second
// failure the step factor is at most kMinFactor; from the third the method restarts at
// order 1 from y_n with the step cut by kRestartFactor.
constexpr int kErrRestart = 3;
constexpr double kRestartFactor = 0.1;
// Inequality constraint y >= 0 (CVODE's constraint option, Hindmarsh et al. 2005): a
// converged step with a component below -1 in weighted-tolerance units is rejected and
// the step cut by this factor. Without it, undershoots of fast species drive the
// bimolecular terms unstable and the step size collapses. The bound is one tolerance unit
// below min(0, start value) (see start_value).
constexpr double kConstraintFactor = 0.25;

// The value a component starts the call from: an input at most one tolerance unit (of the
// caller's tolerances) below zero, as a previous call's result may be, starts at zero;
// any other input as given. The input row itself is not changed.
__device__ __forceinline__ double start_value(double v, double rtol, double atol) {
  return (v < 0.0 && -v <= atol + rtol * -v) ? 0.0 : v;
}
// The step has collapsed: below the caller's minimum, or so small relative to the time t
// reached within the call (t >= 0) that t + h would no longer differ from t. There is no
// other lower bound: the fastest phase-transfer rates exceed 1e11 s^-1, so a cell may
// legitimately start with steps far below a picosecond.
__device__ __forceinline__ bool step_collapsed(double h, double t, double h_min) {
  return h < h_min || h <= 4.0 * __DBL_EPSILON__ * t;
}

// Attempts per cell: 0 Newton with Jacobian reuse; 1 full Newton; 2 full Newton with the
// absolute tolerance tightened by kRetryAtolFactor (a cell whose tiny, atol-controlled
// species undershoot into the constraint over and over integrates at a tolerance at least
// as tight as requested). A cell that fails an attempt (statuses 1-4) goes to the next.
constexpr int kAttempts = 3;
constexpr double kRetryAtolFactor = 0.01;

enum CellStatus : int { ST_OK = 0, ST_MAX_STEPS = 1, ST_H_MIN = 2, ST_ERR_FAIL = 3,
                        ST_NEWTON_FAIL = 4, ST_NONFINITE = 5 };

// Changing the step from h to rho*h re-expresses the history as backward differences, at
// the new spacing, of the polynomial P interpolating it. In Newton backward form
// P(t_n - m rho h) = sum_k R_k(m) D[k] with R_k(m) = prod_{i=1}^{k} (i-1-m rho)/i, i.e. the
// Horner form D0 + c_1(m)(D1 + c_2(m)(D2 + ...)) with c_k(m) = (k-1-m rho)/k. Evaluating P
// at m = 0..q new steps back and differencing those values gives the new D[1..q].
// (k is a compile-time constant wherever this is called: the division is a multiplication by
// the reciprocal, exact for k = 1, 2, 4.)
__device__ __forceinline__ double rescale_coef(int k, int m, double rho) {
  const double inv_k = k == 1 ? 1.0 : k == 2 ? 0.5 : k == 3 ? 1.0 / 3.0 : k == 4 ? 0.25 : 0.2;
  return ((double)(k - 1) - m * rho) * inv_k;
}

// Starting step (Hairer, Norsett & Wanner I, Sect. II.4) for order 1.
__device__ inline double starting_step_h0(double d0, double d1, double span) {
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  return fmin(h0, span);
}
__device__ inline double starting_step(double h0, double d1, double d2, double span) {
  double h1 = (d1 <= 1e-15 && d2 <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : sqrt(0.01 / fmax(d1, d2));
  return fmin(fmin(100.0 * h0, h1), span);
}

// Order/step choice after q+1 equal steps: returns the new order, writes the factor.
__device__ inline int choose_order(int q, int max_order, double err, double err_m, double err_p,
                                   double* factor) {
  double fm = (q > 1 && err_m > 0.0) ? pow(err_m, -1.0 / q) : (q > 1 ? 1e30 : 0.0);
  double f0 = err > 0.0 ? pow(err, -1.0 / (q + 1)) : 1e30;
  double fp = (q < max_order && err_p > 0.0) ? pow(err_p, -1.0 / (q + 2)) : (q < max_order ? 1e30 : 0.0);
  double best = f0;
  int dq = 0;
  if (fm > best) { best = fm; dq = -1; }
  if (fp > best) { best = fp; dq = +1; }
  *factor = fmin(kMaxFactor, kSafety * best);
  return q + dq;
}

}  // namespace camp
