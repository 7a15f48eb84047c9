"""Variable-order, variable-step BDF with Newton iteration (oracle; test infrastructure only).

The paper integrates each air mass's stiff system with CVODE's Backward Differentiation
Formulas and Newton iteration, with variable order, variable step and error control
(Sect. 2.4.1). CVODE's own internals are not given in the paper; this oracle writes the
published backward-difference (quasi-constant step) form of BDF of Shampine & Reichelt
(1997) with kappa = 0, orders 1..5:

* History: D[0] = y_n, D[j] = j-th backward difference of the solution at step h.
* Predictor: y0 = sum_{j=0}^{q} D[j].
* Corrector: with gamma_q = sum_{j=1}^{q} 1/j, the order-q BDF equation is
      (y - y0) + psi - (h / gamma_q) f(y) = 0,   psi = sum_{j=1}^{q} (gamma_j / gamma_q) D[j].
  Solved by full Newton: a fresh Jacobian and a dense partial-pivot LU every iteration.
* Local error estimate: (1 / (q+1)) (y - y0), in the weighted RMS norm with
  weights 1 / (rtol |y_n| + atol) (set at the start of each step).
* Step change by a factor rho: differences are those of the interpolating polynomial at
  the new spacing, D <- (R(rho) R(1))^T D with R_{k,m}(rho) = prod_{i=1}^{k} (i-1-m rho)/i.
* After q+1 accepted steps at one step size, compare the error estimates of orders q-1,
  q and q+1 and take the order allowing the largest step (ties keep the order).
* The last step is shortened to land exactly on the end of the host step.

Reading choices where the paper is silent: Newton tolerance 0.03
of the error tolerance, at most 4 Newton iterations, safety 0.9, step factor in
[0.2, 5] after an accept (<= 1 after a reject), Newton failure halves h, initial step
from the starting-step heuristic of Hairer, Norsett & Wanner (Vol. I, Sect. II.4).
"""
import numpy as np
import scipy.linalg

MAX_ORDER = 5
SAFETY = 0.9
MIN_FACTOR = 0.2
MAX_FACTOR = 5.0
NEWTON_TOL = 0.03
NEWTON_MAXIT = 4
MAX_STEPS = 100_000
MAX_CONSEC_FAIL = 10

GAMMA = np.concatenate(([0.0], np.cumsum(1.0 / np.arange(1, MAX_ORDER + 2))))
ERR_CONST = 1.0 / np.arange(1, MAX_ORDER + 3)          # ERR_CONST[q] = 1/(q+1)

ST_OK, ST_MAX_STEPS, ST_H_MIN, ST_ERR_FAIL, ST_NEWTON_FAIL, ST_NONFINITE = 0, 1, 2, 3, 4, 5


def wrms(v, w):
    return float(np.sqrt(np.mean((v * w) ** 2))) if v.size else 0.0


def interp_matrix(q, rho):
    """R_{k,m}(rho) = prod_{i=1}^{k} (i - 1 - m rho) / i, for k, m = 0..q."""
    R = np.ones((q + 1, q + 1))
    for k in range(1, q + 1):
        for m in range(q + 1):
            R[k, m] = R[k - 1, m] * (k - 1 - m * rho) / k
    return R


def rescale_history(D, q, rho):
    """Re-express D[0..q] as backward differences at step rho*h."""
    T = interp_matrix(q, rho) @ interp_matrix(q, 1.0)
    D[:q + 1] = T.T @ D[:q + 1]


def initial_step(fun, y0, f0, rtol, atol, span):
    """Starting step size (Hairer, Norsett & Wanner I, Sect. II.4) for order 1."""
    with np.errstate(divide="ignore"):
        w = 1.0 / (atol + rtol * np.abs(y0))
    w[~np.isfinite(w)] = 0.0
    d0 = wrms(y0, w)
    d1 = wrms(f0, w)
    if d0 < 1e-5 or d1 < 1e-5:
        h0 = 1e-6
    else:
        h0 = 0.01 * d0 / d1
    h0 = min(h0, span)
    y1 = y0 + h0 * f0
    f1 = fun(y1)
    d2 = wrms(f1 - f0, w) / h0
    if d1 <= 1e-15 and d2 <= 1e-15:
        h1 = max(1e-6, h0 * 1e-3)
    else:
        h1 = (0.01 / max(d1, d2)) ** 0.5
    return min(100.0 * h0, h1, span)


class Stats:
    def __init__(self):
        self.steps = 0
        self.rejected = 0
        self.newton_fail = 0
        self.newton_iters = 0
        self.n_f = 0
        self.n_jac = 0
        self.n_lu = 0

    def as_dict(self):
        return dict(self.__dict__)


def bdf_integrate(fun, jac, y0, t_span, rtol, atol, max_steps=MAX_STEPS, h_min_frac=1e-14,
                  h_init=None):
    """Integrate y' = fun(y) over t_span; returns (y_end, status, Stats)."""
    t0, t_end = float(t_span[0]), float(t_span[1])
    span = t_end - t0
    n = y0.size
    st = Stats()
    y0 = np.asarray(y0, dtype=np.float64)
    f0 = fun(y0)
    st.n_f += 1
    if not np.all(np.isfinite(f0)):
        return y0.copy(), ST_NONFINITE, st
    if span <= 0.0:
        return y0.copy(), ST_OK, st
    h = initial_step(fun, y0, f0, rtol, atol, span) if h_init is None else min(h_init, span)
    st.n_f += 1
    h_min = h_min_frac * span
    D = np.zeros((MAX_ORDER + 3, n))
    D[0] = y0
    D[1] = h * f0
    q = 1
    n_equal = 0
    t = t0
    attempts = 0
    I = np.eye(n)

    while t < t_end:
        # land exactly on t_end
        if t_end - (t + h) <= 1e-12 * span:
            rho = (t_end - t) / h
            if rho != 1.0:
                rescale_history(D, q, rho)
                h = t_end - t
                n_equal = 0
        with np.errstate(divide="ignore"):
            w = 1.0 / (rtol * np.abs(D[0]) + atol)
        if not np.all(np.isfinite(w)):
            return D[0].copy(), ST_NONFINITE, st
        consec_err = 0
        consec_newton = 0
        while True:
            attempts += 1
            if attempts > max_steps:
                return D[0].copy(), ST_MAX_STEPS, st
            if h < h_min:
                return D[0].copy(), ST_H_MIN, st
            y_pred = D[:q + 1].sum(axis=0)
            psi = (GAMMA[1:q + 1] @ D[1:q + 1]) / GAMMA[q]
            c = h / GAMMA[q]
            ok, y_new, d, nonfinite = _newton(fun, jac, y_pred, psi, c, w, I, st)
            if nonfinite:
                return D[0].copy(), ST_NONFINITE, st
            if not ok:
                st.newton_fail += 1
                consec_newton += 1
                if consec_newton >= MAX_CONSEC_FAIL:
                    return D[0].copy(), ST_NEWTON_FAIL, st
                rescale_history(D, q, 0.5)
                h *= 0.5
                n_equal = 0
                continue
            err = wrms(ERR_CONST[q] * d, w)
            if err > 1.0:
                st.rejected += 1
                consec_err += 1
                if consec_err >= MAX_CONSEC_FAIL:
                    return D[0].copy(), ST_ERR_FAIL, st
                rho = max(MIN_FACTOR, SAFETY * err ** (-1.0 / (q + 1)))
                rescale_history(D, q, rho)
                h *= rho
                n_equal = 0
                continue
            break

        # accepted
        st.steps += 1
        t = t_end if t_end - (t + h) <= 1e-12 * span else t + h
        n_equal += 1
        D[q + 2] = d - D[q + 1]
        D[q + 1] = d
        for j in range(q, -1, -1):
            D[j] += D[j + 1]
        if t >= t_end:
            break
        if n_equal < q + 1:
            continue
        err_m = wrms(ERR_CONST[q - 1] * D[q], w) if q > 1 else np.inf
        err_p = wrms(ERR_CONST[q + 1] * D[q + 2], w) if q < MAX_ORDER else np.inf
        with np.errstate(divide="ignore"):
            fac_m = err_m ** (-1.0 / q) if err_m > 0 else np.inf
            fac_0 = err ** (-1.0 / (q + 1)) if err > 0 else np.inf
            fac_p = err_p ** (-1.0 / (q + 2)) if err_p > 0 else np.inf
        best, dq = fac_0, 0
        if fac_m > best:
            best, dq = fac_m, -1
        if fac_p > best:
            best, dq = fac_p, +1
        q += dq
        rho = min(MAX_FACTOR, SAFETY * best)
        rescale_history(D, q, rho)
        h *= rho
        n_equal = 0
    return D[0].copy(), ST_OK, st


def _newton(fun, jac, y_pred, psi, c, w, I, st):
    y = y_pred.copy()
    d = np.zeros_like(y)
    dnorm_old = None
    for it in range(NEWTON_MAXIT):
        fy = fun(y)
        st.n_f += 1
        if not np.all(np.isfinite(fy)):
            return False, y, d, True
        J = jac(y)
        st.n_jac += 1
        M = I - c * J
        lu = scipy.linalg.lu_factor(M, check_finite=False)
        st.n_lu += 1
        dy = scipy.linalg.lu_solve(lu, c * fy - psi - d, check_finite=False)
        st.newton_iters += 1
        if not np.all(np.isfinite(dy)):
            return False, y, d, False
        dnorm = wrms(dy, w)
        rate = None if dnorm_old is None or dnorm_old == 0.0 else dnorm / dnorm_old
        if rate is not None and (rate >= 1.0 or
                                 rate ** (NEWTON_MAXIT - it) / (1.0 - rate) * dnorm > NEWTON_TOL):
            return False, y, d, False
        y = y + dy
        d = d + dy
        if dnorm == 0.0 or (rate is not None and rate / (1.0 - rate) * dnorm < NEWTON_TOL):
            return True, y, d, False
        dnorm_old = dnorm
    return False, y, d, False
