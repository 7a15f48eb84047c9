"""Variable-order, variable-step BDF with Newton iteration (oracle; test infrastructure only).

The paper integrates each air mass's stiff system with Backward Differentiation Formulas
and Newton iteration, with variable order, variable step size and local error control
(Sect. 2.4.1); it gives none of the integrator's internals. This oracle uses the
variable-coefficient ("fully variable step") form of BDF, written from its definition
(Hairer & Wanner, Solving ODEs II, Sect. III.5, variable step size BDF; Brenan, Campbell &
Petzold, Sect. 3.1): the history is the list of the most recent solution points themselves,
and every step builds its formula from the actual times of those points, so nothing is
re-interpolated when the step size changes.

Step from t_n to t_{n+1} = t_n + h at order q (1 <= q <= 5):

* Corrector (the BDF formula). y_{n+1} is the value for which the polynomial of degree q
  through (t_{n+1}, y_{n+1}), (t_n, y_n), ..., (t_{n+1-q}, y_{n+1-q}) has derivative
  f(y_{n+1}) at t_{n+1}. With the Lagrange basis of those q+1 nodes,
      a_0 y_{n+1} + sum_{j=1..q} a_j y_{n+1-j} = f(y_{n+1}),
  a_0 = sum_{j=1..q} 1 / (t_{n+1} - t_{n+1-j}) and a_j the basis derivatives at t_{n+1}
  (``lagrange_derivative_weights``). Divided by a_0 this is G(y) = y - psi - c f(y) = 0 with
  c = 1/a_0 and psi = -c sum_j a_j y_{n+1-j}.
* Predictor. The polynomial through the q+1 most recent past points, evaluated at t_{n+1}
  (Newton's divided-difference form). At the start only y_0 and y'(t_0) = f(y_0) exist, so
  t_0 enters as a double (confluent) node carrying the derivative (Hermite interpolation);
  the first predictor is then y_0 + h f(y_0).
* Newton. Full Newton on G: a fresh Jacobian and a dense partial-pivot LU
  (``scipy.linalg.lu_factor``) at every iteration, starting from the predictor. With
  theta = |dy_k| / |dy_{k-1}| the estimated contraction, the iteration has converged when
  the remaining error theta / (1 - theta) |dy_k| is at most NEWTON_TOL in the weighted norm,
  and has failed when theta >= 1 or after NEWTON_MAXIT iterations (Hairer & Wanner II,
  Sect. IV.8, stopping criterion of the simplified Newton iteration).
* Local error. Interpolating the exact solution at the corrector's nodes, the residual of
  the formula is w'(t_{n+1}) y^(q+1) / (q+1)!, with w(t) = prod_{j=0..q} (t - t_{n+1-j}), so
  w'(t_{n+1}) = prod_{j=1..q} (t_{n+1} - t_{n+1-j}), and the error it causes in y_{n+1} is
  that residual divided by a_0. The derivative term y^(q+1) / (q+1)! is estimated by the
  divided difference of order q+1 over t_{n+1} and the predictor's q+1 nodes:
      err_q = (w'(t_{n+1}) / a_0) y[t_{n+1}, t_n, ..., t_{n-q}].
  The step is accepted when the weighted RMS norm of err_q (weights
  1 / (rtol |y_n| + atol)) is at most 1.
* Step and order. After a rejection h shrinks by max(0.2, 0.9 err^(-1/(q+1))); from the third
  consecutive rejection the order drops to 1 and h shrinks by 10. After q+1 accepted steps
  without a change, the same estimate is formed for orders q-1 and q+1 (divided differences
  of orders q and q+2) and the order allowing the largest step is taken (ties keep q), with
  the step factor 0.9 err_p^(-1/(p+1)) capped at 5. Holding h for q+1 steps between changes
  keeps the variable-coefficient formulas zero-stable.
* The last step is shortened to land exactly on the end of the host step.

Reading choices where the paper is silent: NEWTON_TOL 0.03 in the weighted norm, at most 4
Newton iterations, a Newton failure divides h by 4, safety 0.9, factors in [0.2, 5], the
starting step heuristic of Hairer, Norsett & Wanner (Solving ODEs I, Sect. II.4), and no
lower bound on h other than the roundoff of t (the fastest transfer rates of the large
configuration exceed 1e11 s^-1, and the starting step at tight tolerances is then below
1e-11 s).
"""
import numpy as np
import scipy.linalg

MAX_ORDER = 5
SAFETY = 0.9
MIN_FACTOR = 0.2
MAX_FACTOR = 5.0
NEWTON_TOL = 0.03
NEWTON_MAXIT = 4
NEWTON_FAIL_FACTOR = 0.25
RESTART_AFTER = 3          # consecutive error-test failures before dropping to order 1
RESTART_FACTOR = 0.1
MAX_STEPS = 100_000
MAX_CONSEC_FAIL = 10
KEEP_POINTS = MAX_ORDER + 2

ST_OK, ST_MAX_STEPS, ST_H_MIN, ST_ERR_FAIL, ST_NEWTON_FAIL, ST_NONFINITE = 0, 1, 2, 3, 4, 5


def wrms(v, w):
    """Weighted root-mean-square norm sqrt(mean((v w)^2))."""
    return float(np.sqrt(np.mean((v * w) ** 2))) if v.size else 0.0


def lagrange_derivative_weights(t_new, t_past):
    """Weights a_0, a_1..a_q with P'(t_new) = a_0 y(t_new) + sum_j a_j y(t_past[j-1]) for the
    polynomial P of degree q through the q+1 distinct nodes t_new, t_past[0..q-1]."""
    nodes = [t_new] + list(t_past)
    a = np.zeros(len(nodes))
    for m, xm in enumerate(nodes):
        if m == 0:
            # derivative of l_0 at its own node: sum over the other nodes of 1/(x_0 - x_k)
            a[0] = sum(1.0 / (t_new - xk) for xk in nodes[1:])
        else:
            # l_m(t) = prod_{k != m} (t - x_k) / (x_m - x_k) vanishes at x_0 through the factor
            # (t - x_0); its derivative there is the product of the remaining factors
            num = 1.0
            den = 1.0
            for k, xk in enumerate(nodes):
                if k == m:
                    continue
                den *= xm - xk
                if k != 0:
                    num *= t_new - xk
            a[m] = num / den
    return a


def divided_differences(nodes, values, slopes):
    """Newton coefficients c_k = y[x_0, ..., x_k] of the interpolant through `nodes`.

    values[i] is y at nodes[i]. A node equal to its predecessor is a confluent (double)
    node: slopes[i] then holds y' there and replaces the first-order difference (Hermite
    interpolation). Only adjacent nodes may coincide."""
    m = len(nodes)
    col = [np.asarray(v, dtype=np.float64) for v in values]
    coef = [col[0]]
    for k in range(1, m):
        nxt = []
        for i in range(m - k):
            dx = nodes[i + k] - nodes[i]
            if k == 1 and dx == 0.0:
                nxt.append(np.asarray(slopes[i + 1], dtype=np.float64))
            else:
                nxt.append((col[i + 1] - col[i]) / dx)
        col = nxt
        coef.append(col[0])
    return coef


def newton_eval(coef, nodes, t):
    """Value at t of the Newton-form polynomial sum_k coef[k] prod_{j<k} (t - nodes[j])."""
    out = np.zeros_like(coef[0])
    basis = 1.0
    for k, c in enumerate(coef):
        out = out + basis * c
        if k < len(nodes):
            basis *= t - nodes[k]
    return out


class History:
    """The most recent solution points, newest first, and the slope at the initial point
    (kept while that point is still in the window)."""

    def __init__(self, t0, y0, f0):
        self.t = [t0]
        self.y = [np.array(y0, dtype=np.float64)]
        self.t0 = t0
        self.f0 = np.array(f0, dtype=np.float64)

    def push(self, t, y):
        self.t.insert(0, t)
        self.y.insert(0, np.array(y, dtype=np.float64))
        del self.t[KEEP_POINTS:]
        del self.y[KEEP_POINTS:]

    def nodes(self, count):
        """Up to `count` interpolation nodes, newest first: the stored points, then the
        initial point a second time (with its slope) when it is the oldest stored point.
        Returns (nodes, values, slopes)."""
        ts, ys = list(self.t), list(self.y)
        sl = [None] * len(ts)
        if ts[-1] == self.t0:
            ts.append(self.t0)
            ys.append(self.y[-1])
            sl.append(self.f0)
        return ts[:count], ys[:count], sl[:count]

    def n_nodes(self):
        return len(self.t) + (1 if self.t[-1] == self.t0 else 0)


def order_error(t_new, y_new, hist, p):
    """Estimated local error vector of the order-p formula at t_new (module docstring):
    (w'(t_new) / a_0) times the divided difference of order p+1 over t_new and the p+1
    newest history nodes. None if the history is too short."""
    if p < 1 or hist.n_nodes() < p + 1 or len(hist.t) < p:
        return None
    nodes, vals, sl = hist.nodes(p + 1)
    coef = divided_differences([t_new] + nodes, [y_new] + vals, [None] + sl)
    a = lagrange_derivative_weights(t_new, hist.t[:p])
    wprime = float(np.prod([t_new - tk for tk in hist.t[:p]]))
    return (wprime / a[0]) * coef[p + 1]


def initial_step(fun, y0, f0, rtol, atol, span):
    """Starting step size for order 1 (Hairer, Norsett & Wanner I, Sect. II.4)."""
    with np.errstate(divide="ignore"):
        w = 1.0 / (atol + rtol * np.abs(y0))
    w[~np.isfinite(w)] = 0.0
    d0 = wrms(y0, w)
    d1 = wrms(f0, w)
    h0 = 1e-6 if (d0 < 1e-5 or d1 < 1e-5) else 0.01 * d0 / d1
    h0 = min(h0, span)
    f1 = fun(y0 + h0 * f0)
    d2 = wrms(f1 - f0, w) / h0
    if max(d1, d2) <= 1e-15:
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


def corrector(fun, jac, y_pred, psi, c, w, st):
    """Full Newton on G(y) = y - psi - c f(y) from y_pred.
    Returns (status, y): status 'ok', 'fail' (no convergence) or 'nonfinite'."""
    n = y_pred.size
    y = y_pred.copy()
    prev = None
    for _ in range(NEWTON_MAXIT):
        fy = fun(y)
        st.n_f += 1
        if not np.all(np.isfinite(fy)):
            return "nonfinite", y
        resid = y - psi - c * fy
        newton_matrix = np.eye(n) - c * jac(y)
        st.n_jac += 1
        factors = scipy.linalg.lu_factor(newton_matrix, check_finite=False)
        st.n_lu += 1
        dy = -scipy.linalg.lu_solve(factors, resid, check_finite=False)
        st.newton_iters += 1
        if not np.all(np.isfinite(dy)):
            return "fail", y
        y = y + dy
        size = wrms(dy, w)
        if size == 0.0:
            return "ok", y
        if prev is not None:
            theta = size / prev
            if theta >= 1.0:
                return "fail", y
            if theta / (1.0 - theta) * size <= NEWTON_TOL:
                return "ok", y
        prev = size
    return "fail", y


def bdf_integrate(fun, jac, y0, t_span, rtol, atol, max_steps=MAX_STEPS, h_min=0.0,
                  h_init=None, max_order=MAX_ORDER):
    """Integrate y' = fun(y) over t_span; returns (y_end, status, Stats).

    The step fails (ST_H_MIN) below h_min, and below 4 units of roundoff of t, where t + h
    no longer differs from t."""
    t0, t_end = float(t_span[0]), float(t_span[1])
    span = t_end - t0
    st = Stats()
    y0 = np.asarray(y0, dtype=np.float64)
    f0 = fun(y0)
    st.n_f += 1
    if not np.all(np.isfinite(f0)):
        return y0.copy(), ST_NONFINITE, st
    if span <= 0.0:
        return y0.copy(), ST_OK, st
    if h_init is None:
        h = initial_step(fun, y0, f0, rtol, atol, span)
        st.n_f += 1
    else:
        h = min(h_init, span)
    hist = History(t0, y0, f0)
    q = 1
    held = 0            # accepted steps since the last change of h or q
    attempts = 0
    t = t0
    while t < t_end:
        if t + h >= t_end - 1e-12 * span:
            if h != t_end - t:
                held = 0
            h = t_end - t
        y_n = hist.y[0]
        with np.errstate(divide="ignore"):
            w = 1.0 / (rtol * np.abs(y_n) + atol)
        if not np.all(np.isfinite(w)):
            return y_n.copy(), ST_NONFINITE, st
        err_fails = newton_fails = 0
        while True:
            attempts += 1
            if attempts > max_steps:
                return y_n.copy(), ST_MAX_STEPS, st
            if h < h_min or h <= 4.0 * np.finfo(float).eps * abs(t):
                return y_n.copy(), ST_H_MIN, st
            t_new = t + h
            nodes, vals, sl = hist.nodes(q + 1)
            y_pred = newton_eval(divided_differences(nodes, vals, sl), nodes, t_new)
            a = lagrange_derivative_weights(t_new, hist.t[:q])
            c = 1.0 / a[0]
            psi = -c * sum(a[j] * hist.y[j - 1] for j in range(1, q + 1))
            res, y_new = corrector(fun, jac, y_pred, psi, c, w, st)
            if res == "nonfinite":
                return y_n.copy(), ST_NONFINITE, st
            if res == "fail":
                st.newton_fail += 1
                newton_fails += 1
                if newton_fails >= MAX_CONSEC_FAIL:
                    return y_n.copy(), ST_NEWTON_FAIL, st
                h *= NEWTON_FAIL_FACTOR
                held = 0
                continue
            err = wrms(order_error(t_new, y_new, hist, q), w)
            if err > 1.0:
                st.rejected += 1
                err_fails += 1
                if err_fails >= MAX_CONSEC_FAIL:
                    return y_n.copy(), ST_ERR_FAIL, st
                held = 0
                if err_fails >= RESTART_AFTER:
                    q = 1
                    h *= RESTART_FACTOR
                else:
                    h *= max(MIN_FACTOR, SAFETY * err ** (-1.0 / (q + 1)))
                continue
            break

        st.steps += 1
        hist.push(t_new, y_new)
        t = t_end if t_new >= t_end - 1e-12 * span else t_new
        held += 1
        if t >= t_end or held < q + 1:
            continue
        # order and step choice from the estimates of orders q-1, q and q+1 at this point
        best, best_q = err ** (-1.0 / (q + 1)) if err > 0.0 else np.inf, q
        for p in (q - 1, q + 1):
            if p < 1 or p > max_order:
                continue
            # the newest point is now in the history: estimate at t from the older ones
            older = History.__new__(History)
            older.t, older.y, older.t0, older.f0 = hist.t[1:], hist.y[1:], hist.t0, hist.f0
            e = order_error(t, y_new, older, p)
            if e is None:
                continue
            ep = wrms(e, w)
            fac = ep ** (-1.0 / (p + 1)) if ep > 0.0 else np.inf
            if fac > best:
                best, best_q = fac, p
        q = best_q
        h *= min(MAX_FACTOR, SAFETY * best)
        held = 0
    return hist.y[0].copy(), ST_OK, st
