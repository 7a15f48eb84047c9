"""Pins of the oracle integrator's building blocks against textbook facts (CPU).

* The Lagrange derivative weights on equally spaced nodes are the fixed-step BDF
  coefficients printed in the numerical-analysis literature (Hairer & Wanner II, Sect.
  III.1, BDF formulas of orders 1-5), and on arbitrary nodes they differentiate every
  polynomial of degree <= q exactly.
* Newton's divided-difference interpolant reproduces a polynomial of its degree, also
  with a confluent (Hermite) node that carries a derivative.
* The local error estimate of order q is exact for a solution that is a polynomial of
  degree q+1: it then equals y^(q+1)/(q+1)! w'(t_new) / a_0, the error the order-q formula
  makes on that solution.
"""
import numpy as np
import pytest

from oracle import bdf as B

# Fixed-step BDF coefficients, sum_j alpha_j y_{n+1-j} = h f_{n+1}, from the textbook table.
BDF_TABLE = {
    1: [1.0, -1.0],
    2: [3 / 2, -2.0, 1 / 2],
    3: [11 / 6, -3.0, 3 / 2, -1 / 3],
    4: [25 / 12, -4.0, 3.0, -4 / 3, 1 / 4],
    5: [137 / 60, -5.0, 5.0, -10 / 3, 5 / 4, -1 / 5],
}


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_equal_steps_give_textbook_bdf_coefficients(q):
    h, t = 0.37, 2.0
    a = B.lagrange_derivative_weights(t + h, [t - j * h for j in range(q)])
    assert np.allclose(a * h, BDF_TABLE[q], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_weights_differentiate_polynomials_on_uneven_nodes(q, rng):
    t_new = 1.3
    past = t_new - np.cumsum(rng.uniform(0.05, 0.6, q))
    a = B.lagrange_derivative_weights(t_new, list(past))
    for deg in range(q + 1):
        c = rng.normal(size=deg + 1)
        p = np.polynomial.Polynomial(c)
        got = a[0] * p(t_new) + sum(a[j] * p(past[j - 1]) for j in range(1, q + 1))
        assert got == pytest.approx(p.deriv()(t_new), rel=1e-10, abs=1e-10)


def test_divided_differences_reproduce_polynomial(rng):
    c = rng.normal(size=5)
    p = np.polynomial.Polynomial(c)
    nodes = [0.9, 0.4, 0.1, -0.3, -1.0]
    coef = B.divided_differences(nodes, [np.array([p(x)]) for x in nodes], [None] * 5)
    # the top coefficient of a degree-4 interpolant is the leading coefficient
    assert coef[4][0] == pytest.approx(c[4], rel=1e-11)
    for x in (1.7, -0.05, 2.5):
        assert B.newton_eval(coef, nodes, x)[0] == pytest.approx(p(x), rel=1e-11)


def test_confluent_node_is_hermite_interpolation(rng):
    c = rng.normal(size=4)
    p = np.polynomial.Polynomial(c)
    dp = p.deriv()
    # cubic from y(0.8), y(0.3), y(0) and y'(0): nodes 0.8, 0.3, 0, 0
    nodes = [0.8, 0.3, 0.0, 0.0]
    vals = [np.array([p(x)]) for x in nodes]
    slopes = [None, None, None, np.array([dp(0.0)])]
    coef = B.divided_differences(nodes, vals, slopes)
    for x in (1.1, -0.4):
        assert B.newton_eval(coef, nodes, x)[0] == pytest.approx(p(x), rel=1e-11)
    # first step of an integration: y0 + h f0
    h = B.History(0.0, np.array([2.0]), np.array([-3.0]))
    nd, vv, ss = h.nodes(2)
    assert B.newton_eval(B.divided_differences(nd, vv, ss), nd, 0.25)[0] == pytest.approx(2.0 - 0.75)


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_error_estimate_exact_for_degree_q_plus_1(q, rng):
    # y(t) = t^(q+1): y^(q+1)/(q+1)! = 1, so the order-q error is w'(t_new) / a_0
    ts = sorted(rng.uniform(0.0, 3.0, q + 1))          # past points, oldest first
    t_new = ts[-1] + 0.4
    hist = B.History(ts[0], np.array([ts[0] ** (q + 1)]), np.array([(q + 1) * ts[0] ** q]))
    for t in ts[1:]:
        hist.push(t, np.array([t ** (q + 1)]))
    e = B.order_error(t_new, np.array([t_new ** (q + 1)]), hist, q)
    past = hist.t[:q]
    a0 = sum(1.0 / (t_new - x) for x in past)
    wprime = np.prod([t_new - x for x in past])
    assert e[0] == pytest.approx(wprime / a0, rel=1e-9)


def test_bdf_step_error_matches_estimate_on_polynomial_solution():
    # y' = g(t) with y = t^3 (a non-autonomous check of the corrector): one BDF2 step from
    # exact history has error +y'''/3! w'/a_0 exactly, the value the estimate returns.
    t_past = [1.0, 0.8]                                  # newest first
    t_new = 1.25
    a = B.lagrange_derivative_weights(t_new, t_past)
    y_new = (3 * t_new ** 2 - sum(a[j] * t_past[j - 1] ** 3 for j in (1, 2))) / a[0]
    true_err = y_new - t_new ** 3
    wprime = (t_new - t_past[0]) * (t_new - t_past[1])
    assert true_err == pytest.approx(wprime / a[0], rel=1e-12)
