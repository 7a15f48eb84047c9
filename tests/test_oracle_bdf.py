"""Pins of the oracle's whole integrator (CPU): closed forms, expm, invariants, brute force.

The closed forms are the analytic-solution tests the paper runs per Process class (Sect.
2.5, Table of tests, footnote a); the Henry test is its approximate-solution family made
exact by using a linear two-compartment system.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import solve_ivp

from paper_2111_07436_amd import workloads as W
from oracle import bdf as B
from oracle.expand import expand
from oracle.forcing import DenseSystem
from oracle.rates import rate_constants, rate_constants_cell
from oracle.solve import CellSolver, oracle_solve
from tests import mechs

RTOL, ATOL = 1e-10, 1e-20


def solve1(mech, y0, t, env=None, rtol=RTOL, atol=ATOL, **kw):
    env = mechs.env1() if env is None else env
    y, st, stats = oracle_solve(mech, env, np.atleast_2d(np.asarray(y0, float)), t, 1, rtol, atol, **kw)
    return y[0], st[0], stats[0]


def test_first_order_decay():
    k = 3e-3
    y, st, _ = solve1(mechs.first_order(k), [1e-8, 2e-9], 1000.0)
    assert st == 0
    assert y[0] == pytest.approx(1e-8 * math.exp(-k * 1000.0), rel=1e-8)
    assert y[1] == pytest.approx(2e-9 + 1e-8 * (1 - math.exp(-k * 1000.0)), rel=1e-9)


@pytest.mark.parametrize("k1,k2", [(2e-3, 5e-4), (1e-3, 1e-3)])
def test_consecutive_a_b_c(k1, k2):
    mech = W.Mechanism(mechs.gas(["A", "B", "C"]), [],
                       [W.Reaction(W.RXN_PHOTOLYSIS, [0], [1], [1.0], [k1, 0, 0, 0, 0, 0]),
                        W.Reaction(W.RXN_PHOTOLYSIS, [1], [2], [1.0], [k2, 0, 0, 0, 0, 0])])
    A0, B0, t = 1e-8, 3e-9, 2000.0
    y, st, _ = solve1(mech, [A0, B0, 0.0], t)
    if k1 != k2:
        Bt = B0 * math.exp(-k2 * t) + A0 * k1 * (math.exp(-k1 * t) - math.exp(-k2 * t)) / (k2 - k1)
    else:
        Bt = B0 * math.exp(-k1 * t) + A0 * k1 * t * math.exp(-k1 * t)
    assert y[1] == pytest.approx(Bt, rel=1e-8)
    assert y.sum() == pytest.approx(A0 + B0, rel=1e-12)


def test_second_order_2a():
    kc = 1e-12                                  # cm^3 molecule^-1 s^-1
    mech = W.Mechanism(mechs.gas(["A", "B"]), [], [mechs.arrhenius_rxn([0, 0], [1], [1.0], kc)])
    k = kc * 6.02214076e17                      # m^3 mol^-1 s^-1
    A0, t = 1e-6, 5000.0
    y, st, _ = solve1(mech, [A0, 0.0], t)
    assert y[0] == pytest.approx(A0 / (1 + 2 * k * A0 * t), rel=1e-8)


def test_second_order_a_plus_b():
    kc = 3e-13
    mech = W.Mechanism(mechs.gas(["A", "B", "C"]), [], [mechs.arrhenius_rxn([0, 1], [2], [1.0], kc)])
    k = kc * 6.02214076e17
    A0, B0, t = 2e-6, 5e-7, 3000.0
    y, st, _ = solve1(mech, [A0, B0, 0.0], t)
    a = (A0 - B0) / (1 - (B0 / A0) * math.exp(-(A0 - B0) * k * t))
    assert y[0] == pytest.approx(a, rel=1e-8)
    assert y[1] == pytest.approx(a - (A0 - B0), rel=1e-7)


def test_emission_plus_loss():
    E, k, y0, t = 4e-12, 7e-4, 3e-9, 3600.0
    mech = W.Mechanism(mechs.gas(["A"]), [],
                       [W.Reaction(W.RXN_EMISSION, [], [0], [1.0], [E, 0, 0, 0, 0, 0]),
                        W.Reaction(W.RXN_FIRST_ORDER_LOSS, [0], [], [], [k, 0, 0, 0, 0, 0])])
    y, st, _ = solve1(mech, [y0], t)
    assert y[0] == pytest.approx(E / k + (y0 - E / k) * math.exp(-k * t), rel=1e-9)


def test_henry_two_compartment():
    mech = mechs.henry_mech(5e-3, 1500.0)
    T, r, m = 285.0, 3e-7, 2e-9
    env = mechs.env1(T, 1e5, 1.0, [[r]], [[m]])
    x = expand(mech)
    k = rate_constants_cell(mech, x, T, 1e5, 1.0, env.radius[0], env.mass[0])
    kc, ke = k
    G0, A0 = 4e-9, 1e-10
    t = 0.7 / (kc + ke)
    y, st, _ = solve1(mech, [G0, A0], t, env=env)
    Geq = (G0 + A0) * ke / (kc + ke)
    assert y[0] == pytest.approx(Geq + (G0 - Geq) * math.exp(-(kc + ke) * t), rel=1e-8)


def test_linear_multisection_expm():
    # one gas species partitioning into 4 sections (Henry + SIMPOL), plus emission and loss
    sp = [W.Species("G", -1, mw=0.15, diff=1e-5, accom=0.1), W.Species("H", -1, mw=0.12),
          W.Species("A1", 0), W.Species("A2", 0)]
    ph = [W.Phase("p", [2, 3], 4, density=1400.0, mw_absorber=0.25)]
    rx = [W.Reaction(W.RXN_HENRY_TRANSFER, [0], [2], [1.0], [1e3, 2000.0, 0, 0, 0, 0], phase=0),
          W.Reaction(W.RXN_SIMPOL_TRANSFER, [1], [3], [1.0], [3.9e3, -20.0, 0, 0, 0, 0], phase=0),
          W.Reaction(W.RXN_EMISSION, [], [0], [1.0], [1e-12, 0, 0, 0, 0, 0]),
          W.Reaction(W.RXN_FIRST_ORDER_LOSS, [1], [], [], [1e-4, 0, 0, 0, 0, 0]),
          W.Reaction(W.RXN_PHOTOLYSIS, [0], [1], [0.5], [1e-3, 0, 0, 0, 0, 0])]
    mech = W.Mechanism(sp, ph, rx)
    radius = [[1e-8, 1e-7, 1e-6, 1e-5]]
    mass = [[1e-9, 3e-9, 0.0, 2e-8]]
    env = mechs.env1(290.0, 1e5, 1.0, radius, mass)
    x = expand(mech)
    s = DenseSystem(x)
    k = rate_constants(mech, x, env)[0]
    n = x.n_state
    y0 = np.linspace(1e-10, 3e-9, n)
    y0[x.inst_base[2]:x.inst_base[2] + 2] = 0.0
    # f is affine: f(y) = A y + b
    b = s.f(k, np.zeros(n))
    A = np.column_stack([s.f(k, np.eye(n)[j]) - b for j in range(n)])
    t = 600.0
    aug = np.zeros((n + 1, n + 1))
    aug[:n, :n] = A * t
    aug[:n, n] = b * t
    Ey = scipy.linalg.expm(aug) @ np.append(y0, 1.0)
    y, st, _ = solve1(mech, y0, t, env=env)
    big = np.abs(Ey[:n]) > 1e-15
    assert np.allclose(y[big], Ey[:n][big], rtol=2e-8)
    assert np.all(np.abs(y[~big]) < 1e-18)


@pytest.mark.parametrize("name,span", [("c1", 600.0), ("c3", 60.0)])
def test_weighted_mass_invariant_any_tolerance(name, span):
    wl = W.make_workload(name, n_cells=3)
    mech = mechs.strip_sources(wl.mech)
    w = wl.mech.weights
    for rtol in (1e-4, 1e-7):
        y, st, _ = oracle_solve(mech, wl.env, wl.y0, span, 1, rtol, 1e-14)
        for c in range(3):
            assert st[c] == 0
            assert w @ y[c] == pytest.approx(w @ wl.y0[c], rel=1e-11)


def test_bruteforce_rk4_small_nonstiff():
    mech = W.Mechanism(mechs.gas(["A", "B", "C", "D"]), [],
                       [mechs.arrhenius_rxn([0, 1], [2], [1.0], 2e-12),
                        mechs.arrhenius_rxn([2], [3, 1], [1.0, 0.5], 4e-3),
                        W.Reaction(W.RXN_PHOTOLYSIS, [3], [0], [1.0], [1e-3, 0, 0, 0, 0, 0])])
    x = expand(mech)
    s = DenseSystem(x)
    env = mechs.env1()
    k = rate_constants(mech, x, env)[0]
    y0 = np.array([1e-9, 2e-9, 0.0, 5e-10])
    t_end = 600.0
    lam = np.max(np.abs(np.linalg.eigvals(s.jac(k, y0))))
    nsteps = int(t_end * lam / 1e-3) + 1

    def rk4(n):
        h = t_end / n
        y = y0.copy()
        for _ in range(n):
            k1 = s.f(k, y)
            k2 = s.f(k, y + 0.5 * h * k1)
            k3 = s.f(k, y + 0.5 * h * k2)
            k4 = s.f(k, y + h * k3)
            y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        return y

    ya, yb = rk4(nsteps), rk4(2 * nsteps)
    yr = yb + (yb - ya) / 15.0                 # Richardson
    y, st, _ = solve1(mech, y0, t_end, env=env)
    assert np.allclose(y, yr, rtol=1e-8, atol=1e-20)


def test_radau_crosscheck_c1():
    wl = W.make_workload("c1", n_cells=3)
    cs = CellSolver(wl.mech)
    for c in range(3):
        k = cs.k_cell(wl.env, c)
        sol = solve_ivp(lambda t, v: cs.sys.f(k, v), (0, 600.0), wl.y0[c], method="Radau",
                        rtol=1e-12, atol=1e-24, jac=lambda t, v: cs.sys.jac(k, v))
        y, st, _ = solve1(wl.mech, wl.y0[c], 600.0, env=wl.env.take([c]))
        big = np.abs(sol.y[:, -1]) > 1e-12
        assert np.allclose(y[big], sol.y[big, -1], rtol=1e-7)


def test_self_consistency_c2():
    wl = W.make_workload("c2", n_cells=2)
    a, sa, _ = oracle_solve(wl.mech, wl.env, wl.y0, 3600.0, 1, 1e-10, 1e-20)
    b, sb, _ = oracle_solve(wl.mech, wl.env, wl.y0, 3600.0, 1, 1e-11, 1e-21)
    assert np.all(sa == 0) and np.all(sb == 0)
    big = np.abs(b) > 1e-12
    assert np.max(np.abs(a - b)[big] / np.abs(b[big])) < 1e-7


def test_failure_statuses():
    mech = mechs.first_order(1e-2)
    y0 = [1e-8, 0.0]
    _, st, _ = solve1(mech, y0, 1000.0, rtol=1e-8, atol=1e-20, max_steps=1)
    assert st == B.ST_MAX_STEPS
    _, st, _ = solve1(mech, y0, 1000.0, rtol=1e-8, atol=1e-20, h_min=2000.0)
    assert st == B.ST_H_MIN
    _, st, _ = solve1(mech, y0, 1000.0, rtol=1e-8, atol=0.0)
    assert st == B.ST_NONFINITE
    _, st, _ = solve1(mech, [np.nan, 0.0], 10.0)
    assert st == B.ST_NONFINITE
