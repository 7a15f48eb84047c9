"""Pins of the oracle's remaining rate-constant forms (paper tables of Process classes:
Troe, CustomH2o2, CustomOhHno3, WennbergTunneling, AqueousReversible), against facts the
forms must satisfy rather than their own expressions: fall-off limits and the definition of
Fc as the broadening at the centre of the fall-off curve, the limits of the custom forms,
a hand-evaluated tunneling rate, and equilibria and relaxation closed forms reached by
integration (the paper tests every Process class against an analytic solution, Sect. 2.5).
"""
import math

import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle import rates as OR
from oracle.expand import expand, K_AQREV_FWD, K_AQREV_REV
from oracle.solve import oracle_solve
from tests import mechs

KB = 1.380649e-23
NA = 6.02214076e23


def air(T, P):
    return P / (KB * T) * 1e-6            # molecule cm^-3


def test_troe_centre_is_fc_half_kinf():
    # k0[M] = kinf: the fall-off curve's centre, where the broadening factor is Fc
    T, P = 270.0, 6e4
    kinf = 3e-11
    for Fc, N in ((0.6, 1.0), (0.35, 1.3)):
        p = [kinf / air(T, P), 0.0, 0.0, kinf, 0.0, 0.0, Fc, N]
        assert OR.troe(p, T, P) == pytest.approx(Fc * kinf / 2.0, rel=1e-13)


def test_troe_pressure_limits_and_symmetry():
    T, P = 250.0, 1e5
    M = air(T, P)
    kinf = 2e-11
    for ratio in (1e-200, 1e200):
        p = [ratio * kinf / M, 0.0, 0.0, kinf, 0.0, 0.0, 0.6, 1.0]
        k = OR.troe(p, T, P)
        lim = ratio * kinf if ratio < 1 else kinf          # k0[M] at low, kinf at high pressure
        assert k == pytest.approx(lim, rel=2e-5)
    # the broadening factor depends on |log10(k0[M]/kinf)| only
    def broadening(r):
        p = [r * kinf / M, 0.0, 0.0, kinf, 0.0, 0.0, 0.45, 0.8]
        return OR.troe(p, T, P) / (r * kinf / (1.0 + r))
    for r in (3.0, 40.0, 1e4):
        assert broadening(r) == pytest.approx(broadening(1.0 / r), rel=1e-13)
        assert 0.45 < broadening(r) < 1.0


def test_custom_h2o2_limits():
    T = 280.0
    p = [3e-13, -460.0, 0.0, 2.1e-33, -920.0, 0.0]
    k_zero = OR.custom_h2o2(p, T, 1e-300)
    assert k_zero == pytest.approx(3e-13 * math.exp(460.0 / T), rel=1e-14)
    # linear in pressure at fixed temperature
    k1, k2, k3 = (OR.custom_h2o2(p, T, P) for P in (2e4, 4e4, 6e4))
    assert (k3 - k2) == pytest.approx(k2 - k1, rel=1e-11)
    assert (k2 - k1) == pytest.approx(2.1e-33 * math.exp(920.0 / T) * (air(T, 4e4) - air(T, 2e4)), rel=1e-11)


def test_custom_oh_hno3_limits():
    T = 290.0
    p = [2.4e-14, -460.0, 0.0, 2.7e-17, -2199.0, 0.0, 6.5e-34, -1335.0, 0.0]
    k0 = 2.4e-14 * math.exp(460.0 / T)
    k2 = 2.7e-17 * math.exp(2199.0 / T)
    k3 = 6.5e-34 * math.exp(1335.0 / T)
    assert OR.custom_oh_hno3(p, T, 1e-300) == pytest.approx(k0, rel=1e-14)     # [M] -> 0
    assert OR.custom_oh_hno3(p, T, 1e200) == pytest.approx(k0 + k2, rel=1e-12)  # [M] -> inf
    P_half = k2 / k3 * KB * T * 1e6                    # k3 [M] = k2
    assert OR.custom_oh_hno3(p, T, P_half) == pytest.approx(k0 + k2 / 2.0, rel=1e-12)


def test_tunneling_hand_value_and_reduction():
    # 1e-12 exp(-500/250) exp(1e6/250^3) = 1e-12 e^-2 e^0.064, evaluated by hand
    assert OR.tunneling([1e-12, 500.0, 1e6], 250.0) == pytest.approx(1.4427991674278818e-13, rel=1e-14)
    assert OR.tunneling([7.5, 0.0, 0.0], 211.0) == 7.5


def test_gas_forms_in_mechanism_units():
    # a bimolecular Troe reaction A + B -> C with B in excess: first-order decay of A in
    # molecule cm^-3 units, then converted to mol m^-3
    T, P = 260.0, 8e4
    p = [6e-31, 0.0, -3.0, 1.5e-11, 0.0, -0.5, 0.6, 1.0, 0.0, 0.0]
    mech = W.Mechanism(mechs.gas(["A", "B", "C"]), [], [W.Reaction(W.RXN_TROE, [0, 1], [2], [1.0], p)])
    a0, b = 1e-10, 1e-6                                  # mol m^-3
    env = mechs.env1(T, P)
    t = 30.0
    y, st, _ = oracle_solve(mech, env, np.array([[a0, b, 0.0]]), t, 1, 1e-11, 1e-24)
    assert st[0] == 0
    k_cm3 = OR.troe(p, T, P)
    b_cm3 = b * NA * 1e-6
    # B barely changes (a0 << b): A = a0 exp(-k b t) to first order in a0/b
    a_pred = a0 * math.exp(-k_cm3 * b_cm3 * t)
    assert y[0, 0] == pytest.approx(a_pred, rel=1e-3)
    assert y[0, 0] + y[0, 2] == pytest.approx(a0, rel=1e-12)


def _aq_mech(react, prod, A, C, kr, n_inst=1):
    sp = [W.Species("G", -1)] + [W.Species(f"X{i}", 0) for i in range(3)]
    ph = [W.Phase("aq", [1, 2, 3], n_inst, density=1000.0)]
    rx = [W.Reaction(W.RXN_AQUEOUS_REVERSIBLE, react, prod, [1.0] * len(prod),
                     [A, C, kr, 0, 0, 0, 0, 0, 0, 0], phase=0)]
    return W.Mechanism(sp, ph, rx)


def test_aqueous_reversible_expansion():
    x = expand(_aq_mech([1, 1], [2], 2.0, 0.0, 0.1, n_inst=2))
    kinds = [xr.kind for xr in x.rxns]
    assert kinds == [K_AQREV_FWD, K_AQREV_REV] * 2
    fwd, rev = x.rxns[2], x.rxns[3]                     # second instance: block at 4..6
    assert fwd.react == [4, 4] and fwd.prod == [5]
    assert rev.react == [5] and rev.prod == [4] and rev.yields == [2.0]


@pytest.mark.parametrize("T", [298.0, 275.0])
def test_aqueous_reversible_equilibria(T):
    # A <-> B: [B]/[A] = K_eq(T); 2 A <-> C: [C]/[A]^2 = K_eq(T) (molarities)
    A_, C_, kr = 3.0, 1800.0, 0.05
    K = A_ * math.exp(C_ * (1.0 / T - 1.0 / 298.0))
    m = 2e-9
    V = m / 1000.0
    env = mechs.env1(T, 1e5, 1.0, [[1e-7]], [[m]])
    to_air = 1000.0 * V                                   # M -> mol m^-3 air
    mech = _aq_mech([1], [2], A_, C_, kr)
    y, st, _ = oracle_solve(mech, env, np.array([[0.0, 0.4 * to_air, 0.1 * to_air, 0.0]]), 2e3, 1,
                            1e-11, 1e-26)
    assert st[0] == 0
    assert y[0, 2] / y[0, 1] == pytest.approx(K, rel=1e-7)
    mech2 = _aq_mech([1, 1], [3], A_, C_, kr)
    y, st, _ = oracle_solve(mech2, env, np.array([[0.0, 0.5 * to_air, 0.0, 0.2 * to_air]]), 2e4, 1,
                            1e-11, 1e-26)
    assert st[0] == 0
    a, c = y[0, 1] / to_air, y[0, 3] / to_air
    assert c / (a * a) == pytest.approx(K, rel=1e-6)
    assert a + 2 * c == pytest.approx(0.5 + 2 * 0.2, rel=1e-12)


def test_aqueous_reversible_relaxation():
    # A <-> B, first order both ways: A(t) = A_eq + (A0 - A_eq) exp(-(kf + kr) t)
    T, kr, K = 298.0, 0.02, 4.0
    kf = K * kr
    m = 5e-9
    env = mechs.env1(T, 1e5, 1.0, [[1e-7]], [[m]])
    mech = _aq_mech([1], [2], K, 0.0, kr)
    a0, b0 = 3e-9, 1e-9
    t = 25.0
    y, st, _ = oracle_solve(mech, env, np.array([[0.0, a0, b0, 0.0]]), t, 1, 1e-11, 1e-26)
    a_eq = (a0 + b0) * kr / (kf + kr)
    assert y[0, 1] == pytest.approx(a_eq + (a0 - a_eq) * math.exp(-(kf + kr) * t), rel=1e-8)


def test_aqueous_reversible_zero_mass_instance_is_inert():
    mech = _aq_mech([1], [2], 2.0, 0.0, 0.1, n_inst=2)
    x = expand(mech)
    k = OR.rate_constants_cell(mech, x, 290.0, 1e5, 1.0, np.array([1e-7, 1e-7]),
                               np.array([1e-9, 0.0]))
    assert np.all(k[:2] > 0) and np.all(k[2:] == 0.0)
