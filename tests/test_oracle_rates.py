"""Pins of the oracle's rate constants against physics it must reproduce (CPU).

Each pin uses a relation other than the oracle's own formula: kinetic-theory limits of the
condensation rate, the defining equilibria of Henry's and Raoult's laws reached by
integration, closed-form kinetics in the paper's own (molecule cm^-3) units, and the
paper's printed isoprene parameters (tests/golden/soa_mechanism.txt).
"""
import math
import os

import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle import rates as OR
from oracle.expand import expand
from oracle.solve import oracle_solve
from tests import mechs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
R_GAS = 8.314462618
NA = 6.02214076e23


def read_soa():
    rows = {}
    for line in open(os.path.join(GOLD, "soa_mechanism.txt")):
        line = line.split("#")[0].split()
        if line:
            rows[line[1]] = (line[0], [float(v) for v in line[2:]])
    return rows


def k_of(mech, T=298.0, P=1e5, cos_sza=1.0, radius=None, mass=None, override=None):
    x = expand(mech)
    e = mechs.env1(T, P, cos_sza, radius, mass)
    return OR.rate_constants_cell(mech, x, T, P, cos_sza, e.radius[0], e.mass[0], override), x


def test_condensation_continuum_limit():
    # Kn -> 0: Maxwell's diffusion-limited flux 4 pi r D per particle
    T, r, D, mw, a, N = 298.0, 1e-1, 1e-5, 0.1, 0.1, 1.0
    k = OR.condensation_rate(T, r, N, D, mw, a)
    assert k == pytest.approx(4 * math.pi * r * D * N, rel=1e-4)


def test_condensation_free_molecular_limit():
    # Kn -> inf: gas-kinetic collision rate pi r^2 c_bar alpha per particle
    T, r, D, mw, a, N = 298.0, 1e-11, 1e-5, 0.1, 0.1, 1.0
    c_bar = math.sqrt(8 * R_GAS * T / (math.pi * mw))
    k = OR.condensation_rate(T, r, N, D, mw, a)
    assert k == pytest.approx(math.pi * r * r * c_bar * a * N, rel=1e-3)


def test_henry_reference_temperature():
    assert OR.henry_constant(3.3e-3, 2400.0, 298.0) == 3.3e-3


def _equilibrate(mech, T, radius, mass, y0, span=1e6):
    env = mechs.env1(T, 1e5, 1.0, radius, mass)
    y, st, _ = oracle_solve(mech, env, np.atleast_2d(y0), span, 1, 1e-10, 1e-22)
    assert st[0] == 0
    return y[0]


def test_henry_equilibrium_is_henrys_law():
    # At equilibrium the phase molarity equals H(T) times the gas partial pressure.
    H298, C, T, r, m, rho = 2.0e-2, 3000.0, 280.0, 2e-7, 5e-9, 1000.0
    mech = mechs.henry_mech(H298, C, density=rho)
    y = _equilibrate(mech, T, [[r]], [[m]], [1e-8, 0.0])
    V = m / rho                                   # m^3 of phase per m^3 air
    molarity = y[1] / (1000.0 * V)                # mol per litre of phase
    p_gas = y[0] * R_GAS * T                      # Pa, ideal gas
    H_T = H298 * math.exp(C * (1 / T - 1 / 298.0))  # van 't Hoff form printed in the paper
    assert molarity == pytest.approx(H_T * p_gas, rel=1e-6)
    assert y.sum() == pytest.approx(1e-8, rel=1e-12)


def test_simpol_equilibrium_is_raoults_law_with_paper_parameters():
    soa = read_soa()
    _, (B1, B2, _) = soa["ISOP-P1"]
    T = soa["T_K"][1][0]
    r, m, rho, mw_abs = 1e-7, 2e-8, 1400.0, 0.2
    mech = mechs.simpol_mech([B1, B2], density=rho, mw_abs=mw_abs)
    y = _equilibrate(mech, T, [[r]], [[m]], [1e-7, 0.0])
    x_a = y[1] / (m / mw_abs)                     # mole fraction in the fixed absorber
    p_gas_atm = y[0] * R_GAS * T / 101325.0
    p0 = 10.0 ** (B1 / T + B2)                    # SIMPOL.1 with B3 = B4 = 0
    assert p_gas_atm == pytest.approx(x_a * p0, rel=1e-6)


def test_arrhenius_units_with_paper_isoprene_rate():
    # ISOP + OH with OH in large excess, solved in the paper's molecule cm^-3 units.
    soa = read_soa()
    _, (A, Ea, _) = soa["ISOP+OH"]
    T, P = soa["T_K"][1][0], soa["P_Pa"][1][0]
    mech = W.Mechanism(mechs.gas(["ISOP", "OH", "P1"]), [],
                       [mechs.arrhenius_rxn([0, 1], [2], [1.0], A, Ea)])
    isop0, oh = 1e-9, 1e-5                         # mol m^-3
    env = mechs.env1(T, P)
    t = 50.0
    y, st, _ = oracle_solve(mech, env, np.array([[isop0, oh, 0.0]]), t, 1, 1e-11, 1e-22)
    to_molec_cm3 = NA * 1e-6
    k_cm3 = A * math.exp(-Ea / T)
    a0, b0 = isop0 * to_molec_cm3, oh * to_molec_cm3
    # A + B -> C closed form in molecule cm^-3, written for b0 > a0
    d = b0 - a0
    e = math.exp(-d * k_cm3 * t)
    a = d * e / (b0 / a0 - e)
    assert y[0, 0] == pytest.approx(a / to_molec_cm3, rel=1e-7)


def test_arrhenius_optional_terms():
    # (T/D)^B (1 + E P): doubling T at B = 1 doubles k; E P = 1 doubles k
    mech = W.Mechanism(mechs.gas(["A", "B"]), [],
                       [W.Reaction(W.RXN_ARRHENIUS, [0], [1], [1.0], [2.0, 0.0, 1.0, 300.0, 0.0, 0.0])])
    k1, _ = k_of(mech, T=150.0)
    k2, _ = k_of(mech, T=300.0)
    assert k2[0] == pytest.approx(2 * k1[0], rel=1e-15)
    mech.reactions[0].p = [2.0, 0.0, 0.0, 300.0, 1e-5, 0.0]
    k3, _ = k_of(mech, P=1e5)
    assert k3[0] == pytest.approx(4.0, rel=1e-15)


def test_aqueous_second_order_in_molarity():
    # A + B -> C in an aqueous phase of volume V: closed form in molarity (M) units.
    sp = [W.Species("G", -1), W.Species("A", 0), W.Species("B", 0), W.Species("C", 0)]
    ph = [W.Phase("aq", [1, 2, 3], 1, density=1000.0)]
    kM = 5.0                                       # M^-1 s^-1
    rx = [W.Reaction(W.RXN_CONDENSED_ARRHENIUS, [1, 2], [3], [1.0], [kM, 0, 0, 300, 0, 1.0], phase=0)]
    mech = W.Mechanism(sp, ph, rx)
    m = 1e-9
    V = m / 1000.0
    a0M, b0M = 0.3, 0.1
    y0 = np.array([[0.0, a0M * 1000 * V, b0M * 1000 * V, 0.0]])
    t = 4.0
    env = mechs.env1(298.0, 1e5, 1.0, [[1e-7]], [[m]])
    y, st, _ = oracle_solve(mech, env, y0, t, 1, 1e-11, 1e-24)
    aM = (a0M - b0M) / (1 - (b0M / a0M) * math.exp(-(a0M - b0M) * kM * t))
    assert y[0, 1] / (1000 * V) == pytest.approx(aM, rel=1e-7)


def test_photolysis_diurnal_override_and_zero_aerosol():
    mech = W.Mechanism(mechs.gas(["A", "B"]), [],
                       [W.Reaction(W.RXN_PHOTOLYSIS, [0], [1], [1.0], [1e-3, 1.0, 0, 0, 0, 0]),
                        W.Reaction(W.RXN_EMISSION, [], [0], [1.0], [2e-12, 0, 0, 0, 0, 0])])
    k, _ = k_of(mech, cos_sza=0.5)
    assert k[0] == 0.5e-3 and k[1] == 2e-12
    k, _ = k_of(mech, cos_sza=-0.3)
    assert k[0] == 0.0
    k, _ = k_of(mech, cos_sza=0.5, override=np.array([7e-4, 3e-12]))
    assert k[0] == 7e-4 and k[1] == 3e-12
    hm = mechs.henry_mech(1e-2, 0.0, n_inst=2)
    k, _ = k_of(hm, radius=[[1e-7, 1e-7]], mass=[[1e-9, 0.0]])
    assert np.all(k[:2] > 0) and np.all(k[2:] == 0.0)
