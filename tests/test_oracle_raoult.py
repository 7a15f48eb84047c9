"""Pins of the oracle's full-Raoult partitioning, a rate that depends on a Parameter
(Sect. 2.2.2: a property diagnosed from the state, entering the Jacobian by the chain rule):
equilibrium reached by integration obeys Raoult's law over the whole condensed amount, the
rate reduces to the fixed-absorber form by the exact ratio of the two amounts, and the
analytic Jacobian matches the complex-step derivative (CPU)."""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.expand import expand, K_SIMPOL_EVAP, K_SIMPOL_EVAP_RAOULT
from oracle.forcing import DenseSystem
from oracle.rates import rate_constants
from oracle.solve import oracle_solve
from tests import mechs

R_GAS = 8.314462618
MW_ABS = 0.25


def two_species_mech(B2=(-19.5, -20.0), raoult=1.0, n_inst=1):
    """Gas G1, G2 partitioning by SIMPOL into an organic phase of A1, A2 and a nonvolatile
    species N (state order: G1, G2, A1, A2, N per instance)."""
    sp = [W.Species("G1", -1, mw=0.15, diff=1.2e-5, accom=0.2),
          W.Species("G2", -1, mw=0.18, diff=1.0e-5, accom=0.3),
          W.Species("A1", 0), W.Species("A2", 0), W.Species("N", 0)]
    ph = [W.Phase("org", [2, 3, 4], n_inst, density=1300.0, mw_absorber=MW_ABS)]
    rx = [W.Reaction(W.RXN_SIMPOL_TRANSFER, [0], [2], [1.0], [3000.0, B2[0], 0, 0, raoult, 0], phase=0),
          W.Reaction(W.RXN_SIMPOL_TRANSFER, [1], [3], [1.0], [3000.0, B2[1], 0, 0, raoult, 0], phase=0)]
    return W.Mechanism(sp, ph, rx)


def test_expansion_carries_the_parameter():
    x = expand(two_species_mech(n_inst=2))
    ev = [xr for xr in x.rxns if xr.kind == K_SIMPOL_EVAP_RAOULT]
    assert len(ev) == 4
    for xr in ev:
        inst = xr.inst
        base = 2 + 3 * inst
        assert xr.param_species == [base, base + 1, base + 2]
        assert x.rxns[xr.param_const].react == [] and x.rxns[xr.param_const].inst == inst
    assert not any(xr.kind == K_SIMPOL_EVAP for xr in x.rxns)


def test_equilibrium_obeys_raoults_law_over_total_condensed_amount():
    T, r, m = 290.0, 2e-7, 2.5e-10            # n_abs = m / MW_abs = 1e-9 mol m^-3
    mech = two_species_mech()
    env = mechs.env1(T, 1e5, 1.0, [[r]], [[m]])
    y0 = np.array([[1.2e-8, 6e-9, 0.0, 0.0, 2e-9]])
    y, st, _ = oracle_solve(mech, env, y0, 2e6, 1, 1e-11, 1e-24)
    assert st[0] == 0
    g1, g2, a1, a2, n = y[0]
    n_tot = m / MW_ABS + a1 + a2 + n
    assert a1 > 0.1 * n_tot and a2 > 0.05 * n_tot   # the condensed amount matters
    for g, a, B2 in ((g1, a1, -19.5), (g2, a2, -20.0)):
        p0 = 10.0 ** (3000.0 / T + B2)
        assert g * R_GAS * T / 101325.0 == pytest.approx(a / n_tot * p0, rel=1e-6)
    assert g1 + a1 == pytest.approx(1.2e-8, rel=1e-12)
    assert g2 + a2 == pytest.approx(6e-9, rel=1e-12)
    assert n == pytest.approx(2e-9, rel=1e-12)      # nonvolatile: no forcing


def test_rate_reduces_to_fixed_absorber_by_amount_ratio():
    T, r, m = 280.0, 1e-7, 5e-10
    env = mechs.env1(T, 8e4, 1.0, [[r]], [[m]])
    y = np.array([3e-9, 1e-9, 4e-10, 7e-10, 2e-10])
    rates = []
    for flag in (1.0, 0.0):
        mech = two_species_mech(raoult=flag)
        x = expand(mech)
        s = DenseSystem(x)
        k = rate_constants(mech, x, env)[0]
        rates.append({xr.kind: [] for xr in x.rxns})
        rr = s.rates(k, y)
        for n, xr in enumerate(x.rxns):
            rates[-1][xr.kind].append(rr[n])
    n_abs = m / MW_ABS
    ratio = n_abs / (n_abs + y[2] + y[3] + y[4])
    assert np.allclose(rates[0][K_SIMPOL_EVAP_RAOULT], np.array(rates[1][K_SIMPOL_EVAP]) * ratio,
                       rtol=1e-14, atol=0)


def _complex_step(s, k, y, h=1e-150):
    Jcs = np.empty((len(y), len(y)))
    for j in range(len(y)):
        yc = y.astype(complex)
        yc[j] += 1j * h
        Jcs[:, j] = s.f(k, yc).imag / h
    return Jcs


def test_jacobian_chain_rule_matches_complex_step():
    T, r = 285.0, 1e-7
    mech = two_species_mech(n_inst=2)
    env = mechs.env1(T, 9e4, 1.0, [[r, 3e-7]], [[4e-10, 0.0]])   # second instance empty
    x = expand(mech)
    s = DenseSystem(x)
    k = rate_constants(mech, x, env)[0]
    y = np.array([3e-9, 1e-9, 4e-10, 7e-10, 2e-10, 0.0, 0.0, 0.0])
    J = s.jac(k, y)
    assert np.allclose(J, _complex_step(s, k, y), rtol=1e-13, atol=1e-300)
    # the gas row depends on every condensed species of its instance, through n_tot only
    assert J[0, 3] != 0.0 and J[0, 4] != 0.0 and J[0, 6] == 0.0
    # an instance with no absorber and no condensed mass contributes nothing
    assert not np.any(J[:, 5:]) and not np.any(s.f(k, y)[5:])


def test_zoo_jacobian_complex_step():
    wl = W.make_workload("zoo", n_cells=6)
    x = expand(wl.mech)
    s = DenseSystem(x)
    k = rate_constants(wl.mech, x, wl.env)
    assert any(xr.kind == K_SIMPOL_EVAP_RAOULT for xr in x.rxns)
    for c in range(6):
        y = wl.y0[c]
        assert np.allclose(s.jac(k[c], y), _complex_step(s, k[c], y), rtol=1e-12, atol=1e-300)
