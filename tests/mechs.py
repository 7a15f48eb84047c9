"""Small hand-built mechanisms for closed-form tests (inputs only, no method arithmetic)."""
import numpy as np

from paper_2111_07436_amd import workloads as W


def gas(names):
    return [W.Species(name=n, phase=-1) for n in names]


def env1(T=298.0, P=1.0e5, cos_sza=1.0, radius=None, mass=None):
    radius = np.zeros((1, 0)) if radius is None else np.atleast_2d(np.asarray(radius, float))
    mass = np.zeros((1, 0)) if mass is None else np.atleast_2d(np.asarray(mass, float))
    return W.Environment(T=np.array([T]), P=np.array([P]), cos_sza=np.array([cos_sza]),
                         radius=radius, mass=mass)


def first_order(k, names=("A", "B")):
    """A -> B as a first-order loss-like reaction, via photolysis with constant J0 = k."""
    return W.Mechanism(gas(names), [], [W.Reaction(W.RXN_PHOTOLYSIS, [0], [1], [1.0], [k, 0, 0, 0, 0, 0])])


def arrhenius_rxn(react, prod, yields, A, Ea=0.0):
    return W.Reaction(W.RXN_ARRHENIUS, list(react), list(prod), list(yields), [A, Ea, 0.0, 300.0, 0.0, 0.0])


def henry_mech(H298, C, n_inst=1, gas_mw=0.1, diff=1.5e-5, accom=0.1, density=1000.0):
    sp = [W.Species("G", -1, mw=gas_mw, diff=diff, accom=accom), W.Species("A", 0)]
    ph = [W.Phase("aq", [1], n_inst, density=density, mw_absorber=0.2)]
    rx = [W.Reaction(W.RXN_HENRY_TRANSFER, [0], [1], [1.0], [H298, C, 0, 0, 0, 0], phase=0)]
    return W.Mechanism(sp, ph, rx)


def simpol_mech(B, n_inst=1, gas_mw=0.1, diff=1.5e-5, accom=0.1, density=1400.0, mw_abs=0.2):
    sp = [W.Species("G", -1, mw=gas_mw, diff=diff, accom=accom), W.Species("A", 0)]
    ph = [W.Phase("org", [1], n_inst, density=density, mw_absorber=mw_abs)]
    rx = [W.Reaction(W.RXN_SIMPOL_TRANSFER, [0], [1], [1.0], list(B) + [0, 0], phase=0)]
    return W.Mechanism(sp, ph, rx)


def strip_sources(mech):
    """Copy of a mechanism without emission and first-order-loss processes."""
    keep = [r for r in mech.reactions if r.type not in (W.RXN_EMISSION, W.RXN_FIRST_ORDER_LOSS)]
    return W.Mechanism(mech.species, mech.phases, keep, mech.weights)
