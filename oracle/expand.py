"""Phase x instance expansion (oracle; test infrastructure only).

A Process that acts on an aerosol phase is applied identically to every instance of that
phase (Sect. 2.2.3 and Sect. 2.4.2: the Process operates on each instance as determined
by the aerosol scheme). Gas-phase Processes apply once. Phase transfer
(HenrysLawPhaseTransfer, SimpolPhaseTransfer) becomes, per instance, a condensation
reaction G -> A and an evaporation reaction A -> G (SIMPOL with the full Raoult mole
fraction adds a third, reaction-less entry carrying the instance's absorber amount, and its
evaporation rate is divided by the instance's total condensed moles, a Parameter). In a phase
whose particle radius follows the state (Sect. 2.2.3: an aerosol representation that
computes the effective radius from the particle's mass), both transfer directions carry a
second Parameter, the radius, with reaction-less entries for the instance's particle number
concentration and core volume and for the gas species' mean free path; an AqueousReversible reaction becomes,
per instance, the forward reaction and the reverse one (products -> reactants, a repeated
reactant returning as a product of that multiplicity).

State layout: gas species in input order; then for each phase, for each instance, the
phase's species in the order the phase lists them.
"""
from dataclasses import dataclass
from typing import List

ARRHENIUS, PHOTOLYSIS, EMISSION, LOSS, CONDENSED, HENRY, SIMPOL = 1, 2, 3, 4, 5, 6, 7
TROE, CUSTOM_H2O2, CUSTOM_OH_HNO3, TUNNELING, AQ_REVERSIBLE = 8, 9, 10, 11, 12

# kind of rate constant an expanded reaction carries
K_ARRHENIUS, K_PHOTOLYSIS, K_EMISSION, K_LOSS, K_CONDENSED = 1, 2, 3, 4, 5
K_HENRY_COND, K_HENRY_EVAP, K_SIMPOL_COND, K_SIMPOL_EVAP = 6, 7, 8, 9
K_TROE, K_H2O2, K_OHHNO3, K_TUNNEL, K_AQREV_FWD, K_AQREV_REV = 10, 11, 12, 13, 14, 15
K_SIMPOL_EVAP_RAOULT, K_ABSORBER = 16, 17
K_NUMBER, K_CORE_VOLUME, K_MEAN_PATH = 18, 19, 20
GAS_SPECIAL = {TROE: K_TROE, CUSTOM_H2O2: K_H2O2, CUSTOM_OH_HNO3: K_OHHNO3, TUNNELING: K_TUNNEL}


@dataclass
class XReaction:
    kind: int
    src: int           # input reaction index
    inst: int          # global phase-instance index, -1 for gas
    react: List[int]   # state indices (repeats allowed)
    prod: List[int]
    yields: List[float]
    ext: int = -1      # index among externally-settable reactions, else -1
    # Parameter (Sect. 2.2.2): the rate is divided by p = k[param_const] + sum of y over
    # param_species (a diagnosed total amount), so J gains dr/dp dp/dy; -1: no parameter
    param_const: int = -1
    param_species: List[int] = None
    # radius Parameter: the condensation rate constant k_c(r) is evaluated at the radius
    # r(y) = (3 (V0 + sum_j w_j y_j) / (4 pi N_p))^(1/3) instead of the core radius r0, with
    # V0 = k[radius_core], N_p = k[radius_number], lambda = k[radius_path], w_j = MW_j / rho
    # over radius_species; None: fixed radius
    radius_species: List[int] = None
    radius_weights: List[float] = None
    radius_number: int = -1
    radius_core: int = -1
    radius_path: int = -1
    radius_alpha: float = 0.0


@dataclass
class Expanded:
    n_state: int
    n_gas: int
    gas_state: dict            # species id -> state index (gas)
    inst_base: List[int]       # global instance -> first state index of its block
    inst_phase: List[int]      # global instance -> phase index
    rxns: List[XReaction]


def expand(mech) -> Expanded:
    gas_state = {}
    for sid, s in enumerate(mech.species):
        if s.phase < 0:
            gas_state[sid] = len(gas_state)
    n_gas = len(gas_state)
    inst_base, inst_phase = [], []
    first_inst = []
    pos = n_gas
    for p, ph in enumerate(mech.phases):
        first_inst.append(len(inst_base))
        for _ in range(ph.n_instances):
            inst_base.append(pos)
            inst_phase.append(p)
            pos += len(ph.species)
    n_state = pos

    def cond_index(p, inst_local, sid):
        ph = mech.phases[p]
        return inst_base[first_inst[p] + inst_local] + ph.species.index(sid)

    rxns = []
    n_ext = 0
    for ri, r in enumerate(mech.reactions):
        t = r.type
        if t in (ARRHENIUS, PHOTOLYSIS, EMISSION, LOSS):
            kind = {ARRHENIUS: K_ARRHENIUS, PHOTOLYSIS: K_PHOTOLYSIS,
                    EMISSION: K_EMISSION, LOSS: K_LOSS}[t]
            ext = -1
            if t != ARRHENIUS:
                ext = n_ext
                n_ext += 1
            rxns.append(XReaction(kind, ri, -1, [gas_state[s] for s in r.react],
                                  [gas_state[s] for s in r.prod], list(r.yields), ext))
        elif t in GAS_SPECIAL:
            rxns.append(XReaction(GAS_SPECIAL[t], ri, -1, [gas_state[s] for s in r.react],
                                  [gas_state[s] for s in r.prod], list(r.yields)))
        elif t == AQ_REVERSIBLE:
            p = r.phase
            back = sorted(set(r.react), key=r.react.index)
            for i in range(mech.phases[p].n_instances):
                g = first_inst[p] + i
                rxns.append(XReaction(K_AQREV_FWD, ri, g, [cond_index(p, i, s) for s in r.react],
                                      [cond_index(p, i, s) for s in r.prod], [1.0] * len(r.prod)))
                rxns.append(XReaction(K_AQREV_REV, ri, g, [cond_index(p, i, s) for s in r.prod],
                                      [cond_index(p, i, s) for s in back],
                                      [float(r.react.count(s)) for s in back]))
        elif t == CONDENSED:
            p = r.phase
            for i in range(mech.phases[p].n_instances):
                g = first_inst[p] + i
                rxns.append(XReaction(K_CONDENSED, ri, g,
                                      [cond_index(p, i, s) for s in r.react],
                                      [cond_index(p, i, s) for s in r.prod], list(r.yields)))
        elif t in (HENRY, SIMPOL):
            p = r.phase
            ph = mech.phases[p]
            gas = gas_state[r.react[0]]
            raoult = t == SIMPOL and len(r.p) > 4 and r.p[4] != 0.0
            grows = getattr(ph, "radius_from_state", False)
            if grows and t == HENRY:
                raise ValueError("Henry transfer into a phase whose radius follows the state")
            kc, ke = (K_HENRY_COND, K_HENRY_EVAP) if t == HENRY else (K_SIMPOL_COND, K_SIMPOL_EVAP)
            for i in range(ph.n_instances):
                g = first_inst[p] + i
                aer = cond_index(p, i, r.prod[0])
                block = [cond_index(p, i, s) for s in ph.species]
                cond = XReaction(kc, ri, g, [gas], [aer], [1.0])
                rxns.append(cond)
                if raoult:
                    evap = XReaction(K_SIMPOL_EVAP_RAOULT, ri, g, [aer], [gas], [1.0],
                                     param_species=block)
                else:
                    evap = XReaction(ke, ri, g, [aer], [gas], [1.0])
                rxns.append(evap)
                if raoult:
                    evap.param_const = len(rxns)
                    rxns.append(XReaction(K_ABSORBER, ri, g, [], [], []))
                if grows:
                    geo = dict(radius_species=block,
                               radius_weights=[mech.species[s].mw / ph.density for s in ph.species],
                               radius_number=len(rxns), radius_core=len(rxns) + 1,
                               radius_path=len(rxns) + 2,
                               radius_alpha=mech.species[r.react[0]].accom)
                    for xr in (cond, evap):
                        for key, v in geo.items():
                            setattr(xr, key, v)
                    rxns.append(XReaction(K_NUMBER, ri, g, [], [], []))
                    rxns.append(XReaction(K_CORE_VOLUME, ri, g, [], [], []))
                    rxns.append(XReaction(K_MEAN_PATH, ri, g, [], [], []))
        else:
            raise ValueError(f"unknown reaction type {t}")
    return Expanded(n_state, n_gas, gas_state, inst_base, inst_phase, rxns)
