"""Seeded synthetic workloads: mechanism descriptions, environments and initial states.

This module only *draws* inputs. It holds none of the method's arithmetic (no rate
constants, no forcing, no integration); both the oracle and the HIP path consume what
it produces. All randomness comes from ``numpy.random.Generator(PCG64(seed))`` with a
fixed draw order: mechanism, then environment, then initial state.

Data model (follows the paper's abstraction, Sect. 2.2):

* ``Species``  -- a chemical species that lives either in the gas phase (``phase=-1``)
  or in one aerosol phase (``phase=p``). Gas species carry the transfer properties
  used by phase-transfer processes (molecular weight, gas diffusion coefficient,
  mass accommodation coefficient; Table of Process classes, HenrysLawPhaseTransfer).
* ``Phase``    -- an ``AerosolPhase`` (Sect. 2.2.3): a named set of condensed species
  whose chemistry is identical in each of its ``n_instances`` instances (modes,
  sections or particles).
* ``Reaction`` -- one ``Process`` (Table of Process classes). ``p`` holds the
  type-specific parameters; see ``RXN_*`` below.

State layout (the documented boundary layout): gas species in input order, then for
each phase in order, for each instance in order, the phase's species in the order the
phase lists them. Values are mol m^-3 of air.
"""
from __future__ import annotations

import dataclasses
import hashlib
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Process type codes (shared meaning with include/camp.h).
RXN_ARRHENIUS = 1            # p = [A, Ea/kb (K), B, D (K), E (Pa^-1), 0]
RXN_PHOTOLYSIS = 2           # p = [J0 (s^-1), sza_flag (1: scale by max(0, cos sza))]
RXN_EMISSION = 3             # p = [E (mol m^-3 s^-1)]
RXN_FIRST_ORDER_LOSS = 4     # p = [k (s^-1)]
RXN_CONDENSED_ARRHENIUS = 5  # p = [A, Ea/kb (K), B, D (K), E (Pa^-1), aqueous_flag]
RXN_HENRY_TRANSFER = 6       # p = [H298 (M Pa^-1), C (K)]
RXN_SIMPOL_TRANSFER = 7      # p = [B1, B2, B3, B4, full_raoult]
RXN_TROE = 8                 # p = [A0, Ea0/kb, B0, Ainf, Eainf/kb, Binf, Fc, N]
RXN_CUSTOM_H2O2 = 9          # p = [A1, Ea1/kb, B1, A2, Ea2/kb, B2]
RXN_CUSTOM_OH_HNO3 = 10      # p = [A0, Ea0/kb, B0, A2, Ea2/kb, B2, A3, Ea3/kb, B3]
RXN_WENNBERG_TUNNELING = 11  # p = [A, B (K), C (K^3)]
RXN_AQUEOUS_REVERSIBLE = 12  # p = [A (K_eq at 298 K), C (K), k_r]

EXTERNAL_TYPES = (RXN_PHOTOLYSIS, RXN_EMISSION, RXN_FIRST_ORDER_LOSS)


@dataclass
class Species:
    name: str
    phase: int = -1                 # -1 gas, else phase index
    mw: float = 0.1                 # kg mol^-1 (gas species: used by transfer)
    diff: float = 1.0e-5            # m^2 s^-1 (gas species: used by transfer)
    accom: float = 0.1              # mass accommodation coefficient (gas species)


@dataclass
class Phase:
    name: str
    species: List[int]              # species ids (all with .phase == this index)
    n_instances: int
    density: float = 1400.0         # kg m^-3
    mw_absorber: float = 0.2        # kg mol^-1 (SIMPOL absorbing-mass molar mass)
    radius_from_state: bool = False  # particle radius grows with the condensed species


@dataclass
class Reaction:
    type: int
    react: List[int] = field(default_factory=list)
    prod: List[int] = field(default_factory=list)
    yields: List[float] = field(default_factory=list)
    p: List[float] = field(default_factory=lambda: [0.0] * 10)
    phase: int = -1                 # condensed / transfer reactions: the phase index


@dataclass
class Mechanism:
    species: List[Species]
    phases: List[Phase]
    reactions: List[Reaction]
    # Per-species weights under which every Arrhenius, photolysis, condensed-phase and
    # transfer reaction conserves sum_i w_i y_i exactly (a property of the generator,
    # used by invariant tests). None for hand-built mechanisms.
    weights: Optional[np.ndarray] = None

    @property
    def n_gas(self) -> int:
        return sum(1 for s in self.species if s.phase < 0)

    @property
    def n_instances_total(self) -> int:
        return sum(ph.n_instances for ph in self.phases)

    @property
    def n_state(self) -> int:
        return self.n_gas + sum(len(ph.species) * ph.n_instances for ph in self.phases)

    @property
    def n_external(self) -> int:
        return sum(1 for r in self.reactions if r.type in EXTERNAL_TYPES)

    def state_names(self) -> List[str]:
        names = [s.name for s in self.species if s.phase < 0]
        for ph in self.phases:
            for i in range(ph.n_instances):
                names += [f"{ph.name}[{i}].{self.species[s].name}" for s in ph.species]
        return names


@dataclass
class Environment:
    T: np.ndarray                   # [C] K
    P: np.ndarray                   # [C] Pa
    cos_sza: np.ndarray             # [C]
    radius: np.ndarray              # [C, n_instances_total] m
    mass: np.ndarray                # [C, n_instances_total] kg m^-3 (phase mass per air volume)
    rate_override: Optional[np.ndarray] = None   # [C, n_external] or None

    @property
    def n_cells(self) -> int:
        return int(self.T.shape[0])

    def take(self, idx) -> "Environment":
        idx = np.asarray(idx)
        return Environment(
            T=self.T[idx].copy(), P=self.P[idx].copy(), cos_sza=self.cos_sza[idx].copy(),
            radius=self.radius[idx].copy(), mass=self.mass[idx].copy(),
            rate_override=None if self.rate_override is None else self.rate_override[idx].copy())


@dataclass
class Workload:
    name: str
    mech: Mechanism
    env: Environment
    y0: np.ndarray                  # [C, n_state]
    dt: float
    n_calls: int                    # consecutive host steps of length dt
    rtol: float = 1.0e-4
    atol: float = 1.0e-12
    seed: int = 0
    note: str = ""

    @property
    def n_cells(self) -> int:
        return int(self.y0.shape[0])

    def take(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return dataclasses.replace(self, env=self.env.take(idx), y0=self.y0[idx].copy())


# --------------------------------------------------------------------------------------
# Mechanism recipe
# --------------------------------------------------------------------------------------
#
# Reactant/product selection follows the structure of tropospheric mechanisms: a few
# "hub" oxidant/radical species (OH-, O3-, NO3-like) react with many organics, and each
# organic's products lie a short way downstream in an oxidation chain. This keeps the
# Jacobian sparse after LU fill, as real mechanisms are; a mechanism with uniformly random
# connectivity fills in completely and resembles no published mechanism.


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _conserving_yields(rng, w_react_sum, prod_w, tries_left):
    raw = rng.uniform(0.5, 2.0, len(prod_w))
    s = w_react_sum / float(np.dot(raw, prod_w))
    y = raw * s
    ok = bool(np.all(y >= 0.5) and np.all(y <= 2.0))
    return y, ok


@dataclass
class GasRecipe:
    n_species: int
    n_arrhenius: int
    n_photolysis: int
    n_emission: int
    n_loss: int
    hub_frac: float = 0.1
    window: int = 4
    p_hub_product: float = 0.35
    sza_photolysis: bool = False


def _draw_products(rng, n_p, organic, hubs, organics, window, p_hub, exclude):
    """Distinct product species for one reaction."""
    prods = []
    guard = 0
    while len(prods) < n_p and guard < 200:
        guard += 1
        if rng.random() < p_hub or organic is None:
            if organic is None and rng.random() >= p_hub:
                cand = int(organics[rng.integers(len(organics))])
            else:
                cand = int(hubs[rng.integers(len(hubs))])
        else:
            pos = int(np.searchsorted(organics, organic))
            nxt = pos + int(rng.integers(1, window + 1))
            if nxt >= len(organics):
                cand = int(hubs[rng.integers(len(hubs))])
            else:
                cand = int(organics[nxt])
        if cand in exclude or cand in prods:
            continue
        prods.append(cand)
    return prods


def gen_gas_mechanism(rng, r: GasRecipe):
    """Species and reactions of a synthetic gas-phase mechanism (config recipe)."""
    n = r.n_species
    n_hub = max(2, int(round(r.hub_frac * n)))
    perm = rng.permutation(n)
    hubs = np.sort(perm[:n_hub])
    organics = np.sort(perm[n_hub:])
    w = rng.uniform(1.0, 4.0, n)
    species = [Species(name=f"G{i}", phase=-1, mw=float(rng.uniform(0.05, 0.3)),
                       diff=float(rng.uniform(0.5e-5, 2.0e-5)), accom=0.1) for i in range(n)]
    rxns = []

    def draw_thermal_or_photo(n_r):
        for _attempt in range(200):
            if n_r == 2:
                if rng.random() < 0.85:
                    org = int(organics[rng.integers(len(organics))])
                    hub = int(hubs[rng.integers(len(hubs))])
                    react = [org, hub]
                else:
                    a, b = rng.choice(hubs, 2, replace=False)
                    react = [int(a), int(b)]
                    org = None
            else:
                if rng.random() < 0.8:
                    org = int(organics[rng.integers(len(organics))])
                    react = [org]
                else:
                    react = [int(hubs[rng.integers(len(hubs))])]
                    org = None
            n_p = int(rng.integers(1, 4))
            prods = _draw_products(rng, n_p, org, hubs, organics, r.window,
                                   r.p_hub_product, set(react))
            if not prods:
                continue
            ylds, ok = _conserving_yields(rng, float(w[react].sum()), w[prods], 0)
            if ok:
                return react, prods, ylds
        return react, prods, ylds

    for _ in range(r.n_arrhenius):
        n_r = 2 if rng.random() < 0.7 else 1
        react, prods, ylds = draw_thermal_or_photo(n_r)
        A = float(_loguniform(rng, 1e-20, 1e-10))
        Ea = float(rng.uniform(0.0, 3000.0))
        rxns.append(Reaction(RXN_ARRHENIUS, react, prods, [float(v) for v in ylds],
                             [A, Ea, 0.0, 300.0, 0.0, 0.0]))
    for _ in range(r.n_photolysis):
        react, prods, ylds = draw_thermal_or_photo(1)
        J0 = float(_loguniform(rng, 1e-6, 1e-2))
        rxns.append(Reaction(RXN_PHOTOLYSIS, react, prods, [float(v) for v in ylds],
                             [J0, 1.0 if r.sza_photolysis else 0.0, 0, 0, 0, 0]))
    for _ in range(r.n_emission):
        s = int(rng.integers(n))
        E = float(_loguniform(rng, 5.92e-13, 8.93e-9))
        rxns.append(Reaction(RXN_EMISSION, [], [s], [1.0], [E, 0, 0, 0, 0, 0]))
    for _ in range(r.n_loss):
        s = int(rng.integers(n))
        k = float(_loguniform(rng, 1e-6, 1e-3))
        rxns.append(Reaction(RXN_FIRST_ORDER_LOSS, [s], [], [], [k, 0, 0, 0, 0, 0]))
    return species, rxns, w, organics


@dataclass
class AerosolRecipe:
    n_phases: int
    n_sections: int
    species_per_phase: int
    aq_per_phase: int


def add_aerosol(rng, species, rxns, w_gas, organics, ar: AerosolRecipe):
    """Append aerosol phases, condensed species, aqueous reactions and transfers."""
    phases = []
    w = list(w_gas)
    partners = rng.choice(organics, size=min(len(organics), 2 * ar.n_phases), replace=False)
    for p in range(ar.n_phases):
        ids = []
        g1 = int(partners[(2 * p) % len(partners)])
        g2 = int(partners[(2 * p + 1) % len(partners)])
        for k in range(ar.species_per_phase):
            sid = len(species)
            species.append(Species(name=f"P{p}S{k}", phase=p))
            ids.append(sid)
            if k == 0:
                w.append(w[g1])
            elif k == 1:
                w.append(w[g2])
            else:
                w.append(float(rng.uniform(1.0, 4.0)))
        phases.append(Phase(name=f"phase{p}", species=ids, n_instances=ar.n_sections,
                            density=1400.0, mw_absorber=float(rng.uniform(0.1, 0.3))))
        wa = np.asarray(w)
        for _ in range(ar.aq_per_phase):
            for _attempt in range(200):
                n_r = 2 if rng.random() < 0.5 else 1
                react = [int(v) for v in rng.choice(ids, n_r, replace=False)]
                rest = [s for s in ids if s not in react]
                n_p = int(rng.integers(1, min(3, len(rest)) + 1))
                prods = [int(v) for v in rng.choice(rest, n_p, replace=False)]
                ylds, ok = _conserving_yields(rng, float(wa[react].sum()), wa[prods], 0)
                if ok:
                    break
            if n_r == 1:
                A = float(_loguniform(rng, 1e-6, 1e-2))
            else:
                A = float(_loguniform(rng, 1e-2, 1e2))
            Ea = float(rng.uniform(0.0, 3000.0))
            rxns.append(Reaction(RXN_CONDENSED_ARRHENIUS, react, prods,
                                 [float(v) for v in ylds], [A, Ea, 0.0, 300.0, 0.0, 1.0], phase=p))
        H298 = float(_loguniform(rng, 1e0, 1e6))
        C = float(rng.uniform(0.0, 6000.0))
        rxns.append(Reaction(RXN_HENRY_TRANSFER, [g1], [ids[0]], [1.0], [H298, C, 0, 0, 0, 0], phase=p))
        B1 = float(rng.uniform(3.0e3, 4.5e3))
        B2 = float(rng.uniform(-23.0, -19.0))
        rxns.append(Reaction(RXN_SIMPOL_TRANSFER, [g2], [ids[1]], [1.0], [B1, B2, 0.0, 0.0, 0, 0], phase=p))
    return phases, np.asarray(w)


def state_weights(mech: Mechanism, w_species: np.ndarray) -> np.ndarray:
    """Expand per-species weights onto the documented state layout."""
    out = [w_species[i] for i, s in enumerate(mech.species) if s.phase < 0]
    for ph in mech.phases:
        for _ in range(ph.n_instances):
            out += [w_species[s] for s in ph.species]
    return np.asarray(out, dtype=np.float64)


# --------------------------------------------------------------------------------------
# Environments and initial states
# --------------------------------------------------------------------------------------

def gen_env(rng, mech: Mechanism, n_cells: int, T_range, P_range=None, sza=False,
            zero_aerosol_frac=0.3):
    T = rng.uniform(T_range[0], T_range[1], n_cells)
    if P_range is None:
        P = np.full(n_cells, 1.0e5)
    else:
        P = rng.uniform(P_range[0], P_range[1], n_cells)
    if sza:
        chi = rng.uniform(0.0, np.pi, n_cells)
        cos_sza = np.cos(chi)
    else:
        cos_sza = np.ones(n_cells)
    ni = mech.n_instances_total
    radius = _loguniform(rng, 1e-8, 1e-5, (n_cells, ni)) if ni else np.zeros((n_cells, 0))
    mass = _loguniform(rng, 1e-10, 1e-7, (n_cells, ni)) if ni else np.zeros((n_cells, 0))
    if ni:
        zero = rng.random(n_cells) < zero_aerosol_frac
        mass[zero, :] = 0.0
    return Environment(T=T, P=P, cos_sza=cos_sza, radius=radius, mass=mass)


def gen_y0(rng, mech: Mechanism, env: Environment):
    n_cells = env.n_cells
    ng = mech.n_gas
    cols = [_loguniform(rng, 1e-12, 1e-6, (n_cells, ng))]
    inst = 0
    for ph in mech.phases:
        for _ in range(ph.n_instances):
            blk = _loguniform(rng, 1e-12, 1e-8, (n_cells, len(ph.species)))
            blk[env.mass[:, inst] == 0.0, :] = 0.0
            cols.append(blk)
            inst += 1
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


# --------------------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------------------

GAS_RECIPES = {
    "c1": GasRecipe(20, 30, 4, 3, 3, hub_frac=0.1, window=4, sza_photolysis=False),
    "c2": GasRecipe(72, 186, 25, 11, 11, hub_frac=0.1, window=4, sza_photolysis=True),
    "c5": GasRecipe(200, 510, 60, 15, 15, hub_frac=0.1, window=4, sza_photolysis=True),
}
AEROSOL_RECIPES = {
    "c3": AerosolRecipe(n_phases=6, n_sections=4, species_per_phase=5, aq_per_phase=20),
    "c5": AerosolRecipe(n_phases=10, n_sections=8, species_per_phase=4, aq_per_phase=10),
}
CELLS = {"c1": 100, "c2": 10_000, "c3": 100_000, "c5": 500_000, "zoo": 256}


def gen_rate_type_zoo(rng) -> Mechanism:
    """A small mechanism with every process type: gas-phase Arrhenius, photolysis,
    emission, first-order loss, Troe fall-off, HO2 self-reaction, OH + HNO3, tunneling, and
    an aqueous phase of 3 instances with Henry's-law and SIMPOL transfer, condensed-phase
    Arrhenius and reversible reactions, and an organic phase of 2 instances whose SIMPOL
    partitioning takes the full Raoult mole fraction and whose particles grow with the
    condensed species (two state-dependent Parameters).
    Parameters are drawn from ranges typical of tropospheric kinetics (pre-exponential
    factors in molecule cm^-3 units)."""
    lu = lambda lo, hi: float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    g = [Species(name=f"Z{i}", phase=-1, mw=float(rng.uniform(0.03, 0.2)),
                 diff=float(rng.uniform(0.8e-5, 2.0e-5)), accom=float(rng.uniform(0.05, 0.5)))
         for i in range(12)]
    aq = [Species(name=f"AQ{i}", phase=0) for i in range(5)]
    org = [Species(name=f"ORG{i}", phase=1, mw=0.15 + 0.05 * i) for i in range(3)]
    species = g + aq + org
    A0, A1, A2, A3, A4 = 12, 13, 14, 15, 16
    O0, O1, O2 = 17, 18, 19
    phases = [Phase("aqueous", [A0, A1, A2, A3, A4], 3, density=1000.0, mw_absorber=0.1),
              Phase("organic", [O0, O1, O2], 2, density=1200.0, mw_absorber=0.25,
                    radius_from_state=True)]

    def arr3():
        return [lu(1e-13, 1e-11), float(rng.uniform(-600.0, 600.0)), float(rng.uniform(-1.5, 0.0))]

    rx = [
        Reaction(RXN_ARRHENIUS, [0, 1], [2], [1.0], [lu(1e-13, 1e-11), float(rng.uniform(0, 1500)), 0, 300, 0, 0]),
        Reaction(RXN_ARRHENIUS, [2], [3, 4], [1.0, 1.0], [lu(1e-4, 1e-2), 0, 0, 300, 0, 0]),
        Reaction(RXN_PHOTOLYSIS, [3], [0, 5], [1.0, 1.0], [lu(1e-4, 1e-2), 1.0, 0, 0, 0, 0]),
        Reaction(RXN_EMISSION, [], [0], [1.0], [lu(1e-12, 1e-10), 0, 0, 0, 0, 0]),
        Reaction(RXN_EMISSION, [], [6], [1.0], [lu(1e-12, 1e-10), 0, 0, 0, 0, 0]),
        Reaction(RXN_FIRST_ORDER_LOSS, [4], [], [], [lu(1e-5, 1e-3), 0, 0, 0, 0, 0]),
        # Troe: three-body association, low- and high-pressure limits
        Reaction(RXN_TROE, [5, 1], [7], [1.0],
                 [lu(1e-31, 1e-29), 0.0, float(rng.uniform(-4.0, -1.0)), lu(1e-12, 1e-10), 0.0,
                  float(rng.uniform(-1.0, 0.0)), 0.6, 1.0, 0, 0]),
        Reaction(RXN_TROE, [6, 1], [8], [1.0],
                 [lu(1e-31, 1e-29), 0.0, float(rng.uniform(-4.0, -1.0)), lu(1e-12, 1e-10), 0.0,
                  float(rng.uniform(-1.0, 0.0)), float(rng.uniform(0.3, 0.7)), 1.0, 0, 0]),
        # HO2-like self-reaction with a pressure-dependent term
        Reaction(RXN_CUSTOM_H2O2, [9, 9], [10], [1.0],
                 [lu(1e-13, 1e-12), float(rng.uniform(-700, -300)), 0.0, lu(1e-33, 1e-32),
                  float(rng.uniform(-1100, -700)), 0.0, 0, 0, 0, 0]),
        # OH + HNO3-like
        Reaction(RXN_CUSTOM_OH_HNO3, [1, 11], [5], [1.0],
                 [lu(1e-14, 1e-13), float(rng.uniform(-900, -700)), 0.0, lu(1e-17, 1e-16),
                  float(rng.uniform(-2500, -2000)), 0.0, lu(1e-34, 1e-33),
                  float(rng.uniform(-1200, -900)), 0.0, 0]),
        # tunneling isomerization
        Reaction(RXN_WENNBERG_TUNNELING, [7], [9], [1.0],
                 [lu(1e6, 1e9), float(rng.uniform(5000, 6000)), float(rng.uniform(1e7, 1e8)), 0, 0, 0, 0, 0, 0, 0]),
        Reaction(RXN_ARRHENIUS, [10], [11], [1.0], [lu(1e-5, 1e-3), 0, 0, 300, 0, 0]),
        Reaction(RXN_PHOTOLYSIS, [8], [6, 9], [1.0, 1.0], [lu(1e-5, 1e-3), 0.0, 0, 0, 0, 0]),
        # aqueous phase
        Reaction(RXN_HENRY_TRANSFER, [2], [A0], [1.0], [lu(1e-4, 1e-2), float(rng.uniform(1000, 3000)), 0, 0, 0, 0], phase=0),
        Reaction(RXN_SIMPOL_TRANSFER, [8], [A2], [1.0], [float(rng.uniform(3.0e3, 4.5e3)), float(rng.uniform(-23, -19)), 0, 0, 0, 0], phase=0),
        Reaction(RXN_AQUEOUS_REVERSIBLE, [A0], [A1], [1.0], [lu(0.5, 20.0), float(rng.uniform(-2000, 2000)), lu(1e-3, 1e-1), 0, 0, 0, 0, 0, 0, 0], phase=0),
        Reaction(RXN_AQUEOUS_REVERSIBLE, [A2, A2], [A3], [1.0], [lu(0.1, 10.0), float(rng.uniform(-2000, 2000)), lu(1e-3, 1e-1), 0, 0, 0, 0, 0, 0, 0], phase=0),
        Reaction(RXN_CONDENSED_ARRHENIUS, [A1, A3], [A4], [1.0], [lu(0.1, 10.0), 0, 0, 300, 0, 1.0], phase=0),
    ]
    # organic phase: two semi-volatile species absorbed by Raoult's law over the whole
    # condensed amount, one converted to a nonvolatile product
    rx += [
        Reaction(RXN_SIMPOL_TRANSFER, [8], [O0], [1.0],
                 [float(rng.uniform(3.0e3, 4.5e3)), float(rng.uniform(-21, -17)), 0, 0, 1.0, 0], phase=1),
        Reaction(RXN_SIMPOL_TRANSFER, [10], [O1], [1.0],
                 [float(rng.uniform(3.0e3, 4.5e3)), float(rng.uniform(-21, -17)), 0, 0, 1.0, 0], phase=1),
        Reaction(RXN_CONDENSED_ARRHENIUS, [O0], [O2], [1.0], [lu(1e-5, 1e-3), 0, 0, 300, 0, 0.0], phase=1),
    ]
    return Mechanism(species=species, phases=phases, reactions=rx)


def make_mechanism(name: str, seed: int = 0) -> Mechanism:
    """The mechanism of a named config ("c1", "c2", "c3" or "c5"), or the rate-type test
    mechanism "zoo"."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if name == "zoo":
        return gen_rate_type_zoo(rng)
    gas_key = {"c1": "c1", "c2": "c2", "c3": "c2", "c5": "c5"}[name]
    species, rxns, w, organics = gen_gas_mechanism(rng, GAS_RECIPES[gas_key])
    phases = []
    if name in AEROSOL_RECIPES:
        phases, w = add_aerosol(rng, species, rxns, w, organics, AEROSOL_RECIPES[name])
    mech = Mechanism(species=species, phases=phases, reactions=rxns)
    mech.weights = state_weights(mech, w)
    return mech


def make_workload(name: str, n_cells: Optional[int] = None, seed: int = 0) -> Workload:
    """A named config's workload; ``n_cells`` overrides the cell count (same recipe)."""
    mech = make_mechanism(name, seed)
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    C = CELLS[name] if n_cells is None else int(n_cells)
    if name == "c1":
        env = gen_env(rng, mech, C, (260.0, 310.0), None, sza=False)
        dt, calls = 60.0, 60
    elif name in ("c2", "c3"):
        env = gen_env(rng, mech, C, (220.0, 310.0), (2.0e4, 1.013e5), sza=True)
        dt, calls = 3600.0, 1
    elif name == "c5":
        env = gen_env(rng, mech, C, (200.0, 320.0), (2.0e4, 1.013e5), sza=True)
        dt, calls = 3600.0, 1
    elif name == "zoo":
        env = gen_env(rng, mech, C, (230.0, 310.0), (2.0e4, 1.013e5), sza=True)
        dt, calls = 600.0, 1
    else:
        raise ValueError(name)
    y0 = gen_y0(rng, mech, env)
    return Workload(name=name, mech=mech, env=env, y0=y0, dt=dt, n_calls=calls, seed=seed)


def request_seed(trace_seed: int, index: int) -> int:
    h = hashlib.sha256(f"{trace_seed}:{index}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def make_request_trace(n_requests: int, seed: int = 0, rate_hz: float = 200.0,
                       cells_lo: int = 1000, cells_hi: int = 200_000):
    """Served-stream trace: Poisson arrivals, log-uniform sizes, uniform mechanism choice."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    arrival = np.cumsum(gaps)
    cells = np.floor(_loguniform(rng, cells_lo, cells_hi, n_requests)).astype(np.int64)
    mech_id = rng.integers(0, 2, n_requests)
    return arrival, cells, mech_id


def make_request(mech: Mechanism, n_cells: int, trace_seed: int, index: int):
    """Environment and initial state of one served request."""
    rng = np.random.Generator(np.random.PCG64(request_seed(trace_seed, index)))
    env = gen_env(rng, mech, n_cells, (220.0, 310.0), (2.0e4, 1.013e5), sza=True)
    y0 = gen_y0(rng, mech, env)
    return env, y0
