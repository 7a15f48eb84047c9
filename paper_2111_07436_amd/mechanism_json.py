"""Writes a mechanism description (workloads.Mechanism) as the JSON document the library
reads with camp_mech_load_json (keys listed at the top of csrc/mech_json.cpp). Reading is
done by the library itself (camp.Mech.from_json); this module only serializes, so that
mechanisms built in Python can be stored as run-time configuration files.
"""
import json

from . import workloads as W

TYPE_NAMES = {
    W.RXN_ARRHENIUS: "ARRHENIUS", W.RXN_PHOTOLYSIS: "PHOTOLYSIS", W.RXN_EMISSION: "EMISSION",
    W.RXN_FIRST_ORDER_LOSS: "FIRST_ORDER_LOSS", W.RXN_CONDENSED_ARRHENIUS: "CONDENSED_PHASE_ARRHENIUS",
    W.RXN_HENRY_TRANSFER: "HENRYS_LAW_PHASE_TRANSFER", W.RXN_SIMPOL_TRANSFER: "SIMPOL_PHASE_TRANSFER",
    W.RXN_TROE: "TROE", W.RXN_CUSTOM_H2O2: "CUSTOM_H2O2", W.RXN_CUSTOM_OH_HNO3: "CUSTOM_OH_HNO3",
    W.RXN_WENNBERG_TUNNELING: "WENNBERG_TUNNELING", W.RXN_AQUEOUS_REVERSIBLE: "AQUEOUS_REVERSIBLE",
}


def _k(p, i):
    return {"A": p[i], "Ea/kb [K]": p[i + 1], "B": p[i + 2]}


def to_dict(mech: W.Mechanism) -> dict:
    names = [s.name for s in mech.species]
    species = []
    for s in mech.species:
        e = {"name": s.name, "phase": "gas" if s.phase < 0 else mech.phases[s.phase].name}
        if s.phase < 0:
            e.update({"molecular weight [kg mol-1]": s.mw, "diffusion coeff [m2 s-1]": s.diff,
                      "accommodation coefficient": s.accom})
        elif getattr(mech.phases[s.phase], "radius_from_state", False):
            e["molecular weight [kg mol-1]"] = s.mw
        species.append(e)
    phases = [{"name": ph.name, "species": [names[i] for i in ph.species],
               "density [kg m-3]": ph.density, "absorber molecular weight [kg mol-1]": ph.mw_absorber}
              for ph in mech.phases]
    for e, ph in zip(phases, mech.phases):
        if getattr(ph, "radius_from_state", False):
            e["radius from state"] = True
    procs = []
    for r in mech.reactions:
        p = list(r.p) + [0.0] * (10 - len(r.p))
        e = {"type": TYPE_NAMES[r.type]}
        if r.phase >= 0:
            e["phase"] = mech.phases[r.phase].name
        if r.type in (W.RXN_HENRY_TRANSFER, W.RXN_SIMPOL_TRANSFER):
            e["gas species"] = names[r.react[0]]
            e["aerosol species"] = names[r.prod[0]]
        else:
            reac = {}
            for i in r.react:
                reac[names[i]] = reac.get(names[i], 0) + 1
            e["reactants"] = reac
            e["products"] = {names[i]: y for i, y in zip(r.prod, r.yields)}
        t = r.type
        if t in (W.RXN_ARRHENIUS, W.RXN_CONDENSED_ARRHENIUS):
            e.update({"A": p[0], "Ea/kb [K]": p[1], "B": p[2], "D [K]": p[3], "E [Pa-1]": p[4]})
            if t == W.RXN_CONDENSED_ARRHENIUS:
                e["aqueous"] = bool(p[5])
        elif t == W.RXN_PHOTOLYSIS:
            e.update({"J0 [s-1]": p[0], "scale by cos(sza)": bool(p[1])})
        elif t == W.RXN_EMISSION:
            e["rate [mol m-3 s-1]"] = p[0]
        elif t == W.RXN_FIRST_ORDER_LOSS:
            e["rate constant [s-1]"] = p[0]
        elif t == W.RXN_HENRY_TRANSFER:
            e.update({"H298 [M Pa-1]": p[0], "C [K]": p[1]})
        elif t == W.RXN_SIMPOL_TRANSFER:
            e["B"] = p[:4]
            if p[4]:
                e["full Raoult"] = True
        elif t == W.RXN_TROE:
            e.update({"k0": _k(p, 0), "kinf": _k(p, 3), "Fc": p[6], "N": p[7]})
        elif t == W.RXN_CUSTOM_H2O2:
            e.update({"k1": _k(p, 0), "k2": _k(p, 3)})
        elif t == W.RXN_CUSTOM_OH_HNO3:
            e.update({"k0": _k(p, 0), "k2": _k(p, 3), "k3": _k(p, 6)})
        elif t == W.RXN_WENNBERG_TUNNELING:
            e.update({"A": p[0], "B [K]": p[1], "C [K3]": p[2]})
        elif t == W.RXN_AQUEOUS_REVERSIBLE:
            e.update({"A": p[0], "C [K]": p[1], "k_reverse": p[2]})
        procs.append(e)
    doc = {"species": species, "phases": phases, "processes": procs}
    if mech.phases:
        doc["aerosol representation"] = {"type": "sections",
                                         "instances": {ph.name: ph.n_instances for ph in mech.phases}}
    return doc


def to_json(mech: W.Mechanism, indent=None) -> str:
    return json.dumps(to_dict(mech), indent=indent)
