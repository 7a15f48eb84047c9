"""Rate constants from the environment (oracle; test infrastructure only).

One value per expanded reaction and cell. The rate constants are held fixed over one
host time step: the host updates rates before each solve (Sect. 2.4.2, runtime
workflow), and Process objects recompute environment-dependent parameters only when the
environment changes (Table of Process functions, update_for_new_environmental_state).

State concentrations are mol m^-3 of air. Formulas (Table of Process classes):

* Arrhenius: k = A exp(-Ea/(kb T)) (T/D)^B (1 + E P), with A in (molecule cm^-3)^-(n_r-1)
  s^-1; Ea is supplied already divided by kb (in K). Converted to (mol m^-3)^-(n_r-1) s^-1
  by (N_A * 1e-6)^(n_r - 1).
* Photolysis, Emission, FirstOrderLoss: the configured value, or the host-supplied value
  (Sect. 2.4.2: Process-connection objects). Photolysis may be scaled by max(0, cos sza).
* CondensedPhaseArrhenius: Arrhenius form; aqueous rate constants are in M^-(n_r-1) s^-1
  and act on molarities [X] = y_X / (1000 V), so in air units k_air = k (1000 V)^(1-n_r),
  with V = m / rho the phase volume per volume of air.
* Phase transfer (HenrysLawPhaseTransfer, SimpolPhaseTransfer): condensation
  k_c = 4 pi r D_g f_fs(Kn, alpha) per particle, times the particle number concentration
  N = m / (rho 4/3 pi r^3). Fuchs-Sutugin f_fs with Kn = lambda / r,
  lambda = 3 D_g / c_bar, c_bar = sqrt(8 R T / (pi MW)).
  Henry: H(T) = H298 exp(C (1/T - 1/298)) in M Pa^-1; at equilibrium the phase molarity
  is H times the gas partial pressure, so A_eq / G_eq = H 1000 V R T and
  k_evap = k_c / (H 1000 V R T).
  SIMPOL.1: log10 p0[atm] = B1/T + B2 + B3 T + B4 ln T; with Raoult's law over a fixed
  absorbing amount n_abs = m / MW_abs, G_eq = (A / n_abs) p0 101325 / (R T), so
  k_evap = k_c p0 101325 / (R T n_abs). With the full Raoult mole fraction (p[4] != 0) the
  amount absorbing is n_abs plus every condensed species of the instance: the evaporation
  rate is k_c p0 101325 / (R T) A / n_tot, its rate constant k_c p0 101325 / (R T), and the
  instance's absorber amount n_abs is carried by a reaction-less entry.
* Troe fall-off: k = k0[M] / (1 + k0[M]/kinf) Fc^E with E = 1 / (1 + (1/N) log10(k0[M]/kinf)^2);
  CustomH2o2: k = k1 + k2[M]; CustomOhHno3: k = k0 + k3[M] / (1 + k3[M]/k2); every k_i of
  the Arrhenius form with D = 300 K and E = 0, [M] the number density of air (molecule
  cm^-3, ideal gas). WennbergTunneling: k = A exp(-B/T) exp(C/T^3). All in molecule cm^-3
  units, converted as the Arrhenius form.
* AqueousReversible: K_eq = A exp(C (1/T - 1/298)); reverse rate constant k_r, forward
  K_eq k_r; both act on molarities like an aqueous CondensedPhaseArrhenius rate, so in air
  units k (1000 V)^(1 - n) with n the reactant count of that direction.
* A phase whose radius follows the state keeps the environment's radius r0 and mass m0 as
  the particle core: number concentration N_p = m0 / (rho 4/3 pi r0^3) and core volume
  V0 = m0 / rho (reaction-less entries), and the gas species' mean free path
  lambda = 3 D_g / c_bar; the transfer rate constants are those at r0, rescaled at every
  evaluation by the radius Parameter (forcing).
* An instance with zero phase mass has no particles and no phase volume: every rate
  constant of that instance is 0 (the limit 0 * (1/0) is taken as 0).
"""
import math

import numpy as np

from .expand import (K_ARRHENIUS, K_PHOTOLYSIS, K_EMISSION, K_LOSS, K_CONDENSED,
                     K_HENRY_COND, K_HENRY_EVAP, K_SIMPOL_COND, K_SIMPOL_EVAP,
                     K_TROE, K_H2O2, K_OHHNO3, K_TUNNEL, K_AQREV_FWD, K_AQREV_REV,
                     K_SIMPOL_EVAP_RAOULT, K_ABSORBER, K_NUMBER, K_CORE_VOLUME, K_MEAN_PATH)

AVOGADRO = 6.02214076e23          # mol^-1
BOLTZMANN = 1.380649e-23          # J K^-1
GAS_CONSTANT = 8.314462618        # J mol^-1 K^-1
ATM_PA = 101325.0                 # Pa atm^-1
MOLEC_CM3_PER_MOL_M3 = AVOGADRO * 1.0e-6


def arrhenius(A, Ea_K, B, D, E, T, P):
    """Arrhenius-like rate constant in the paper's units (Table of Process classes)."""
    k = A * math.exp(-Ea_K / T)
    if B != 0.0:
        k *= (T / D) ** B
    if E != 0.0:
        k *= 1.0 + E * P
    return k


def air_number_density(T, P):
    """[M]: molecules per cm^3 of an ideal gas at T (K), P (Pa)."""
    return P / (BOLTZMANN * T) * 1.0e-6


def arrhenius_300(A, Ea_K, B, T):
    """The Arrhenius form with D = 300 K and E = 0."""
    return arrhenius(A, Ea_K, B, 300.0, 0.0, T, 0.0)


def troe(p, T, P):
    """Troe fall-off rate constant; p = [A0, Ea0, B0, Ainf, Eainf, Binf, Fc, N]."""
    k0m = arrhenius_300(p[0], p[1], p[2], T) * air_number_density(T, P)
    kinf = arrhenius_300(p[3], p[4], p[5], T)
    if k0m == 0.0:
        return 0.0
    x = math.log10(k0m / kinf)
    return k0m / (1.0 + k0m / kinf) * p[6] ** (1.0 / (1.0 + x * x / p[7]))


def custom_h2o2(p, T, P):
    """k1 + k2 [M]; p = [A1, Ea1, B1, A2, Ea2, B2]."""
    return arrhenius_300(p[0], p[1], p[2], T) + arrhenius_300(p[3], p[4], p[5], T) * air_number_density(T, P)


def custom_oh_hno3(p, T, P):
    """k0 + k3[M] / (1 + k3[M]/k2); p = [A0, Ea0, B0, A2, Ea2, B2, A3, Ea3, B3]."""
    k3m = arrhenius_300(p[6], p[7], p[8], T) * air_number_density(T, P)
    return arrhenius_300(p[0], p[1], p[2], T) + k3m / (1.0 + k3m / arrhenius_300(p[3], p[4], p[5], T))


def tunneling(p, T):
    """A exp(-B/T) exp(C/T^3)."""
    return p[0] * math.exp(-p[1] / T) * math.exp(p[2] / T ** 3)


def equilibrium_constant(A, C, T):
    """K_eq(T) = A exp(C (1/T - 1/298))."""
    return A * math.exp(C * (1.0 / T - 1.0 / 298.0))


def fuchs_sutugin(Kn, alpha):
    """Fuchs-Sutugin transition-regime correction (HenrysLawPhaseTransfer)."""
    return 0.75 * alpha * (1.0 + Kn) / (Kn * Kn + Kn + 0.283 * Kn * alpha + 0.75 * alpha)


def mean_free_path(T, diff, mw):
    """lambda = 3 D_g / c_bar with the mean molecular speed c_bar = sqrt(8 R T / (pi MW))."""
    return 3.0 * diff / math.sqrt(8.0 * GAS_CONSTANT * T / (math.pi * mw))


def condensation_rate(T, radius, number_conc, diff, mw, alpha):
    """First-order condensation rate constant k_c N (s^-1) onto one phase instance."""
    lam = mean_free_path(T, diff, mw)
    Kn = lam / radius
    return 4.0 * math.pi * radius * diff * fuchs_sutugin(Kn, alpha) * number_conc


def henry_constant(H298, C, T):
    """H(T) = H(298 K) exp(C (1/T - 1/298)) in M Pa^-1."""
    return H298 * math.exp(C * (1.0 / T - 1.0 / 298.0))


def simpol_p0_atm(B1, B2, B3, B4, T):
    """SIMPOL.1 pure-component vapour pressure (atm)."""
    return 10.0 ** (B1 / T + B2 + B3 * T + B4 * math.log(T))


def rate_constants_cell(mech, x, T, P, cos_sza, radius, mass, override=None):
    """Rate constant of every expanded reaction for one cell (1-D array, length R)."""
    k = np.zeros(len(x.rxns))
    for n, xr in enumerate(x.rxns):
        r = mech.reactions[xr.src]
        p = r.p
        if xr.kind == K_ARRHENIUS:
            nr = len(xr.react)
            k[n] = arrhenius(p[0], p[1], p[2], p[3], p[4], T, P) * MOLEC_CM3_PER_MOL_M3 ** (nr - 1)
        elif xr.kind in (K_TROE, K_H2O2, K_OHHNO3, K_TUNNEL):
            f = {K_TROE: lambda: troe(p, T, P), K_H2O2: lambda: custom_h2o2(p, T, P),
                 K_OHHNO3: lambda: custom_oh_hno3(p, T, P), K_TUNNEL: lambda: tunneling(p, T)}
            k[n] = f[xr.kind]() * MOLEC_CM3_PER_MOL_M3 ** (len(xr.react) - 1)
        elif xr.kind in (K_PHOTOLYSIS, K_EMISSION, K_LOSS):
            if override is not None:
                k[n] = override[xr.ext]
            elif xr.kind == K_PHOTOLYSIS and p[1] != 0.0:
                k[n] = p[0] * max(0.0, cos_sza)
            else:
                k[n] = p[0]
        else:
            g = xr.inst
            ph = mech.phases[x.inst_phase[g]]
            m = mass[g]
            if m == 0.0:
                k[n] = 0.0
                continue
            rad = radius[g]
            volume = m / ph.density
            if xr.kind == K_ABSORBER:
                k[n] = m / ph.mw_absorber
                continue
            if xr.kind == K_NUMBER:
                k[n] = m / (ph.density * (4.0 / 3.0) * math.pi * rad ** 3)
                continue
            if xr.kind == K_CORE_VOLUME:
                k[n] = volume
                continue
            if xr.kind == K_MEAN_PATH:
                gas_sp = mech.species[r.react[0]]
                k[n] = mean_free_path(T, gas_sp.diff, gas_sp.mw)
                continue
            if xr.kind in (K_AQREV_FWD, K_AQREV_REV):
                kk = p[2]
                if xr.kind == K_AQREV_FWD:
                    kk *= equilibrium_constant(p[0], p[1], T)
                k[n] = kk * (1000.0 * volume) ** (1 - len(xr.react))
                continue
            if xr.kind == K_CONDENSED:
                kk = arrhenius(p[0], p[1], p[2], p[3], p[4], T, P)
                if p[5] != 0.0:
                    kk *= (1000.0 * volume) ** (1 - len(xr.react))
                k[n] = kk
                continue
            gas_sp = mech.species[r.react[0]]
            number_conc = m / (ph.density * (4.0 / 3.0) * math.pi * rad ** 3)
            kc = condensation_rate(T, rad, number_conc, gas_sp.diff, gas_sp.mw, gas_sp.accom)
            if xr.kind in (K_HENRY_COND, K_SIMPOL_COND):
                k[n] = kc
            elif xr.kind == K_HENRY_EVAP:
                H = henry_constant(p[0], p[1], T)
                k[n] = kc / (H * 1000.0 * volume * GAS_CONSTANT * T)
            elif xr.kind == K_SIMPOL_EVAP:
                n_abs = m / ph.mw_absorber
                p0 = simpol_p0_atm(p[0], p[1], p[2], p[3], T)
                k[n] = kc * p0 * ATM_PA / (GAS_CONSTANT * T * n_abs)
            elif xr.kind == K_SIMPOL_EVAP_RAOULT:
                p0 = simpol_p0_atm(p[0], p[1], p[2], p[3], T)
                k[n] = kc * p0 * ATM_PA / (GAS_CONSTANT * T)
            else:
                raise ValueError(xr.kind)
    return k


def rate_constants(mech, x, env, cells=None):
    """[C, R] rate constants for the requested cells (all cells if None)."""
    idx = range(env.n_cells) if cells is None else cells
    out = []
    for c in idx:
        ov = None if env.rate_override is None else env.rate_override[c]
        out.append(rate_constants_cell(mech, x, float(env.T[c]), float(env.P[c]),
                                       float(env.cos_sza[c]), env.radius[c], env.mass[c], ov))
    return np.asarray(out)
