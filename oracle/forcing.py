"""Forcing f(y) and its analytic Jacobian (oracle; test infrastructure only).

The forcing of species i is the sum over processes of each process's contribution, and
the Jacobian entry (i, j) is the sum of the processes' partial derivatives (Sect. 2.4.2,
the two sums over processes k). Every expanded reaction here is generalized mass action:
its rate is r = k * prod_{occurrences o} y_{j_o}; it removes one unit of each reactant
occurrence and adds ``yield`` units of each product. Hence

    f = S r,        S[i, k] = sum(yields of i in k) - (occurrences of i among reactants of k)
    J = S (dr/dy),  dr_k/dy_j = k_k * sum over occurrences o of j of prod_{o' != o} y_{j_o'}

A reaction may also depend on a Parameter (Sect. 2.2.2, a property diagnosed from the
state): the full Raoult evaporation divides its rate by the instance's total condensed
amount p = c + sum_{j in S} y_j, so r = k prod(y) / p, and by the chain rule
dr/dy_j = (d mass-action term / dy_j) / p - r / p for j in S (dp/dy_j = 1). A p of exactly 0
(an instance without absorber or condensed species) gives r = 0.

A transfer into a phase whose particle radius follows the state carries a second
Parameter, the radius r(y) = (3 V(y) / (4 pi N_p))^(1/3) with the particle volume
V(y) = V0 + sum_j w_j y_j (w_j = MW_j / rho). Its rate constant, given at the core radius
r0, is multiplied by psi = r F(lambda / r) / (r0 F(lambda / r0)), the ratio of the
condensation rates 4 pi r D_g F(Kn) N_p at the two radii (F the Fuchs-Sutugin factor).
By the chain rule dr/dy_j gains r (d ln psi / dr) w_j / (4 pi N_p r^2) for j in the set,
with d ln psi / dr = (F(Kn) - Kn F'(Kn)) / (r F(Kn)).

Both are computed densely; the arithmetic works for complex y so that the Jacobian can
be checked by the complex-step derivative.
"""
import numpy as np


def _fs(Kn, alpha):
    """Fuchs-Sutugin factor F(Kn) and its derivative dF/dKn."""
    num = 0.75 * alpha * (1.0 + Kn)
    den = Kn * Kn + Kn + 0.283 * Kn * alpha + 0.75 * alpha
    dden = 2.0 * Kn + 1.0 + 0.283 * alpha
    return num / den, (0.75 * alpha * den - num * dden) / (den * den)


class DenseSystem:
    """Dense S, reactant index table and f/J evaluation for one expanded mechanism."""

    def __init__(self, x):
        n, R = x.n_state, len(x.rxns)
        self.n = n
        S = np.zeros((n, R))
        react = np.full((R, 3), n, dtype=np.int64)   # index n points at a constant 1
        for k, xr in enumerate(x.rxns):
            for o, j in enumerate(xr.react):
                react[k, o] = j
                S[j, k] -= 1.0
            for i, yl in zip(xr.prod, xr.yields):
                S[i, k] += yl
        self.S = S
        self.react = react
        # Jacobian contributions: for reaction k, reactant occurrence o (species j) and every
        # species i with S[i, k] != 0, J[i, j] += S[i, k] * dr_k/dy_j(occurrence o).
        ii, jj, kk, oo, cc = [], [], [], [], []
        for k, xr in enumerate(x.rxns):
            members = np.nonzero(S[:, k])[0]
            for o, j in enumerate(xr.react):
                for i in members:
                    ii.append(i); jj.append(j); kk.append(k); oo.append(o); cc.append(S[i, k])
        self.jc = (np.array(ii, dtype=np.int64), np.array(jj, dtype=np.int64),
                   np.array(kk, dtype=np.int64), np.array(oo, dtype=np.int64), np.array(cc))
        self.params = [(k, xr.param_const, list(xr.param_species), np.nonzero(S[:, k])[0])
                       for k, xr in enumerate(x.rxns) if xr.param_const >= 0]
        self.radius = [(k, xr, np.nonzero(S[:, k])[0])
                       for k, xr in enumerate(x.rxns) if xr.radius_species is not None]

    def radius_terms(self, k, y):
        """Per radius-parameterized reaction: (psi, d ln psi / dy_j over its species)."""
        out = {}
        for kk, xr, _ in self.radius:
            n_p = k[xr.radius_number]
            if n_p == 0:
                out[kk] = (0.0, None)
                continue
            v0, lam, a = k[xr.radius_core], k[xr.radius_path], xr.radius_alpha
            vol = v0 + sum(w * y[j] for j, w in zip(xr.radius_species, xr.radius_weights))
            r = (3.0 * vol / (4.0 * np.pi * n_p)) ** (1.0 / 3.0)
            r0 = (3.0 * v0 / (4.0 * np.pi * n_p)) ** (1.0 / 3.0)
            f, df = _fs(lam / r, a)
            f0, _ = _fs(lam / r0, a)
            psi = r * f / (r0 * f0)
            dlnpsi_dr = (f - (lam / r) * df) / (r * f)
            drdy = np.array(xr.radius_weights) / (4.0 * np.pi * n_p * r * r)
            out[kk] = (psi, dlnpsi_dr * drdy)
        return out

    def factors(self, k, y):
        """Per-reaction parameter factor: 1/p times psi (1 for reactions without one)."""
        phi = np.ones(len(k), dtype=np.result_type(y, k))
        for kk, d, spec, _ in self.params:
            p = k[d] + sum(y[j] for j in spec)
            phi[kk] = 0.0 if p == 0 else 1.0 / p
        for kk, (psi, _) in self.radius_terms(k, y).items():
            phi[kk] = phi[kk] * psi
        return phi

    def rates(self, k, y):
        ye = np.append(y, 1.0)
        g = ye[self.react]                            # [R, 3]
        return k * g[:, 0] * g[:, 1] * g[:, 2] * self.factors(k, y)

    def f(self, k, y):
        return self.S @ self.rates(k, y)

    def jac(self, k, y):
        n = self.n
        ye = np.append(y, 1.0)
        g = ye[self.react]
        # occurrence o: derivative of g0*g1*g2 w.r.t. g_o is the product of the other two
        others = np.stack([g[:, 1] * g[:, 2], g[:, 0] * g[:, 2], g[:, 0] * g[:, 1]], axis=1)
        phi = self.factors(k, y)
        ii, jj, kk, oo, cc = self.jc
        J = np.zeros((n, n), dtype=np.result_type(y, k))
        np.add.at(J, (ii, jj), cc * (k * phi)[kk] * others[kk, oo])
        # chain rule through the parameters: dr/dp dp/dy_j = -r / p for every j in the set of
        # a 1/p factor, and r d ln psi / dy_j for the radius
        if self.params or self.radius:
            r = self.rates(k, y)
            for kk_, d, spec, members in self.params:
                p = k[d] + sum(y[j] for j in spec)
                inv_p = 0.0 if p == 0 else 1.0 / p
                for i in members:
                    for j in spec:
                        J[i, j] += self.S[i, kk_] * (-r[kk_] * inv_p)
            rt = self.radius_terms(k, y)
            for kk_, xr, members in self.radius:
                psi, dln = rt[kk_]
                if dln is None:
                    continue
                for i in members:
                    for j, g in zip(xr.radius_species, dln):
                        J[i, j] += self.S[i, kk_] * r[kk_] * g
        return J
