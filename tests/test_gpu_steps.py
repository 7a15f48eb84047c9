"""Kernel-level parity of the hot-path steps (rate constants, forcing, Newton matrix, LU,
triangular solves) against the oracle, through the C ABI.

Each step runs the fused engine's device code on row-major inputs; the oracle computes the
same quantity densely in FP64. Bars: rate constants and forcing to a few ulps of their
magnitude; the Newton matrix to ulps of its contribution sum; LU and solves by the
residual against the dense matrix.
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.expand import expand
from oracle.forcing import DenseSystem
from oracle.rates import rate_constants
from oracle.sparse import lu_nopivot
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module", params=["c1", "c2", "c3", "c5", "zoo"])
def setup(request, torch):
    from paper_2111_07436_amd import camp
    name = request.param
    n = {"c1": 100, "c2": 130, "c3": 130, "c5": 70, "zoo": 100}[name]   # ragged: not multiples of 64
    wl = W.make_workload(name, n_cells=n)
    m = camp.Mech(wl.mech)
    x = expand(wl.mech)
    log(f"setup {name}: cells {n}, info {m.info}")
    return name, wl, m, x


def _abs_jac(s, k, y):
    # sum of |contributions| per Jacobian entry (the rounding scale of the assembly)
    ye = np.append(y, 1.0)
    g = ye[s.react]
    others = np.stack([g[:, 1] * g[:, 2], g[:, 0] * g[:, 2], g[:, 0] * g[:, 1]], axis=1)
    ii, jj, kk, oo, cc = s.jc
    J = np.zeros((s.n, s.n))
    np.add.at(J, (ii, jj), np.abs(cc * k[kk] * others[kk, oo]))
    return J


def _dense_from_slots(m, vals):
    perm, rp, col, p0 = m.export()
    n = len(perm)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    return A


def test_rate_constants(setup, torch):
    from paper_2111_07436_amd import camp
    name, wl, m, x = setup
    denv = camp.DeviceEnv(wl.env)
    k = m.rate_constants(denv, wl.n_cells).cpu().numpy()
    kref = rate_constants(wl.mech, x, wl.env)
    assert np.array_equal(k == 0.0, kref == 0.0)
    nz = kref != 0.0
    rel = np.abs(k[nz] - kref[nz]) / np.abs(kref[nz])
    log(f"{name} rate constants: max rel {rel.max():.2e}")
    assert rel.max() <= 1e-13


def test_forcing(setup, torch):
    name, wl, m, x = setup
    s = DenseSystem(x)
    kref = rate_constants(wl.mech, x, wl.env)
    rng = np.random.Generator(np.random.PCG64(3))
    y = wl.y0 * rng.uniform(0.5, 1.5, wl.y0.shape)
    f = m.forcing(torch.from_numpy(kref).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
    worst = 0.0
    for c in range(wl.n_cells):
        fr = s.f(kref[c], y[c])
        scale = np.abs(s.S) @ np.abs(s.rates(kref[c], y[c]))
        err = np.abs(f[c] - fr)
        assert np.all(err <= 1e-14 * scale + 1e-300), name
        worst = max(worst, float(np.max(err / np.maximum(scale, 1e-300))))
    log(f"{name} forcing: max err / scale {worst:.2e}")


def test_newton_matrix(setup, torch):
    name, wl, m, x = setup
    s = DenseSystem(x)
    kref = rate_constants(wl.mech, x, wl.env)
    perm, rp, col, p0 = m.export()
    gamma = 37.5
    M = m.newton_matrix(torch.from_numpy(kref).cuda(), torch.from_numpy(wl.y0).cuda(), gamma).cpu().numpy()
    for c in range(0, wl.n_cells, 7):
        J = s.jac(kref[c], wl.y0[c])[np.ix_(perm, perm)]
        ref = np.eye(len(perm)) - gamma * J
        A = _dense_from_slots(m, M[c])
        err = np.abs(A - ref)
        scale = np.abs(ref) + gamma * _abs_jac(s, kref[c], wl.y0[c])[np.ix_(perm, perm)] + 1e-300
        assert np.all(err <= 1e-13 * scale), name
        # nothing outside the pattern
        mask = np.zeros_like(A, dtype=bool)
        for i in range(len(perm)):
            mask[i, col[rp[i]:rp[i + 1]]] = True
        assert np.all(ref[~mask] == 0.0)
    log(f"{name} newton matrix: ok")


def test_lu_and_solve(setup, torch):
    name, wl, m, x = setup
    s = DenseSystem(x)
    kref = rate_constants(wl.mech, x, wl.env)
    perm, rp, col, p0 = m.export()
    n = len(perm)
    gamma = 12.0
    Md = m.newton_matrix(torch.from_numpy(kref).cuda(), torch.from_numpy(wl.y0).cuda(), gamma)
    M0 = Md.cpu().numpy().copy()
    LU = m.lu_factor(Md)
    rng = np.random.Generator(np.random.PCG64(9))
    b = rng.normal(size=(wl.n_cells, n))
    xg = m.lu_solve(LU, torch.from_numpy(b.copy()).cuda()).cpu().numpy()
    LUh = LU.cpu().numpy()
    worst_lu, worst_res = 0.0, 0.0
    for c in range(0, wl.n_cells, 5):
        A = _dense_from_slots(m, M0[c])                       # permuted space
        got = _dense_from_slots(m, LUh[c])
        L = np.tril(got, -1) + np.eye(n)
        U = np.triu(got)
        # backward error of the factorization: |L U - A| <= c u |L| |U| (no pivoting)
        scale = np.abs(L) @ np.abs(U) + 1e-300
        e_lu = np.max(np.abs(L @ U - A) / scale)
        worst_lu = max(worst_lu, e_lu)
        # same fill as the oracle's dense no-pivot LU (structural zeros stay zero)
        ref = lu_nopivot(A)
        assert np.all(got[ref == 0.0] == 0.0)
        # solve: x is in user state order; A is in elimination order
        Au = np.zeros_like(A)
        Au[np.ix_(perm, perm)] = A
        res = Au @ xg[c] - b[c]
        rel_res = np.linalg.norm(res) / (np.linalg.norm(Au) * np.linalg.norm(xg[c]) + np.linalg.norm(b[c]))
        worst_res = max(worst_res, rel_res)
    log(f"{name} LU: max err/scale {worst_lu:.2e}; solve: max rel residual {worst_res:.2e}")
    assert worst_lu <= 1e-13
    assert worst_res <= 1e-13
