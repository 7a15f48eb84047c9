"""Pins of the oracle's symbolic fill and no-pivot LU (CPU)."""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.expand import expand
from oracle.sparse import lu_nopivot, lu_solve_nopivot, structural_pattern, symbolic_fill


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fill_matches_numeric_lu_nonzeros(name, rng):
    # Generic random values on the pattern: the numeric LU's nonzeros are exactly the
    # symbolic fill (no accidental cancellation for random reals).
    x = expand(W.make_mechanism(name))
    P = structural_pattern(x)
    order = rng.permutation(x.n_state)
    F = symbolic_fill(P, order)
    n = x.n_state
    M = np.where(P, rng.uniform(0.1, 1.0, (n, n)), 0.0) + np.eye(n) * n
    LU = lu_nopivot(M[np.ix_(order, order)])
    assert np.array_equal(LU != 0.0, F)


def test_fill_example_arrow():
    # arrow matrix: eliminating the hub first fills everything, last fills nothing
    n = 5
    P = np.eye(n, dtype=bool)
    P[0, :] = P[:, 0] = True
    assert symbolic_fill(P, np.arange(n)).all()
    F = symbolic_fill(P, np.array([1, 2, 3, 4, 0]))
    assert F.sum() == P.sum()


def test_lu_nopivot_solves(rng):
    n = 30
    M = rng.normal(size=(n, n)) + n * np.eye(n)
    b = rng.normal(size=n)
    LU = lu_nopivot(M)
    x = lu_solve_nopivot(LU, b)
    assert np.allclose(x, np.linalg.solve(M, b), rtol=1e-12)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    assert np.allclose(L @ U, M, rtol=1e-13, atol=1e-12)


def test_pattern_contains_jacobian_nonzeros(rng):
    from oracle.forcing import DenseSystem
    from oracle.rates import rate_constants
    wl = W.make_workload("c3", n_cells=2)
    x = expand(wl.mech)
    P = structural_pattern(x)
    s = DenseSystem(x)
    k = rate_constants(wl.mech, x, wl.env)
    J = s.jac(k[0], wl.y0[0])
    assert not np.any((J != 0) & ~P)
