"""The fused kernel's factor-and-solve table program, run on the host (CPU).

camp_emulate_factor_solve executes the level-scheduled term lists a layout holds (Crout
levels, pivot finalization, U row scaling, the dense tail's Gauss-Jordan inversion of its
Schur complement, forward sweep, product with the inverse, diagonal step, backward sweep)
in order on one matrix. The result must solve the linear system to roundoff: compared with
numpy's dense LU solve of the same matrix (a library routine, independent of both the
compiler and the oracle).
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W

camp = pytest.importorskip("paper_2111_07436_amd.camp", reason="libcamp.so not built")

LAYOUTS = [(64, False), (64, True), (128, True), (256, True)]


def random_system(m, rng, dominance=1.0):
    """Values on the unfilled pattern (fill slots 0), diagonally dominant; dense copy in
    elimination order."""
    perm, rp, col, p0 = m.export()
    n, z = m.n_state, m.nnz
    vals = np.where(p0 == 1, rng.uniform(-1.0, 1.0, z), 0.0)
    A = np.zeros((n, n))
    for i in range(n):
        q = slice(rp[i], rp[i + 1])
        d = rp[i] + int(np.nonzero(col[q] == i)[0][0])
        vals[d] = 0.0
        vals[d] = np.abs(vals[q]).sum() + dominance
        A[i, col[q]] = vals[q]
    return vals, A


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5", "zoo"])
def test_table_program_solves_the_system(name, rng):
    m = camp.Mech(W.make_mechanism(name))
    vals, A = random_system(m, rng)
    b = rng.normal(size=m.n_state)
    x_ref = np.linalg.solve(A, b)
    for lanes, tail in LAYOUTS:
        _, x = m.emulate_factor_solve(vals, b, lanes, tail)
        err = np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref))
        assert err < 1e-13, (name, lanes, tail, err)


def test_dense_tail_cuts_the_dependency_levels():
    # C5: the trailing rows form a chain of one-row sweep levels; the inverse of their
    # Schur complement replaces it by one product level
    m = camp.Mech(W.make_mechanism("c5"))
    plain = m.info["fwd_levels"] + m.info["bwd_levels"]
    lay = m.layout_info(256)
    assert lay["tail_k"] >= 16
    assert lay["fwd_levels"] + lay["bwd_levels"] + 1 < plain / 2


def test_tail_factors_hold_the_schur_complement_inverse(rng):
    m = camp.Mech(W.make_mechanism("c2"))
    vals, A = random_system(m, rng)
    perm, rp, col, _ = m.export()
    n = m.n_state
    K = m.layout_info(64)["tail_k"]
    assert K > 0
    f, _ = m.emulate_factor_solve(vals, np.zeros(n), 64, True)
    s = n - K
    S = A[s:, s:] - A[s:, :s] @ np.linalg.solve(A[:s, :s], A[:s, s:])
    got = np.zeros((K, K))
    for i in range(s, n):
        for q in range(rp[i], rp[i + 1]):
            if col[q] >= s:
                got[i - s, col[q] - s] = f[q]
    assert np.allclose(got, np.linalg.inv(S), rtol=1e-11, atol=1e-14)


def test_zero_pivot_is_reported(rng):
    m = camp.Mech(W.make_mechanism("c1"))
    vals, _ = random_system(m, rng)
    perm, rp, col, _ = m.export()
    n = m.n_state
    # zero row and column of the last position: the tail's last Gauss-Jordan pivot is 0
    last = n - 1
    for i in range(n):
        for q in range(rp[i], rp[i + 1]):
            if i == last or col[q] == last:
                vals[q] = 0.0
    with pytest.raises(camp.CampError) as e:
        m.emulate_factor_solve(vals, np.ones(n), 64, True)
    assert e.value.code == camp.ESOLVE
