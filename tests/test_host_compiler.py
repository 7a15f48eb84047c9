"""Host mechanism compiler through the C ABI, checked against the oracle (CPU).

The C++ compiler's expansion, Jacobian pattern and symbolic LU fill must equal the
oracle's brute-force constructions bit for bit (integer work).
"""
import re

import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.expand import expand
from oracle.sparse import structural_pattern, symbolic_fill
from tests import mechs

camp = pytest.importorskip("paper_2111_07436_amd.camp", reason="libcamp.so not built")


def test_library_exports_every_declared_symbol():
    import ctypes
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "camp.h")).read()
    declared = set(re.findall(r"^(?:int|void|size_t|const char\*)\s+(camp_[a-z_]+)\s*\(", hdr, re.M))
    lib = ctypes.CDLL(camp.LIB_PATH)
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert declared == set(camp.EXPORTED)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5", "zoo"])
def test_expansion_pattern_and_fill_match_oracle(name):
    mech = W.make_mechanism(name)
    m = camp.Mech(mech)
    x = expand(mech)
    assert m.info["n_state"] == x.n_state
    assert m.info["n_rxn_expanded"] == len(x.rxns)
    assert m.info["n_external"] == mech.n_external
    perm, rp, col, p0 = m.export()
    n = x.n_state
    assert sorted(perm) == list(range(n))
    P = structural_pattern(x)
    F = symbolic_fill(P, perm) if n <= 200 else None
    dense = np.zeros((n, n), dtype=bool)
    dense0 = np.zeros((n, n), dtype=bool)
    for i in range(n):
        cols = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        dense[i, cols] = True
        dense0[i, cols] = p0[rp[i]:rp[i + 1]] == 1
    assert np.array_equal(dense0, P[np.ix_(perm, perm)])
    # the stored pattern is the symbolic fill plus a fully stored trailing block
    K = m.info["tail_k"]
    tail = np.zeros((n, n), dtype=bool)
    tail[n - K:, n - K:] = True
    assert np.all(dense[tail])
    if F is not None:
        assert np.array_equal(dense, F | tail)
    assert m.info["nnz_pattern"] == P.sum()
    assert m.info["nnz_fill"] == dense.sum()


def test_c5_fill_size_is_the_configs():
    m = camp.Mech(W.make_mechanism("c5"))
    assert 5400 <= m.info["nnz_fill"] <= 6600    # "Jacobian nnz ~ 6,000 per cell after fill"


def test_fill_c5_matches_bruteforce_numeric():
    # c5 is too large for the pure-python boolean elimination in reasonable time: check the
    # filled pattern against the nonzeros of a numeric no-pivot LU of random values instead.
    from oracle.sparse import lu_nopivot
    mech = W.make_mechanism("c5")
    m = camp.Mech(mech)
    x = expand(mech)
    perm, rp, col, p0 = m.export()
    n = x.n_state
    P = structural_pattern(x)[np.ix_(perm, perm)]
    rng = np.random.Generator(np.random.PCG64(5))
    M = np.where(P, rng.uniform(0.1, 1.0, (n, n)), 0.0) + np.eye(n) * n
    LU = lu_nopivot(M)
    dense = np.zeros((n, n), dtype=bool)
    for i in range(n):
        dense[i, col[rp[i]:rp[i + 1]]] = True
    K = m.info["tail_k"]
    tail = np.zeros((n, n), dtype=bool)
    tail[n - K:, n - K:] = True
    assert np.array_equal((LU != 0.0) | tail, dense)


def _expect_einval(mech):
    with pytest.raises(camp.CampError) as e:
        camp.Mech(mech)
    assert e.value.code == camp.EINVAL


def test_validation_errors():
    g = mechs.gas(["A", "B"])
    _expect_einval(W.Mechanism(g, [], [mechs.arrhenius_rxn([0, 5], [1], [1.0], 1e-12)]))
    _expect_einval(W.Mechanism(g, [], [mechs.arrhenius_rxn([0], [1], [1.0], -1.0)]))
    _expect_einval(W.Mechanism(g, [], [mechs.arrhenius_rxn([0], [1], [1.0], float("nan"))]))
    _expect_einval(W.Mechanism(g, [], [W.Reaction(W.RXN_EMISSION, [0], [1], [1.0], [1e-12, 0, 0, 0, 0, 0])]))
    # transfer whose gas partner is condensed
    sp = [W.Species("G", -1), W.Species("A", 0), W.Species("B", 0)]
    ph = [W.Phase("p", [1, 2], 2)]
    _expect_einval(W.Mechanism(sp, ph, [W.Reaction(W.RXN_HENRY_TRANSFER, [1], [2], [1.0],
                                                   [1.0, 0, 0, 0, 0, 0], phase=0)]))
    # phase without instances / species
    _expect_einval(W.Mechanism(sp, [W.Phase("p", [1, 2], 0)], []))
    _expect_einval(W.Mechanism(sp[:1], [W.Phase("p", [], 1)], []))
    # a phase whose radius follows the state: no Henry transfer, species need a molecular weight
    grow = [W.Phase("p", [1, 2], 2, radius_from_state=True)]
    _expect_einval(W.Mechanism(sp, grow, [W.Reaction(W.RXN_HENRY_TRANSFER, [0], [1], [1.0],
                                                     [1.0, 0, 0, 0, 0, 0], phase=0)]))
    simpol = W.Reaction(W.RXN_SIMPOL_TRANSFER, [0], [1], [1.0], [3000.0, -20.0, 0, 0, 1.0, 0], phase=0)
    sp0 = [W.Species("G", -1), W.Species("A", 0), W.Species("B", 0, mw=0.0)]
    _expect_einval(W.Mechanism(sp0, grow, [simpol]))
    camp.Mech(W.Mechanism(sp, grow, [simpol]))   # accepted with molecular weights
    # the full-Raoult flag is 0 or 1
    bad_flag = W.Reaction(W.RXN_SIMPOL_TRANSFER, [0], [1], [1.0], [3000.0, -20.0, 0, 0, 0.5, 0], phase=0)
    _expect_einval(W.Mechanism(sp, [W.Phase("p", [1, 2], 2)], [bad_flag]))


def test_cell_order_must_be_a_permutation():
    """camp_solve checks a host cell order before any device work."""
    wl = W.make_workload("c1", n_cells=8)
    m = camp.Mech(wl.mech)
    for bad in ([0, 1, 2, 3, 4, 5, 6, 6], [0, 1, 2, 3, 4, 5, 6, 8], [-1, 1, 2, 3, 4, 5, 6, 7]):
        opts = camp.make_opts("wave", cell_order=np.asarray(bad, dtype=np.int32))
        with pytest.raises(camp.CampError) as e:
            m.solve(wl.env, wl.y0, wl.dt, 1e-4, 1e-12, opts)
        assert e.value.code == camp.EINVAL
        assert "cell_order" in str(e.value)
    with pytest.raises(ValueError):
        camp.make_opts("wave", cell_order=np.arange(8, dtype=np.int64))


def test_schedule_counts_consistent():
    m = camp.Mech(W.make_mechanism("c2"))
    inf = m.info
    assert inf["lu_pairs"] > 0 and inf["lu_levels"] > 0
    assert inf["fwd_levels"] > 0 and inf["bwd_levels"] > 0
    assert inf["n_partials"] >= 0 and inf["n_terms"] > 0 and inf["n_jac_contrib"] > 0


def test_probes_reject_bad_arguments():
    """The measurement probes validate their arguments before any device call."""
    import ctypes
    v = ctypes.c_double(0)
    lib = camp._lib
    assert lib.camp_probe_copy(None, None, 1024, 1, None, ctypes.byref(v)) == camp.EINVAL
    buf = (ctypes.c_double * 4)()
    assert lib.camp_probe_copy(buf, buf, 3, 1, None, ctypes.byref(v)) == camp.EINVAL   # odd n
    assert lib.camp_probe_copy(buf, buf, 4, 0, None, ctypes.byref(v)) == camp.EINVAL   # no reps
    assert lib.camp_probe_fma(None, 1, 1, None, ctypes.byref(v)) == camp.EINVAL
    assert lib.camp_probe_fma(buf, 0, 1, None, ctypes.byref(v)) == camp.EINVAL
