"""Generator: determinism, config sizes, conservation weights (CPU)."""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.expand import expand


def test_determinism():
    a = W.make_workload("c1")
    b = W.make_workload("c1")
    assert np.array_equal(a.y0, b.y0)
    assert np.array_equal(a.env.T, b.env.T)
    assert [r.p for r in a.mech.reactions] == [r.p for r in b.mech.reactions]
    c = W.make_workload("c1", seed=1)
    assert not np.array_equal(a.y0, c.y0)


@pytest.mark.parametrize("name,N,R", [("c1", 20, 40), ("c2", 72, 233), ("c3", 192, 809), ("c5", 520, 1720)])
def test_config_sizes(name, N, R):
    m = W.make_mechanism(name)
    x = expand(m)
    assert m.n_state == N == x.n_state
    assert len(x.rxns) == R


def test_c3_zero_aerosol_fraction_and_layout():
    wl = W.make_workload("c3", n_cells=2000)
    zero = np.all(wl.env.mass == 0.0, axis=1)
    assert 0.25 < zero.mean() < 0.35
    ng = wl.mech.n_gas
    assert np.all(wl.y0[zero, ng:] == 0.0)
    assert np.all(wl.y0[~zero, ng:] > 0.0)
    # interleaved, not blocked: zero-aerosol cells appear in every group of 64
    groups = zero[: (len(zero) // 64) * 64].reshape(-1, 64)
    assert np.all(groups.any(axis=1))


def test_request_trace():
    arr, cells, mid = W.make_request_trace(2000)
    assert np.all(np.diff(arr) > 0)
    assert 1000 <= cells.min() and cells.max() <= 200_000
    rate = len(arr) / arr[-1]
    assert 170 < rate < 230
    assert set(np.unique(mid)) == {0, 1}
