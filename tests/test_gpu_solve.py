"""End-to-end parity of every engine against the oracle (forcing, Jacobian, LU, solves, BDF
control and the fused kernels), through the C ABI.

Gate: with the GPU at rtol 1e-8 / atol 1e-18
and the oracle at rtol 1e-10 / atol 1e-20, every species with |y_ref| >= 1e-12 mol m^-3
agrees to 1e-4 relative and every species below that floor to 1e-12 absolute.
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.solve import oracle_solve
from tests import mechs
from tests.gpu_util import assert_parity, log, require_gpu

pytestmark = pytest.mark.gpu

GPU_RTOL, GPU_ATOL = 1e-8, 1e-18
OR_RTOL, OR_ATOL = 1e-10, 1e-20
ENGINES = ["wave", "lane", "plain"]


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def gpu_solve(m, wl, engine, rtol=GPU_RTOL, atol=GPU_ATOL, calls=None, **kw):
    from paper_2111_07436_amd import camp
    import torch
    denv = camp.DeviceEnv(wl.env)
    y = torch.from_numpy(wl.y0.copy()).cuda()
    status = torch.empty(wl.n_cells, dtype=torch.int32, device="cuda")
    opts = camp.make_opts(engine=engine, max_steps=kw.pop("max_steps", 20000), **kw)
    for _ in range(wl.n_calls if calls is None else calls):
        m.solve_device(denv, y, wl.dt, rtol, atol, opts, d_status=status)
        torch.cuda.synchronize()
        assert int((status != 0).sum()) == 0, status.cpu().numpy()
    return y.cpu().numpy()


@pytest.mark.parametrize("engine", ENGINES)
def test_c1_all_cells_60_calls(torch, engine):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c1")                       # 100 cells: one full wave + a ragged tail
    m = camp.Mech(wl.mech)
    log(f"c1 engine {engine}: {wl.n_cells} cells x {wl.n_calls} calls of {wl.dt} s")
    y = gpu_solve(m, wl, engine)
    sample = list(range(0, 100, 9)) + [99]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(y[sample], yr, what=f"c1/{engine}")


@pytest.mark.parametrize("engine", ENGINES)
def test_c3_multiphase_sample(torch, engine):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c3", n_cells=70)
    m = camp.Mech(wl.mech)
    log(f"c3 engine {engine}: {wl.n_cells} cells, dt {wl.dt}")
    y = gpu_solve(m, wl, engine)
    zero = np.all(wl.env.mass == 0.0, axis=1)
    sample = [int(np.nonzero(zero)[0][0]), int(np.nonzero(~zero)[0][0]), int(np.nonzero(~zero)[0][1]), 69]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, 1, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(y[sample], yr, what=f"c3/{engine}")
    # zero-aerosol cells keep zero condensed species
    ng = wl.mech.n_gas
    assert np.all(y[zero, ng:] == 0.0)


@pytest.mark.parametrize("engine", ENGINES)
def test_rate_type_zoo(torch, engine):
    """Every process type (Troe, custom H2O2 and OH + HNO3, tunneling, aqueous reversible,
    transfer, condensed-phase, photolysis, emission, loss) in one mechanism."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("zoo", n_cells=100)
    m = camp.Mech(wl.mech)
    log(f"zoo engine {engine}: {wl.n_cells} cells, dt {wl.dt}")
    y = gpu_solve(m, wl, engine)
    zero = np.all(wl.env.mass == 0.0, axis=1)
    sample = [int(np.nonzero(zero)[0][0]), int(np.nonzero(~zero)[0][0]), 50, 99]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, 1, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(y[sample], yr, what=f"zoo/{engine}")


def test_json_and_unpacked_mechanisms_solve_identically(torch):
    """A mechanism read from its JSON description and one unpacked from camp_mech_pack give
    the same states, bit for bit, as the mechanism given as arrays."""
    from paper_2111_07436_amd import camp
    from paper_2111_07436_amd import mechanism_json as MJ
    wl = W.make_workload("zoo", n_cells=100)
    a = camp.Mech(wl.mech)
    ref = gpu_solve(a, wl, "wave")
    for label, m in (("json", camp.Mech.from_json(MJ.to_json(wl.mech))),
                     ("unpacked", camp.Mech.unpack(a.pack()))):
        log(f"zoo {label}")
        assert np.array_equal(gpu_solve(m, wl, "wave"), ref), label


def test_c2_full_size_sampled(torch):
    """All 10,000 cells of the realistic gas config in the benchmark's launch configuration."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c2")
    m = camp.Mech(wl.mech)
    log(f"c2 full: {wl.n_cells} cells, engine auto")
    y = gpu_solve(m, wl, "auto")
    sample = [0, 1, 4999, 9998, 9999]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, 1, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(y[sample], yr, what="c2/full")


def test_engines_agree_and_tiling_invariant(torch):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c2", n_cells=300)
    m = camp.Mech(wl.mech)
    a = gpu_solve(m, wl, "wave", persistent=1, wg_per_cu=1)
    b = gpu_solve(m, wl, "wave", persistent=0)
    c = gpu_solve(m, wl, "wave", persistent=1, wg_per_cu=16)
    assert np.array_equal(a, b) and np.array_equal(a, c)      # no cross-cell arithmetic
    d = gpu_solve(m, wl, "lane")
    e = gpu_solve(m, wl, "plain")
    assert np.array_equal(d, e)                               # same phase functions
    assert_parity(a, d, rel_tol=1e-4, what="wave vs lane")


def test_closed_forms_on_gpu(torch):
    from paper_2111_07436_amd import camp
    import math
    # emission + loss and A -> B -> C in one mechanism, several cells with different rates
    sp = mechs.gas(["E", "A", "B", "C"])
    rx = [W.Reaction(W.RXN_EMISSION, [], [0], [1.0], [4e-12, 0, 0, 0, 0, 0]),
          W.Reaction(W.RXN_FIRST_ORDER_LOSS, [0], [], [], [7e-4, 0, 0, 0, 0, 0]),
          W.Reaction(W.RXN_PHOTOLYSIS, [1], [2], [1.0], [2e-3, 1.0, 0, 0, 0, 0]),
          W.Reaction(W.RXN_PHOTOLYSIS, [2], [3], [1.0], [5e-4, 0, 0, 0, 0, 0])]
    mech = W.Mechanism(sp, [], rx)
    n = 65
    cz = np.linspace(-0.2, 1.0, n)
    env = W.Environment(T=np.full(n, 290.0), P=np.full(n, 1e5), cos_sza=cz,
                        radius=np.zeros((n, 0)), mass=np.zeros((n, 0)))
    y0 = np.tile([3e-9, 1e-8, 3e-9, 0.0], (n, 1))
    wl = W.Workload("closed", mech, env, y0, 3600.0, 1)
    m = camp.Mech(mech)
    for engine in ENGINES:
        y = gpu_solve(m, wl, engine)
        t = 3600.0
        E, kl = 4e-12, 7e-4
        k1 = 2e-3 * np.maximum(cz, 0.0)
        k2 = 5e-4
        yE = E / kl + (3e-9 - E / kl) * math.exp(-kl * t)
        A = 1e-8 * np.exp(-k1 * t)
        # B = B0 e^{-k2 t} + A0 k1 e^{-k2 t} (1 - e^{-(k1-k2) t}) / (k1 - k2), stable near k1 = k2
        dk = k1 - k2
        with np.errstate(divide="ignore", invalid="ignore"):
            frac = np.where(dk == 0.0, t, -np.expm1(-dk * t) / dk)
        B = 3e-9 * math.exp(-k2 * t) + 1e-8 * k1 * math.exp(-k2 * t) * frac
        assert_parity(y[:, 0], np.full(n, yE), what=f"emission/{engine}")
        assert_parity(y[:, 1], A, what=f"A/{engine}")
        assert_parity(y[:, 2], B, what=f"B/{engine}")
        assert np.allclose(y[:, 1:].sum(1), 1.3e-8, rtol=1e-12)


def test_edge_cases(torch):
    from paper_2111_07436_amd import camp
    import torch as T
    wl = W.make_workload("c1", n_cells=3)
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    # zero cells
    y = T.zeros((0, m.n_state), dtype=T.float64, device="cuda")
    st = T.zeros(0, dtype=T.int32, device="cuda")
    m.solve_device(denv, y, 60.0, 1e-4, 1e-12, camp.make_opts("wave"), d_status=st)
    # one cell, each engine, matches the 3-cell run's first row bitwise
    for engine in ENGINES:
        full = gpu_solve(m, wl, engine, calls=1)
        one = gpu_solve(m, wl.take([0]), engine, calls=1)
        assert np.array_equal(full[0], one[0]), engine
    # invalid arguments
    with pytest.raises(camp.CampError):
        m.solve_device(denv, T.from_numpy(wl.y0.copy()).cuda(), -1.0, 1e-4, 1e-12)
    with pytest.raises(camp.CampError):
        m.solve_device(denv, T.from_numpy(wl.y0.copy()).cuda(), 60.0, 0.0, 1e-12)


@pytest.mark.parametrize("engine", ENGINES)
def test_failure_statuses(torch, engine):
    from paper_2111_07436_amd import camp
    import torch as T
    wl = W.make_workload("c1", n_cells=4)
    wl.env.T[2] = np.nan                                  # non-finite rate constants
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    y = T.from_numpy(wl.y0.copy()).cuda()
    st = T.empty(4, dtype=T.int32, device="cuda")
    m.solve_device(denv, y, 60.0, 1e-6, 1e-14, camp.make_opts(engine, max_steps=20000), d_status=st)
    s = st.cpu().numpy()
    out = y.cpu().numpy()
    assert s[2] == 5 and s[0] == 0 and s[1] == 0 and s[3] == 0, s
    assert np.array_equal(out[2], wl.y0[2])               # failed cell keeps its input
    assert camp.count_failed(st) == 1
    # max_steps = 1 -> status 1 everywhere; h_min larger than dt -> status 2
    y = T.from_numpy(wl.y0.copy()).cuda()
    m.solve_device(denv, y, 60.0, 1e-6, 1e-14, camp.make_opts(engine, max_steps=1), d_status=st)
    s = st.cpu().numpy()
    assert s[0] == 1 and s[1] == 1, s
    y = T.from_numpy(wl.y0.copy()).cuda()
    m.solve_device(denv, y, 60.0, 1e-6, 1e-14, camp.make_opts(engine, h_min=100.0), d_status=st)
    s = st.cpu().numpy()
    assert s[0] == 2 and s[1] == 2, s
    assert np.array_equal(y.cpu().numpy()[0], wl.y0[0])


def test_launch_modes_bit_identical(torch):
    """Table staging, rate-constant placement and cells per workgroup change where data
    lives, not the arithmetic: every launch mode gives bit-identical states."""
    from paper_2111_07436_amd import camp
    for name, n, modes in (("c2", 300, (0, 1, 2, 3, 4)), ("c3", 70, (0, 1, 3, 4))):
        wl = W.make_workload(name, n_cells=n)
        m = camp.Mech(wl.mech)
        ref = None
        for mode in modes:
            for waves in ((1, 2, 12) if name == "c2" and mode >= 3 else (1, 2)):
                log(f"{name} mode {mode} waves {waves}")
                y = gpu_solve(m, wl, "wave", stage_tables=mode, waves_per_wg=waves, persistent=1,
                              wg_per_cu=1)
                if ref is None:
                    ref = y
                assert np.array_equal(y, ref), (name, mode, waves)


@pytest.mark.parametrize("lanes", [128, 256])
def test_workgroup_per_cell_parity(torch, lanes):
    """One workgroup of 2 or 4 wavefronts per cell (group-wide reductions and barriers):
    same gate against the oracle, and bit-identical across launch modes."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c3", n_cells=70)
    m = camp.Mech(wl.mech)
    ref = None
    for mode in (0, 1, 3):
        log(f"c3 lanes {lanes} mode {mode}")
        y = gpu_solve(m, wl, "wave", lanes_per_cell=lanes, stage_tables=mode, persistent=1, wg_per_cu=2)
        if ref is None:
            ref = y
        assert np.array_equal(y, ref), mode
    sample = [0, 1, 33, 69]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, 1, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(ref[sample], yr, what=f"c3/lanes {lanes}")
    y = gpu_solve(m, wl, "wave", lanes_per_cell=lanes, persistent=0)
    assert np.array_equal(y, ref)


def test_cell_order_identical(torch):
    """A caller's cell order changes which slot integrates a cell and when, not the
    arithmetic: states are bit-identical to index order for every group size; an order
    that is not a permutation is ignored on the device path; the host-array entry point
    takes a host order and gives the same states."""
    from paper_2111_07436_amd import camp
    for name, n, lanes, mode in (("c2", 500, 64, 3), ("c2", 500, 64, 0), ("c3", 70, 128, 3),
                                 ("c3", 70, 256, 1)):
        wl = W.make_workload(name, n_cells=n)
        m = camp.Mech(wl.mech)
        kw = dict(lanes_per_cell=lanes, stage_tables=mode, persistent=1, wg_per_cu=1)
        log(f"{name} lanes {lanes} mode {mode}: index order")
        ref = gpu_solve(m, wl, "wave", **kw)
        perm = np.random.default_rng(3).permutation(n).astype(np.int32)
        log(f"{name} lanes {lanes} mode {mode}: permuted order")
        d_perm = torch.from_numpy(perm).cuda()
        assert np.array_equal(gpu_solve(m, wl, "wave", cell_order=d_perm, **kw), ref)
        dup = d_perm.clone()
        dup[1] = dup[0]
        log(f"{name} lanes {lanes} mode {mode}: repeated entry (ignored)")
        assert np.array_equal(gpu_solve(m, wl, "wave", cell_order=dup, **kw), ref)
        log(f"{name} lanes {lanes} mode {mode}: host arrays")
        opts = camp.make_opts("wave", max_steps=20000, cell_order=perm, **kw)
        y, st, _ = m.solve(wl.env, wl.y0, wl.dt, GPU_RTOL, GPU_ATOL, opts)
        assert np.all(st == 0) and np.array_equal(y, ref)


def test_slightly_negative_inputs(torch):
    """A previous call's result may undershoot zero by up to a tolerance unit. Such an input
    starts at zero and integrates on every engine; no component ends more than one
    tolerance unit below zero."""
    from paper_2111_07436_amd import camp
    import torch as T
    wl = W.make_workload("c3", n_cells=96)
    rng = np.random.default_rng(11)
    y0 = wl.y0.copy()
    flip = (y0 < 1e-10) & (rng.random(y0.shape) < 0.3)
    assert flip.sum() > 100
    y0[flip] = -0.9e-12
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    for engine, kw in (("wave", {}), ("wave", dict(lanes_per_cell=128)), ("lane", {}),
                       ("plain", {})):
        log(f"negative inputs: {engine} {kw}")
        y = T.from_numpy(y0.copy()).cuda()
        st = T.empty(wl.n_cells, dtype=T.int32, device="cuda")
        m.solve_device(denv, y, wl.dt, 1e-4, 1e-12, camp.make_opts(engine, **kw), d_status=st)
        T.cuda.synchronize()
        s = st.cpu().numpy()
        assert np.all(s == 0), (engine, kw, np.bincount(s))
        out = y.cpu().numpy()
        assert np.all(np.isfinite(out))
        assert np.all(out >= np.minimum(0.0, y0) - 1.0e-12 - 1e-4 * np.abs(out) - 1e-15), (engine, kw)


def test_plain_graph_replay_identical(torch):
    """The plain multi-kernel form replays a captured chunk of step-attempt launches; the
    states equal those of direct launches."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c2", n_cells=200)
    m = camp.Mech(wl.mech)
    a = gpu_solve(m, wl, "plain", use_graph=0)
    b = gpu_solve(m, wl, "plain", use_graph=1)
    c = gpu_solve(m, wl, "plain", use_graph=1)
    assert np.array_equal(a, b) and np.array_equal(b, c)


def test_full_newton_parity(torch):
    """Full Newton from the start (fresh Jacobian and LU every iteration)."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c1")
    m = camp.Mech(wl.mech)
    y = gpu_solve(m, wl, "wave", full_newton=1)
    sample = [0, 37, 99]
    yr, st, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, OR_RTOL, OR_ATOL, cells=sample)
    assert np.all(st == 0)
    assert_parity(y[sample], yr, what="c1/full newton")


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_oracle_reference.py {name})")
    with open(path) as f:
        return json.load(f)


def _stored_sample(g, minimum):
    ok = np.asarray(g["status"]) == 0
    cells = np.asarray(g["cells"])[ok]
    assert ok.sum() >= minimum, g["status"]          # a sample, not an empty check
    return cells, np.asarray(g["y"])[ok]


def test_c3_full_size_against_stored_oracle(torch):
    """All 100,000 cells of the multiphase config in the autotuned launch, sampled cells
    against oracle states written by tests/golden/make_oracle_reference.py."""
    from paper_2111_07436_amd import camp
    g = _golden("c3")
    wl = W.make_workload("c3", n_cells=g["n_cells"])
    assert wl.n_calls == g["n_calls"] and wl.dt == g["dt"]
    m = camp.Mech(wl.mech)
    log(f"c3 full: {wl.n_cells} cells, engine auto")
    y = gpu_solve(m, wl, "auto")
    cells, ref = _stored_sample(g, 6)
    assert_parity(y[cells], ref, what="c3/full vs stored oracle")


@pytest.mark.timeout(900)
def test_c5_full_size_against_stored_oracle(torch):
    """All 500,000 cells of the large config (520 state variables) in the autotuned launch
    the benchmark times, sampled cells (first, last, zero-aerosol, spread) against stored
    oracle states."""
    from paper_2111_07436_amd import camp
    g = _golden("c5")
    wl = W.make_workload("c5", n_cells=g["n_cells"])
    assert wl.n_cells == 500_000 and wl.n_calls == g["n_calls"] and wl.dt == g["dt"]
    assert g["zero_aerosol_cells"] and 499_999 in g["cells"]
    m = camp.Mech(wl.mech)
    log(f"c5 full: {wl.n_cells} cells, engine auto")
    y = gpu_solve(m, wl, "auto")
    cells, ref = _stored_sample(g, 14)
    assert_parity(y[cells], ref, what="c5/full vs stored oracle")


def test_c5_sample_against_stored_oracle(torch):
    """The large mechanism on its stored sample cells alone, for each group size, launch
    mode and the lane engine."""
    from paper_2111_07436_amd import camp
    g = _golden("c5")
    wl = W.make_workload("c5", n_cells=g["n_cells"])
    cells, ref = _stored_sample(g, 14)
    sub = wl.take(cells)
    m = camp.Mech(sub.mech)
    for kw in ({"engine": "wave", "stage_tables": 0}, {"engine": "wave", "stage_tables": 3},
               {"engine": "wave", "stage_tables": 3, "lanes_per_cell": 128},
               {"engine": "wave", "stage_tables": 3, "lanes_per_cell": 256}, {"engine": "lane"}):
        log(f"c5 sample: {len(cells)} cells, {kw}")
        y = gpu_solve(m, sub, **kw)
        assert_parity(y, ref, what=f"c5/{kw}")


def test_peak_probes(torch):
    from paper_2111_07436_amd import camp
    gbs = camp.probe_copy(mib=512, reps=4)
    tf = camp.probe_fma(blocks=1024, iters=2000)
    log(f"copy {gbs:.0f} GB/s, FP64 FMA {tf:.1f} TFLOP/s")
    assert 500.0 < gbs < 8000.0 * 1.05    # below the published HBM peak
    assert 1.0 < tf < 78.6 * 1.05         # below the published FP64 vector peak
