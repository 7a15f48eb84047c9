"""Plans: one solve captured as a HIP graph and replayed (through the C ABI).

Every replay is checked against the direct solve of the same input, bit for bit (the same
kernels in the same launch shape), with the program's own eager work (state reset, status
reads) and synchronizations between replays; one replay is also checked against the oracle.
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from oracle.solve import oracle_solve
from tests.gpu_util import assert_parity, log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("name,n,kw", [
    ("c2", 300, dict(engine="auto")),
    ("c2", 300, dict(engine="wave", stage_tables=3, waves_per_wg=12, persistent=1)),
    ("c3", 70, dict(engine="wave", lanes_per_cell=128, stage_tables=1, persistent=0)),
])
def test_plan_replays_equal_direct_solves(torch, name, n, kw):
    from paper_2111_07436_amd import camp
    wl = W.make_workload(name, n_cells=n)
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    opts = camp.make_opts(max_steps=20000, **kw)
    y0 = torch.from_numpy(wl.y0.copy()).cuda()
    y = y0.clone()
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    log(f"plan {name} {kw}: direct solve")
    m.solve_device(denv, y, wl.dt, 1e-8, 1e-18, opts, d_status=st)
    torch.cuda.synchronize()
    ref = y.cpu().numpy()
    assert int((st != 0).sum()) == 0
    ys = y0.clone()
    ps = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = camp.Plan(m, denv, ys, wl.dt, 1e-8, 1e-18, opts, d_status=ps)
    for rep in range(3):
        ys.copy_(y0)                      # eager work between replays
        ps.fill_(-1)
        torch.cuda.synchronize()
        log(f"plan {name}: replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        assert int((ps != 0).sum()) == 0
        assert np.array_equal(ys.cpu().numpy(), ref), rep
    plan.close()
    sample = [0, n // 2, n - 1]
    yr, sr, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, 1, 1e-10, 1e-20, cells=sample)
    assert np.all(sr == 0)
    assert_parity(ref[sample], yr, what=f"plan {name}")


def test_plan_rejects_other_engines(torch):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c1", n_cells=8)
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    y = torch.from_numpy(wl.y0.copy()).cuda()
    for eng in ("plain", "lane"):
        with pytest.raises(camp.CampError) as e:
            camp.Plan(m, denv, y, 60.0, 1e-4, 1e-12, camp.make_opts(eng))
        assert e.value.code == camp.EINVAL


def test_c1_sixty_calls_by_replay(torch):
    """The plain box model's 60 consecutive 60 s calls, each a replay of one plan, against
    the oracle (the integrator restarts every call)."""
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c1")
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    y = torch.from_numpy(wl.y0.copy()).cuda()
    st = torch.empty(wl.n_cells, dtype=torch.int32, device="cuda")
    plan = camp.Plan(m, denv, y, wl.dt, 1e-8, 1e-18, camp.make_opts("wave", max_steps=20000),
                     d_status=st)
    for _ in range(wl.n_calls):
        plan.launch()
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    plan.close()
    sample = [0, 50, 99]
    yr, sr, _ = oracle_solve(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, 1e-10, 1e-20, cells=sample)
    assert np.all(sr == 0)
    assert_parity(y.cpu().numpy()[sample], yr, what="c1 by replay")
