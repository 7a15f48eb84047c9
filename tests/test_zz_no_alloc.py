"""The no-allocation solve (camp_solve_device_noalloc) through the C ABI (collected last).

Its output must equal camp_solve_device's with the same launch choice, bit for bit, on two
calls in a row, the second with a smaller input (the shared scratch keeps the first call's
contents, so whatever must start at zero has to be cleared). Also: a caller's cell order,
engine AUTO after the autotuner has run, and the error paths (tables not resident, too
much scratch needed, an engine that is not the fused wavefront one).
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from tests.gpu_util import assert_parity, log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _direct_and_noalloc(torch, m, wl, opts, noalloc_opts=None):
    from paper_2111_07436_amd import camp
    denv = camp.DeviceEnv(wl.env)
    y = torch.from_numpy(wl.y0.copy()).cuda()
    st = torch.empty(wl.n_cells, dtype=torch.int32, device="cuda")
    m.solve_device(denv, y, wl.dt, 1e-8, 1e-18, opts, d_status=st)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    z = torch.from_numpy(wl.y0.copy()).cuda()
    sz = torch.full((wl.n_cells,), -7, dtype=torch.int32, device="cuda")
    m.solve_device_noalloc(denv, z, wl.dt, 1e-8, 1e-18, noalloc_opts or opts, d_status=sz)
    torch.cuda.synchronize()
    assert int((sz != 0).sum()) == 0
    return y.cpu().numpy(), z.cpu().numpy()


def test_noalloc_equals_direct_two_calls_shrinking(torch):
    from paper_2111_07436_amd import camp
    for name, sizes, kw in (("c2", (600, 130), dict(stage_tables=3, waves_per_wg=12)),
                            ("c3", (200, 70), dict(stage_tables=3, lanes_per_cell=128)),
                            ("c3", (150, 65), dict(stage_tables=1, lanes_per_cell=256))):
        mech = W.make_mechanism(name)
        m = camp.Mech(mech)
        opts = camp.make_opts("wave", max_steps=20000, persistent=1, **kw)
        for n in sizes:
            log(f"noalloc {name} {kw}: {n} cells")
            wl = W.make_workload(name, n_cells=n)
            a, b = _direct_and_noalloc(torch, m, wl, opts)
            assert np.array_equal(a, b), (name, n)


def test_noalloc_cell_order_and_auto(torch):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c2", n_cells=500)
    m = camp.Mech(wl.mech)
    perm = torch.from_numpy(np.random.default_rng(5).permutation(500).astype(np.int32)).cuda()
    opts = camp.make_opts("wave", max_steps=20000, stage_tables=4, persistent=1, cell_order=perm)
    log("noalloc c2 500 cells with a cell order")
    a, b = _direct_and_noalloc(torch, m, wl, opts)
    assert np.array_equal(a, b)
    log("noalloc c2 500 cells, engine auto (the autotuner's cached choice)")
    auto = camp.make_opts("auto", max_steps=20000)
    a, b = _direct_and_noalloc(torch, m, wl, auto)
    assert np.array_equal(a, b)
    wl2 = W.make_workload("c2", n_cells=37)
    log("noalloc c2 37 cells, engine auto (smaller bucket, no trials)")
    c, d = _direct_and_noalloc(torch, m, wl2, camp.make_opts("wave", max_steps=20000), auto)
    assert_parity(d, c, rel_tol=1e-6, what="noalloc auto default vs direct")


def test_noalloc_errors(torch):
    from paper_2111_07436_amd import camp
    wl = W.make_workload("c1", n_cells=8)
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    y = torch.from_numpy(wl.y0.copy()).cuda()
    st = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(camp.CampError) as e:          # tables not resident yet
        m.solve_device_noalloc(denv, y, 60.0, 1e-4, 1e-12, None, d_status=st)
    assert e.value.code == camp.EINVAL and "resident" in str(e.value)
    m.solve_device(denv, y, 60.0, 1e-4, 1e-12, None, d_status=st)
    for eng in ("plain", "lane"):
        with pytest.raises(camp.CampError) as e:
            m.solve_device_noalloc(denv, y, 60.0, 1e-4, 1e-12, camp.make_opts(eng), d_status=st)
        assert e.value.code == camp.EINVAL
    # the large mechanism with one wavefront per cell and rate constants in global scratch
    # for 16 workgroups per CU needs far more than the 32 MiB array: rejected before launch
    wl5 = W.make_workload("c5", n_cells=16384)
    m5 = camp.Mech(wl5.mech)
    d5 = camp.DeviceEnv(wl5.env)
    sub = wl5.take(list(range(64)))                   # makes the tables resident
    m5.solve_device(camp.DeviceEnv(sub.env), torch.from_numpy(sub.y0.copy()).cuda(), 3600.0, 1e-4,
                    1e-12, camp.make_opts("wave", max_steps=20000),
                    d_status=torch.empty(64, dtype=torch.int32, device="cuda"))
    y5 = torch.from_numpy(wl5.y0.copy()).cuda()
    s5 = torch.empty(16384, dtype=torch.int32, device="cuda")
    big = camp.make_opts("wave", lanes_per_cell=64, stage_tables=3, waves_per_wg=2, wg_per_cu=16,
                         persistent=1)
    assert camp._lib.camp_noalloc_scratch_bytes() == 32 << 20
    with pytest.raises(camp.CampError) as e:
        m5.solve_device_noalloc(d5, y5, 3600.0, 1e-4, 1e-12, big, d_status=s5)
    assert e.value.code == camp.EINVAL and "scratch" in str(e.value)
