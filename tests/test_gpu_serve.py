"""Served requests: continuous batching keeps every result identical to a solo solve.

Requests of different sizes on two resident mechanisms (the gas mechanism and the
multiphase one) are submitted together; each result must equal, bit for bit, the result
of solving that request alone (no arithmetic crosses cells or requests). A tight memory
budget must queue requests (admission by footprint) without changing any result.
"""
import numpy as np
import pytest

from paper_2111_07436_amd import workloads as W
from tests.gpu_util import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _requests(camp, torch, sizes):
    mechs = [camp.Mech(W.make_mechanism("c2")), camp.Mech(W.make_mechanism("c3"))]
    out = []
    for i, n in enumerate(sizes):
        m = mechs[i % 2]
        env, y0 = W.make_request(m.src, n, trace_seed=0, index=i)
        out.append(dict(m=m, denv=camp.DeviceEnv(env), y0=torch.from_numpy(y0).cuda(), n=n))
    return mechs, out


def _solo(camp, torch, reqs, opts):
    res = []
    for r in reqs:
        y = r["y0"].clone()
        st = torch.empty(r["n"], dtype=torch.int32, device="cuda")
        r["m"].solve_device(r["denv"], y, 3600.0, 1e-4, 1e-12, opts, d_status=st)
        torch.cuda.synchronize()
        res.append((y.cpu().numpy(), st.cpu().numpy()))
    return res


@pytest.mark.parametrize("budget_mode", ["roomy", "tight"])
def test_alone_equals_mix(torch, budget_mode):
    from paper_2111_07436_amd import camp
    sizes = [700, 2100, 130, 4000, 1500, 65]
    mechs, reqs = _requests(camp, torch, sizes)
    opts = camp.make_opts("wave", max_steps=20000)
    solo = _solo(camp, torch, reqs, opts)
    budget = 0 if budget_mode == "roomy" else 600_000     # bytes: forces queueing
    srv = camp.Server(max_bytes=budget, max_inflight=4)
    outs, tickets = [], []
    saw_queue = False
    for r in reqs:
        outs.append((r["y0"].clone(), torch.full((r["n"],), -7, dtype=torch.int32, device="cuda")))
    torch.cuda.synchronize()          # inputs ready; no device-wide sync between submissions
    for r, (y, st) in zip(reqs, outs):
        tickets.append(srv.submit(r["m"], r["denv"], y, 3600.0, 1e-4, 1e-12, st, opts))
        inflight, queued = srv.progress()
        saw_queue |= queued > 0
    lat = []
    for t in tickets:
        srv.wait(t)
        done, nf, l = srv.poll(t)
        assert done
        lat.append(l)
    torch.cuda.synchronize()
    for (y, st), (ys, ss), r in zip(outs, solo, reqs):
        assert np.array_equal(st.cpu().numpy(), ss)
        assert np.array_equal(y.cpu().numpy(), ys), r["n"]
    log(f"serve {budget_mode}: latencies {np.round(lat, 4).tolist()} queued seen {saw_queue}")
    if budget_mode == "tight":
        assert saw_queue
    assert all(l > 0 for l in lat)
    srv.close()


def test_poisoned_request_fails_alone(torch):
    from paper_2111_07436_amd import camp
    mechs, reqs = _requests(camp, torch, [300, 300])
    bad_env, y0 = W.make_request(mechs[0].src, 300, trace_seed=0, index=0)
    bad_env.T[:] = np.nan
    bad = dict(m=mechs[0], denv=camp.DeviceEnv(bad_env), y0=torch.from_numpy(y0).cuda(), n=300)
    opts = camp.make_opts("wave", max_steps=20000)
    solo = _solo(camp, torch, [reqs[1]], opts)[0]
    srv = camp.Server(max_inflight=2)
    yb, sb = bad["y0"].clone(), torch.empty(300, dtype=torch.int32, device="cuda")
    yg, sg = reqs[1]["y0"].clone(), torch.empty(300, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    tb = srv.submit(bad["m"], bad["denv"], yb, 3600.0, 1e-4, 1e-12, sb, opts)
    tg = srv.submit(reqs[1]["m"], reqs[1]["denv"], yg, 3600.0, 1e-4, 1e-12, sg, opts)
    srv.wait(tb)
    srv.wait(tg)
    assert srv.poll(tb)[1] == 300
    assert srv.poll(tg)[1] == int(np.sum(solo[1] != 0))
    assert np.array_equal(sg.cpu().numpy(), solo[1])
    assert np.array_equal(yg.cpu().numpy(), solo[0])
    assert np.array_equal(yb.cpu().numpy(), bad["y0"].cpu().numpy())
    srv.close()


def test_auto_engine_cold_cache_matches_solo(torch, monkeypatch):
    # Fresh mechanisms: the server autotunes each cold (mechanism, size) bucket on its own
    # thread; solo solves afterwards reuse the cached launch, so results agree bit for bit.
    from paper_2111_07436_amd import camp
    monkeypatch.delenv("CAMP_TUNE_CACHE", raising=False)
    sizes = [5000, 300, 4000, 9000]
    mechs, reqs = _requests(camp, torch, sizes)
    srv = camp.Server(max_bytes=0, max_inflight=3)
    outs = [(r["y0"].clone(), torch.full((r["n"],), -7, dtype=torch.int32, device="cuda")) for r in reqs]
    torch.cuda.synchronize()
    tickets = [srv.submit(r["m"], r["denv"], y, 3600.0, 1e-4, 1e-12, st, None)
               for r, (y, st) in zip(reqs, outs)]
    for t in tickets:
        srv.wait(t)
        assert srv.poll(t)[0]
    torch.cuda.synchronize()
    srv.close()
    solo = _solo(camp, torch, reqs, None)
    for (y, st), (ys, ss), r in zip(outs, solo, reqs):
        assert np.array_equal(st.cpu().numpy(), ss)
        assert np.array_equal(y.cpu().numpy(), ys), r["n"]
        assert not np.any(ss), r["n"]
