"""Benchmark: cell-steps/s of the batched stiff-chemistry solve on one MI355X.

One benchmark step = one host time step (dt = 3600 s) of every cell of the workload: rate
constants, then variable-order BDF with Newton iteration over the sparse LU, until every
cell reaches the end of the step. The default workload is the realistic-size gas-phase
configuration (10,000 cells, 72 species / 233 reactions, diurnal photolysis, FP64,
rtol 1e-4, atol 1e-12). Inputs are resident in device memory before timing starts; each
step re-solves the same initial state.

Prints one JSON line. Extra fields: the plain per-cell GPU BDF rate at the same tolerance
(`plain_value`, `speedup_vs_plain`), the accuracy of both forms against the oracle on
sampled cells, the roofline of the dominant kernel and the CPU-oracle baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 flop/clk)
HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel per launch, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (KiB per dispatch), each scaled by the ratio of the known
# size to the counter's reading for a plain device copy (`--calibrate-copy`). Valid only
# for the kernel and table-compiler sources it was taken with (their SHA-256 prefix);
# otherwise reported null.
KERNEL_SOURCES = ["paper_2111_07436_amd/csrc/engine_wave.hpp", "paper_2111_07436_amd/csrc/device.hpp",
                  "paper_2111_07436_amd/csrc/bdf_common.hpp", "paper_2111_07436_amd/csrc/compile.cpp"]
MEASURED_TRAFFIC = {
    # bdf_wave_kernel<2, 4, 64> (launch mode 4, 12 cells per workgroup, 256 workgroups,
    # persistent; the autotuner's pick), mean of the timed launches
    "c2": {"fetch_kib": 298560.3, "fetch_scale": 1048576 / 524299.5,
           "write_kib": 87035.3, "write_scale": 1048576 / 1048576.0, "sources": "776d4cb60417046c"},
}

WORKLOADS = {
    "c2": "gas-phase realistic size: 10,000 cells, 72 species / 233 reactions, 1 x 3600 s",
    "c1": "plain box model: 100 cells, 20 species / 40 reactions, 60 x 60 s",
    "c3": "multiphase: 100,000 cells, 72 gas + 6 phases x 4 sections (192 state / 809 reactions), 1 x 3600 s",
    "c5": "large: 500,000 cells, 200 gas + 10 phases x 8 sections (520 state / 1720 reactions), 1 x 3600 s",
}


CPU_SAMPLE = {"c1": 100, "c2": 10000, "c3": 1024, "c5": 128}
# The plain per-cell form is timed on at most this many cells of the workload (its rate in
# cell-steps/s does not depend on the count once the GPU is full).
PLAIN_CELLS = 20_000


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _progress(what):
    """Logs oracle progress about every tenth of the sample."""
    def cb(done, total):
        if done == total or done % max(1, total // 10) == 0:
            log(f"{what}: {done}/{total} cells")
    return cb


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel, or None when not measured for the
    current kernel sources."""
    t = MEASURED_TRAFFIC.get(workload)
    if not t or t["sources"] != kernel_source_hash():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def calibrate_copy(mib=1024, reps=5):
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps,
                      "kib_per_copy": n * 8 / 1024}), flush=True)


def algorithmic_flops(info, mech, stats_mean):
    """FP64 flops one cell's solve needs: the per-cell counters (forcing evaluations, Jacobians,
    LU factorizations, Newton iterations, steps) times the operation counts of the compiled
    mechanism (products, terms, contributions, LU pairs and the filled pattern)."""
    N, Z = info["n_state"], info["nnz_fill"]
    sum_nr_nr1 = 0
    for r in mech.reactions:
        nr = len(r.react)
        mult = 1
        if r.phase >= 0 and r.type == 5:
            mult = mech.phases[r.phase].n_instances
        elif r.type in (6, 7):
            mult = 2 * mech.phases[r.phase].n_instances
            nr = 1
        sum_nr_nr1 += mult * nr * (nr - 1)
    f_flops = info["n_partials"] + 2 * info["n_terms"]
    j_flops = sum_nr_nr1 + 2 * info["n_jac_contrib"] + 2 * Z
    lu_flops = 2 * info["lu_pairs"] + (Z - N) // 2
    solve_flops = 2 * (Z - N) + N
    s = stats_mean
    return (s["n_f"] * f_flops + s["n_jac"] * j_flops + s["n_lu"] * lu_flops
            + s["newton_iters"] * (solve_flops + 8 * N) + s["steps"] * 30 * N)


def run_gpu(name, engine, steps, warmup, rtol, atol, n_cells=None):
    import torch

    from paper_2111_07436_amd import camp
    from paper_2111_07436_amd import workloads as W

    wl = W.make_workload(name, n_cells=n_cells)
    m = camp.Mech(wl.mech)
    denv = camp.DeviceEnv(wl.env)
    y0 = torch.from_numpy(wl.y0).cuda()
    y = torch.empty_like(y0)
    st = torch.empty(wl.n_cells, dtype=torch.int32, device="cuda")
    opts = camp.make_opts(engine)

    def one_step():
        for _ in range(wl.n_calls):
            m.solve_device(denv, y, wl.dt, rtol, atol, opts, d_status=st)

    log(f"{name}/{engine}: {wl.n_cells} cells, warmup {warmup}")
    for _ in range(warmup):
        y.copy_(y0)
        one_step()
        torch.cuda.synchronize()
        log("warmup step done")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        y.copy_(y0)
        ev[i][0].record()
        one_step()
        ev[i][1].record()
        if wl.n_cells > PLAIN_CELLS:
            ev[i][1].synchronize()
            log(f"timed step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev])) / wl.n_calls
    failed = camp.count_failed(st)
    # counters of one extra solve
    y.copy_(y0)
    stats = torch.zeros((wl.n_cells, 8), dtype=torch.int32, device="cuda")
    for _ in range(wl.n_calls):
        m.solve_device(denv, y, wl.dt, rtol, atol, opts, d_status=st, d_stats=stats)
    torch.cuda.synchronize()
    s = stats.cpu().numpy().astype(np.float64)
    mean = {f: float(s[:, i].mean()) for i, f in enumerate(camp.STATS_FIELDS)}
    return dict(wl=wl, mech=m, seconds=t1 - t0, kernel_ms=kernel_ms, failed=failed, stats=mean,
                y=y.cpu().numpy())


def accuracy(wl, y_gpu, cells, processes):
    from oracle.solve import oracle_solve_parallel
    yr, st = oracle_solve_parallel(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, 1e-10, 1e-20, cells, processes,
                                   progress=_progress("accuracy oracle"))
    ref = yr[st == 0]
    got = y_gpu[np.asarray(cells)[st == 0]]
    big = np.abs(ref) >= 1e-12
    rel = np.abs(got[big] - ref[big]) / np.abs(ref[big])
    frac_fail = float(np.mean(rel > 1e-4)) if rel.size else 0.0
    return {"max_rel": float(rel.max()), "p99_rel": float(np.quantile(rel, 0.99)),
            "frac_species_over_1e-4": frac_fail, "cells": len(cells), "oracle_rtol": 1e-10}


def cpu_baseline(wl, rtol, atol, sample, processes):
    from oracle.solve import oracle_solve_parallel
    cells = np.linspace(0, wl.n_cells - 1, sample).astype(int)
    t = time.perf_counter()
    _, st = oracle_solve_parallel(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, rtol, atol, cells, processes,
                                  progress=_progress("cpu baseline"))
    dt = time.perf_counter() - t
    return {"value": len(cells) * 1 / dt, "unit": "cell-steps/s", "cores": processes, "kind": "oracle",
            "sample": f"{len(cells)} cells evenly strided over the {wl.n_cells}-cell workload, "
                      f"one host step each, rtol {rtol:g}, atol {atol:g}, one single-threaded "
                      f"process per core",
            "seconds": dt, "failed": int(np.sum(st != 0))}


def run_served(n_requests, seed=0, max_inflight=8, load_frac=0.7):
    """Served stream: Poisson arrivals of requests of 1e3..2e5 cells (log-uniform) on two
    resident mechanisms (gas c2 / multiphase c3), continuous batching through the server.
    The configured 200 requests/s offers far more work than one GPU sustains, so arrivals
    are replayed at `load_frac` of the capacity measured from solo solves."""
    import torch

    from paper_2111_07436_amd import camp
    from paper_2111_07436_amd import workloads as W

    mechs = [camp.Mech(W.make_mechanism("c2")), camp.Mech(W.make_mechanism("c3"))]
    arrival, cells, mech_id = W.make_request_trace(n_requests, seed=seed)
    reqs = []
    log = lambda msg: print(f"[served] {msg}", file=sys.stderr, flush=True)
    log(f"generating {n_requests} requests, {int(np.sum(cells))} cells")
    for i in range(n_requests):
        m = mechs[int(mech_id[i])]
        env, y0 = W.make_request(m.src, int(cells[i]), trace_seed=seed, index=i)
        reqs.append(dict(m=m, denv=camp.DeviceEnv(env), y0=torch.from_numpy(y0).cuda(),
                         y=torch.empty((int(cells[i]), m.n_state), dtype=torch.float64, device="cuda"),
                         st=torch.empty(int(cells[i]), dtype=torch.int32, device="cuda"), n=int(cells[i])))
    opts = camp.make_opts("auto")
    # warm the autotuner for every size bucket, then measure capacity from solo solves
    for r in reqs:
        r["y"].copy_(r["y0"])
        r["m"].solve_device(r["denv"], r["y"], 3600.0, 1e-4, 1e-12, opts, d_status=r["st"])
    torch.cuda.synchronize()
    log("autotuner warm")
    solo_s, solo_cells = 0.0, 0
    for r in reqs:
        r["y"].copy_(r["y0"])
        torch.cuda.synchronize()
        t = time.perf_counter()
        r["m"].solve_device(r["denv"], r["y"], 3600.0, 1e-4, 1e-12, opts, d_status=r["st"])
        torch.cuda.synchronize()
        solo_s += time.perf_counter() - t
        solo_cells += r["n"]
        log(f"solo {len(reqs)} reqs: {r['n']} cells on {'c3' if r['m'] is mechs[1] else 'c2'} "
            f"in {time.perf_counter() - t:.3f} s")
    capacity = solo_cells / solo_s
    mean_cells = float(np.mean(cells))
    rate = load_frac * capacity / mean_cells
    gaps = np.diff(np.concatenate(([0.0], arrival))) * (200.0 / rate)   # same Poisson draws, rescaled
    for r in reqs:
        r["y"].copy_(r["y0"])
    torch.cuda.synchronize()
    srv = camp.Server(max_inflight=max_inflight)
    t0 = time.perf_counter()
    next_t = t0
    tickets = []
    for i, r in enumerate(reqs):
        next_t += gaps[i]
        while time.perf_counter() < next_t:
            time.sleep(min(0.0005, max(0.0, next_t - time.perf_counter())))
        tickets.append(srv.submit(r["m"], r["denv"], r["y"], 3600.0, 1e-4, 1e-12, r["st"], opts))
        if i % 4 == 0:
            log(f"submitted {i + 1}/{n_requests} at t={time.perf_counter() - t0:.2f} s")
    lat, failed = [], 0
    for t in tickets:
        srv.wait(t)
        done, nf, l = srv.poll(t)
        lat.append(l)
        failed += nf
    t1 = time.perf_counter()
    srv.close()
    total = int(np.sum(cells))
    return {
        "metric": "served p50/p99 latency and sustained cell-steps/s (Poisson stream, continuous batching)",
        "value": total / (t1 - t0), "unit": "cell-steps/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic (seeded generator, PCG64 seed 0)",
        "config": {"workload": "served stream: requests of 1e3..2e5 cells (log-uniform), gas c2 or "
                               "multiphase c3 mechanism (uniform), Poisson arrivals",
                   "requests": n_requests, "max_inflight": max_inflight,
                   "offered_rate_hz_configured": 200.0,
                   "offered_cell_steps_s_configured": 200.0 * mean_cells,
                   "replayed_rate_hz": rate, "replayed_load_frac_of_capacity": load_frac},
        "capacity_cell_steps_s_solo": capacity,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(np.max(lat)), "failed_cells": failed, "total_cells": total,
        "wall_s": t1 - t0,
    }


def run_cost_ordered(run, steps, rtol, atol):
    """The second host step of the workload's cells, timed in index order and with the
    cells taken costliest first (cell_order from the first step's per-cell Newton
    iterations), as a host model would schedule it from its previous step's counters."""
    import torch

    from paper_2111_07436_amd import camp

    wl, m = run["wl"], run["mech"]
    denv = camp.DeviceEnv(wl.env)
    n = wl.n_cells
    y1 = torch.from_numpy(wl.y0).cuda()
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    stats = torch.zeros((n, 8), dtype=torch.int32, device="cuda")
    m.solve_device(denv, y1, wl.dt, rtol, atol, None, d_status=st, d_stats=stats)
    iters = stats[:, camp.STATS_FIELDS.index("newton_iters")].cpu().numpy()
    order = torch.from_numpy(np.argsort(-iters, kind="stable").astype(np.int32)).cuda()
    y = torch.empty_like(y1)
    res = {}
    for label, opts in (("index_order", None), ("cost_ordered", camp.make_opts(cell_order=order))):
        y.copy_(y1)
        m.solve_device(denv, y, wl.dt, rtol, atol, opts, d_status=st)   # warm
        ms = []
        for _ in range(steps):
            y.copy_(y1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            m.solve_device(denv, y, wl.dt, rtol, atol, opts, d_status=st)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        res[label] = float(np.median(ms))
        log(f"second host step, {label}: {res[label]:.2f} ms")
    return {"what": "second host step of the same cells; cells taken costliest first by the "
                    "first step's per-cell Newton iterations (camp_opts.cell_order)",
            "value": n / (res["cost_ordered"] * 1e-3), "unit": "cell-steps/s",
            "ms_per_step": res["cost_ordered"], "index_order_ms_per_step": res["index_order"],
            "index_order_value": n / (res["index_order"] * 1e-3), "steps": steps,
            "failed_cells": camp.count_failed(st)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["c4"])
    ap.add_argument("--requests", type=int, default=24, help="served stream (c4) length")
    ap.add_argument("--engine", default="auto")
    ap.add_argument("--rtol", type=float, default=1e-4)
    ap.add_argument("--atol", type=float, default=1e-12)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-ordered", action="store_true",
                    help="skip the second-host-step cost-ordered measurement (default: run it "
                         "for workloads up to 100 000 cells)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="cells in the CPU-oracle sample (default: about 10-30 s on the host's "
                         "cores for the workload: c1 100, c2 10000, c3 1024, c5 128)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every cell is independent, so several GPUs would each "
              "take a share of the cells with no exchange; only --gpus 1 is supported.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    processes = max(1, min(16, os.cpu_count() or 1))
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "c4":
        print(json.dumps(run_served(args.requests)), flush=True)
        return

    main_run = run_gpu(args.workload, args.engine, args.steps, args.warmup, args.rtol, args.atol)
    wl = main_run["wl"]
    cells = wl.n_cells
    value = cells * args.steps / main_run["seconds"]
    out = {
        "metric": "cell-steps/sec at rtol 1e-4 vs plain per-cell BDF; served p50/p99 latency",
        "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * main_run["seconds"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator, PCG64 seed 0)",
        "config": {"workload": WORKLOADS[args.workload], "cells": cells, "dt_s": wl.dt,
                   "rtol": args.rtol, "atol": args.atol, "engine": args.engine},
        "failed_cells": main_run["failed"],
        "cell_stats_mean": main_run["stats"],
    }
    if not args.no_plain:
        pc = min(cells, PLAIN_CELLS)
        plain = run_gpu(args.workload, "plain", 1, 1, args.rtol, args.atol, n_cells=pc)
        pv = pc / plain["seconds"]
        out["plain_value"] = pv
        out["plain_cells"] = pc
        out["speedup_vs_plain"] = value / pv
    flops = algorithmic_flops(main_run["mech"].info, wl.mech, main_run["stats"]) * cells
    achieved = flops / (main_run["kernel_ms"] * 1e-3) / 1e12
    compulsory = 8.0 * cells * (2 * wl.mech.n_state + 3) * wl.n_calls
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                       "traffic": measured_traffic(args.workload),
                       "kernel": "bdf_wave_kernel", "kernel_ms": main_run["kernel_ms"],
                       "flops_per_launch": flops,
                       "compulsory_hbm_GBs": compulsory / (main_run["kernel_ms"] * 1e-3) / 1e9}
    if not args.no_ordered and cells <= 100_000:
        out["second_step_cost_ordered"] = run_cost_ordered(main_run, max(3, min(args.steps, 10)),
                                                           args.rtol, args.atol)
    if not args.no_accuracy:
        log("accuracy against the oracle")
        sample = list(np.linspace(0, min(cells, PLAIN_CELLS) - 1, 16).astype(int))
        out["accuracy"] = accuracy(wl, main_run["y"], sample, processes)
        if not args.no_plain:
            out["accuracy_plain"] = accuracy(plain["wl"], plain["y"], sample, processes)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        sample = args.cpu_sample or CPU_SAMPLE[args.workload]
        out["cpu_baseline"] = cpu_baseline(wl, args.rtol, args.atol, min(sample, cells), processes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
