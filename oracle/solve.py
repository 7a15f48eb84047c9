"""Per-cell solve driver (oracle; test infrastructure only).

For each cell independently: compute the rate constants from that cell's environment
(held fixed over the host step), then integrate dy/dt = f(y) from the cell's state over
``dt`` (Sect. 2.4.2, runtime workflow: the host passes state and time step, the solver
integrates, the final state is returned). ``n_calls`` consecutive host steps restart
the integrator each call, as each host call is a fresh solve.
"""
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from .bdf import bdf_integrate
from .expand import expand
from .forcing import DenseSystem
from .rates import rate_constants_cell


class CellSolver:
    def __init__(self, mech):
        self.mech = mech
        self.x = expand(mech)
        self.sys = DenseSystem(self.x)

    def k_cell(self, env, c):
        ov = None if env.rate_override is None else env.rate_override[c]
        return rate_constants_cell(self.mech, self.x, float(env.T[c]), float(env.P[c]),
                                   float(env.cos_sza[c]), env.radius[c], env.mass[c], ov)

    def solve_cell(self, env, y0_row, c, dt, n_calls, rtol, atol, **kw):
        k = self.k_cell(env, c)
        sys = self.sys
        y = np.array(y0_row, dtype=np.float64)
        stats = []
        for _ in range(n_calls):
            y_new, status, st = bdf_integrate(lambda v: sys.f(k, v), lambda v: sys.jac(k, v),
                                              y, (0.0, dt), rtol, atol, **kw)
            stats.append(st.as_dict())
            if status != 0:
                return np.array(y0_row, dtype=np.float64), status, stats
            y = y_new
        return y, 0, stats


def oracle_solve(mech, env, y0, dt, n_calls, rtol, atol, cells=None, **kw):
    """Solve the listed cells (default: all). Returns (y [n, N], status [n], stats)."""
    cs = CellSolver(mech)
    idx = list(range(y0.shape[0])) if cells is None else list(cells)
    out = np.empty((len(idx), y0.shape[1]))
    status = np.zeros(len(idx), dtype=np.int32)
    stats = []
    for n, c in enumerate(idx):
        out[n], status[n], st = cs.solve_cell(env, y0[c], c, dt, n_calls, rtol, atol, **kw)
        stats.append(st)
    return out, status, stats


_WORKER = {}


def _init_worker(mech, env, y0, dt, n_calls, rtol, atol):
    # one process per core: keep each worker's BLAS single-threaded
    from threadpoolctl import threadpool_limits
    _WORKER.update(limits=threadpool_limits(limits=1), cs=CellSolver(mech), env=env, y0=y0,
                   dt=dt, n_calls=n_calls, rtol=rtol, atol=atol)


def _work(chunk):
    w = _WORKER
    res = []
    for c in chunk:
        y, s, _ = w["cs"].solve_cell(w["env"], w["y0"][c], c, w["dt"], w["n_calls"],
                                     w["rtol"], w["atol"])
        res.append((c, y, s))
    return res


def oracle_solve_parallel(mech, env, y0, dt, n_calls, rtol, atol, cells, processes, progress=None):
    """Same as ``oracle_solve`` with cells split over worker processes (one per core).
    ``progress(done, total)`` is called as cells complete."""
    from concurrent.futures import as_completed
    cells = list(cells)
    per = max(1, len(cells) // (4 * processes))
    chunks = [cells[i:i + per] for i in range(0, len(cells), per)]
    out = np.empty((len(cells), y0.shape[1]))
    status = np.zeros(len(cells), dtype=np.int32)
    pos = {c: n for n, c in enumerate(cells)}
    done = 0
    with ProcessPoolExecutor(max_workers=min(processes, len(chunks)), initializer=_init_worker,
                             initargs=(mech, env, y0, dt, n_calls, rtol, atol)) as ex:
        for fut in as_completed([ex.submit(_work, ch) for ch in chunks]):
            for c, y, s in fut.result():
                out[pos[c]] = y
                status[pos[c]] = s
                done += 1
            if progress:
                progress(done, len(cells))
    return out, status
