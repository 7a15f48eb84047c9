"""ctypes binding of libcamp.so (argument marshalling only; every step runs in the library).

Device arrays are torch CUDA (HIP) tensors: the binding passes their data pointers and the
current torch stream to the C ABI declared in include/camp.h. Importing this module loads
the library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcamp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_07436_amd.build`")
# torch ships its own libamdhip64.so.7; load it first so that libcamp.so binds to the same
# HIP runtime (two runtimes in one process do not share devices, memory or streams).
try:
    import torch  # noqa: F401
except ImportError:
    torch = None
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ESOLVE = 0, -1, -2, -3, -4
ENGINE_AUTO, ENGINE_PLAIN, ENGINE_FUSED_WAVE, ENGINE_FUSED_LANE = 0, 1, 2, 3
ENGINES = {"auto": 0, "plain": 1, "wave": 2, "lane": 3}


class CampError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"camp error {code}: {msg}")
        self.code = code


class Species(C.Structure):
    _fields_ = [("name", C.c_char_p), ("phase", C.c_int), ("mw_kg_mol", C.c_double),
                ("diff_m2_s", C.c_double), ("accom", C.c_double)]


class Phase(C.Structure):
    _fields_ = [("name", C.c_char_p), ("n_species", C.c_int), ("species", C.POINTER(C.c_int)),
                ("n_instances", C.c_int), ("density_kg_m3", C.c_double),
                ("mw_absorber_kg_mol", C.c_double), ("radius_from_state", C.c_int)]


class Reaction(C.Structure):
    _fields_ = [("type", C.c_int), ("phase", C.c_int), ("n_react", C.c_int), ("react", C.c_int * 3),
                ("n_prod", C.c_int), ("prod", C.c_int * 3), ("yield_", C.c_double * 3),
                ("p", C.c_double * 10)]


class MechInfo(C.Structure):
    _fields_ = [("n_state", C.c_int), ("n_gas", C.c_int), ("n_instances", C.c_int),
                ("n_rxn_expanded", C.c_int), ("n_external", C.c_int), ("nnz_pattern", C.c_int),
                ("nnz_fill", C.c_int), ("lu_pairs", C.c_longlong), ("lu_levels", C.c_int),
                ("fwd_levels", C.c_int), ("bwd_levels", C.c_int), ("n_partials", C.c_int),
                ("n_terms", C.c_int), ("n_jac_contrib", C.c_int), ("tail_k", C.c_int),
                ("nnz_lu", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Env(C.Structure):
    _fields_ = [("T_K", C.c_void_p), ("P_Pa", C.c_void_p), ("cos_sza", C.c_void_p),
                ("radius_m", C.c_void_p), ("aer_mass_kg_m3", C.c_void_p), ("rate_override", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("max_order", C.c_int), ("max_steps", C.c_int), ("newton_max_iter", C.c_int),
                ("h_min", C.c_double), ("h_init", C.c_double), ("engine", C.c_int),
                ("wg_per_cu", C.c_int), ("persistent", C.c_int), ("use_graph", C.c_int),
                ("waves_per_wg", C.c_int), ("stage_tables", C.c_int), ("lanes_per_cell", C.c_int),
                ("full_newton", C.c_int), ("cell_order", C.c_void_p),
                ("lu_gamma_drift", C.c_double), ("lu_max_age", C.c_int), ("newton_tol", C.c_double)]


class CellStats(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("steps", "rejected", "newton_fail", "newton_iters", "n_f",
                                       "n_jac", "n_lu", "order")]


STATS_FIELDS = [f for f, _ in CellStats._fields_]

_P = C.c_void_p
_sig = {
    "camp_mech_load": (C.c_int, [C.POINTER(Reaction), C.c_int, C.POINTER(Species), C.c_int,
                                 C.POINTER(Phase), C.c_int, C.POINTER(_P)]),
    "camp_mech_info": (C.c_int, [_P, C.POINTER(MechInfo)]),
    "camp_mech_load_json": (C.c_int, [C.c_char_p, C.POINTER(_P)]),
    "camp_mech_pack": (C.c_int, [_P, _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "camp_mech_unpack": (C.c_int, [_P, C.c_size_t, C.POINTER(_P)]),
    "camp_mech_export": (C.c_int, [_P, _P, _P, _P, _P]),
    "camp_mech_free": (None, [_P]),
    "camp_emulate_factor_solve": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "camp_mech_layout_info": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P]),
    "camp_tuned_launch": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P]),
    "camp_solve": (C.c_int, [_P, C.c_int, _P, C.POINTER(Env), C.c_double, C.c_double, C.c_double,
                             C.POINTER(Opts), _P, _P]),
    "camp_solve_device": (C.c_int, [_P, C.c_int, _P, C.POINTER(Env), C.c_double, C.c_double,
                                    C.c_double, C.POINTER(Opts), _P, _P, _P]),
    "camp_rate_constants_device": (C.c_int, [_P, C.c_int, C.POINTER(Env), _P, _P]),
    "camp_forcing_device": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "camp_newton_matrix_device": (C.c_int, [_P, C.c_int, _P, _P, C.c_double, _P, _P]),
    "camp_lu_factor_device": (C.c_int, [_P, C.c_int, _P, _P]),
    "camp_lu_solve_device": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "camp_count_failed": (C.c_int, [C.c_int, _P, C.POINTER(C.c_int), _P]),
    "camp_probe_copy": (C.c_int, [_P, _P, C.c_size_t, C.c_int, _P, C.POINTER(C.c_double)]),
    "camp_probe_fma": (C.c_int, [_P, C.c_int, C.c_int, _P, C.POINTER(C.c_double)]),
    "camp_plan_create": (C.c_int, [_P, C.c_int, _P, C.POINTER(Env), C.c_double, C.c_double,
                                   C.c_double, C.POINTER(Opts), _P, _P, _P, C.POINTER(_P)]),
    "camp_plan_launch": (C.c_int, [_P, _P]),
    "camp_plan_free": (None, [_P]),
    "camp_solve_device_noalloc": (C.c_int, [_P, C.c_int, _P, C.POINTER(Env), C.c_double, C.c_double,
                                            C.c_double, C.POINTER(Opts), _P, _P, _P]),
    "camp_noalloc_scratch_bytes": (C.c_size_t, []),
    "camp_serve_create": (C.c_int, [C.c_longlong, C.c_int, C.POINTER(_P)]),
    "camp_serve_submit": (C.c_int, [_P, _P, C.c_int, _P, C.POINTER(Env), C.c_double, C.c_double,
                                    C.c_double, C.POINTER(Opts), _P, C.POINTER(C.c_longlong)]),
    "camp_serve_poll": (C.c_int, [_P, C.c_longlong, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_double)]),
    "camp_serve_wait": (C.c_int, [_P, C.c_longlong]),
    "camp_serve_progress": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "camp_serve_destroy": (None, [_P]),
    "camp_last_error": (C.c_char_p, []),
}
for _n, (_res, _args) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


def _check(rc):
    if rc != OK:
        raise CampError(rc, _lib.camp_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(engine="auto", max_order=0, max_steps=0, newton_max_iter=0, h_min=0.0, h_init=0.0,
              wg_per_cu=0, persistent=-1, use_graph=0, waves_per_wg=0, stage_tables=-1,
              lanes_per_cell=0, full_newton=0, cell_order=None, lu_gamma_drift=0.0, lu_max_age=0,
              newton_tol=0.0):
    """camp_opts; ``cell_order`` is an int32 torch tensor (device solves) or numpy array
    (host solves) holding a permutation of the cells, kept alive by the returned object."""
    e = ENGINES[engine] if isinstance(engine, str) else int(engine)
    ptr = None
    if cell_order is not None:
        if isinstance(cell_order, np.ndarray):
            if cell_order.dtype != np.int32 or not cell_order.flags.c_contiguous:
                raise ValueError("cell_order must be a contiguous int32 array")
            ptr = cell_order.ctypes.data
        else:
            import torch
            if cell_order.dtype != torch.int32 or not cell_order.is_contiguous():
                raise ValueError("cell_order must be a contiguous int32 tensor")
            ptr = cell_order.data_ptr()
    o = Opts(max_order, max_steps, newton_max_iter, h_min, h_init, e, wg_per_cu,
             persistent, use_graph, waves_per_wg, stage_tables, lanes_per_cell, full_newton, ptr,
             lu_gamma_drift, lu_max_age, newton_tol)
    o._keep = cell_order
    return o


class Mech:
    """A compiled mechanism (wraps camp_mech): from a workloads.Mechanism, or with
    Mech.from_json / Mech.unpack."""

    @classmethod
    def _from_handle(cls, h, src=None):
        self = cls.__new__(cls)
        self.src = src
        self._names, self._phase_ids = [], []
        self.h = h
        inf = MechInfo()
        _check(_lib.camp_mech_info(h, C.byref(inf)))
        self.info = inf.as_dict()
        return self

    @classmethod
    def from_json(cls, text):
        """camp_mech_load_json on a JSON document (str or bytes)."""
        h = C.c_void_p()
        _check(_lib.camp_mech_load_json(text.encode() if isinstance(text, str) else text, C.byref(h)))
        return cls._from_handle(h)

    @classmethod
    def unpack(cls, data: bytes):
        """camp_mech_unpack of a camp_mech_pack buffer."""
        h = C.c_void_p()
        buf = C.create_string_buffer(bytes(data), len(data))
        _check(_lib.camp_mech_unpack(buf, len(data), C.byref(h)))
        return cls._from_handle(h)

    def pack(self) -> bytes:
        """camp_mech_pack: the compiled mechanism as bytes."""
        n = C.c_size_t(0)
        _check(_lib.camp_mech_pack(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(_lib.camp_mech_pack(self.h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def __init__(self, mech):
        self.src = mech
        sp = (Species * len(mech.species))()
        self._names = []
        for i, s in enumerate(mech.species):
            nm = s.name.encode()
            self._names.append(nm)
            sp[i] = Species(nm, s.phase, s.mw, s.diff, s.accom)
        ph = (Phase * max(1, len(mech.phases)))()
        self._phase_ids = []
        for i, p in enumerate(mech.phases):
            ids = (C.c_int * len(p.species))(*p.species)
            self._phase_ids.append(ids)
            nm = p.name.encode()
            self._names.append(nm)
            ph[i] = Phase(nm, len(p.species), ids, p.n_instances, p.density, p.mw_absorber,
                          int(getattr(p, "radius_from_state", False)))
        rx = (Reaction * max(1, len(mech.reactions)))()
        for i, r in enumerate(mech.reactions):
            rr = Reaction()
            rr.type = r.type
            rr.phase = r.phase
            rr.n_react = len(r.react)
            rr.n_prod = len(r.prod)
            for k, v in enumerate(r.react):
                rr.react[k] = v
            for k, v in enumerate(r.prod):
                rr.prod[k] = v
                rr.yield_[k] = r.yields[k]
            for k, v in enumerate(list(r.p)[:10]):
                rr.p[k] = v
            rx[i] = rr
        h = C.c_void_p()
        _check(_lib.camp_mech_load(rx, len(mech.reactions), sp, len(mech.species), ph,
                                   len(mech.phases), C.byref(h)))
        self.h = h
        inf = MechInfo()
        _check(_lib.camp_mech_info(h, C.byref(inf)))
        self.info = inf.as_dict()

    def close(self):
        if getattr(self, "h", None):
            _lib.camp_mech_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_state(self):
        return self.info["n_state"]

    @property
    def n_rxn(self):
        return self.info["n_rxn_expanded"]

    @property
    def nnz(self):
        return self.info["nnz_fill"]

    def export(self):
        n, z = self.info["n_state"], self.info["nnz_fill"]
        perm = np.zeros(n, np.int32)
        rp = np.zeros(n + 1, np.int32)
        col = np.zeros(z, np.int32)
        p0 = np.zeros(z, np.int32)
        _check(_lib.camp_mech_export(self.h, perm.ctypes.data, rp.ctypes.data, col.ctypes.data,
                                     p0.ctypes.data))
        return perm, rp, col, p0

    def layout_info(self, lanes_per_cell):
        """camp_mech_layout_info: dict of the fused kernel's table layout."""
        v = [C.c_int(0) for _ in range(5)]
        _check(_lib.camp_mech_layout_info(self.h, int(lanes_per_cell), *[C.byref(a) for a in v]))
        return dict(zip(["tail_k", "fwd_levels", "bwd_levels", "lu_levels", "staged_bytes"],
                        [a.value for a in v]))

    def tuned_launch(self, n_cells):
        """camp_tuned_launch: the autotuner's cached choice for this size bucket, or None."""
        v = [C.c_int(0) for _ in range(5)]
        if _lib.camp_tuned_launch(self.h, int(n_cells), *[C.byref(a) for a in v]) != OK:
            return None
        return dict(zip(["engine", "lanes_per_cell", "launch_mode", "cells_per_wg", "wg_per_cu"],
                        [a.value for a in v]))

    def emulate_factor_solve(self, m, b, lanes_per_cell=64, dense_tail=True):
        """camp_emulate_factor_solve on host arrays: returns (factors, x) for a Newton matrix
        m[Z] (slot order) and right-hand side b[N] (elimination order)."""
        m = np.ascontiguousarray(m, dtype=np.float64).copy()
        x = np.ascontiguousarray(b, dtype=np.float64).copy()
        _check(_lib.camp_emulate_factor_solve(self.h, int(lanes_per_cell), int(bool(dense_tail)),
                                              m.ctypes.data, x.ctypes.data))
        return m, x

    # ------------------------------------------------------------------ host solve
    def solve(self, env, y, dt, rtol, atol, opts: Optional[Opts] = None, stats=False):
        """camp_solve on host arrays; returns (y_out, status, stats or None)."""
        y = np.ascontiguousarray(y, dtype=np.float64).copy()
        n = y.shape[0]
        arrs = _host_env(env)
        e = Env(*[None if a is None else a.ctypes.data for a in arrs])
        st = np.zeros(n, np.int32)
        cs = (CellStats * max(1, n))() if stats else None
        rc = _lib.camp_solve(self.h, n, y.ctypes.data, C.byref(e), dt, rtol, atol,
                             None if opts is None else C.byref(opts), st.ctypes.data, cs)
        if rc not in (OK, ESOLVE):
            _check(rc)
        out_stats = None
        if stats:
            out_stats = np.array([[getattr(cs[i], f) for f in STATS_FIELDS] for i in range(n)])
        return y, st, out_stats

    # ------------------------------------------------------------------ device solve
    def solve_device(self, denv, d_state, dt, rtol, atol, opts: Optional[Opts] = None,
                     d_status=None, d_stats=None):
        """camp_solve_device on torch tensors (in place on d_state). Returns d_status."""
        import torch
        n = d_state.shape[0]
        if d_status is None:
            d_status = torch.empty(n, dtype=torch.int32, device=d_state.device)
        e = denv.c_env()
        _check(_lib.camp_solve_device(self.h, n, _ptr(d_state), C.byref(e), dt, rtol, atol,
                                      None if opts is None else C.byref(opts), _ptr(d_status),
                                      _ptr(d_stats), _stream()))
        return d_status

    def solve_device_noalloc(self, denv, d_state, dt, rtol, atol, opts: Optional[Opts] = None,
                             d_status=None, d_stats=None):
        """camp_solve_device_noalloc on torch tensors (in place on d_state); d_status is
        required (allocate it beforehand). Returns d_status."""
        e = denv.c_env()
        _check(_lib.camp_solve_device_noalloc(self.h, d_state.shape[0], _ptr(d_state), C.byref(e),
                                              dt, rtol, atol, None if opts is None else C.byref(opts),
                                              _ptr(d_status), _ptr(d_stats), _stream()))
        return d_status

    def rate_constants(self, denv, n_cells):
        import torch
        k = torch.empty((n_cells, self.n_rxn), dtype=torch.float64, device="cuda")
        e = denv.c_env()
        _check(_lib.camp_rate_constants_device(self.h, n_cells, C.byref(e), _ptr(k), _stream()))
        return k

    def forcing(self, d_k, d_y):
        import torch
        f = torch.empty_like(d_y)
        _check(_lib.camp_forcing_device(self.h, d_y.shape[0], _ptr(d_k), _ptr(d_y), _ptr(f), _stream()))
        return f

    def newton_matrix(self, d_k, d_y, gamma):
        import torch
        m = torch.empty((d_y.shape[0], self.nnz), dtype=torch.float64, device=d_y.device)
        _check(_lib.camp_newton_matrix_device(self.h, d_y.shape[0], _ptr(d_k), _ptr(d_y),
                                              float(gamma), _ptr(m), _stream()))
        return m

    def lu_factor(self, d_m):
        _check(_lib.camp_lu_factor_device(self.h, d_m.shape[0], _ptr(d_m), _stream()))
        return d_m

    def lu_solve(self, d_lu, d_b):
        _check(_lib.camp_lu_solve_device(self.h, d_b.shape[0], _ptr(d_lu), _ptr(d_b), _stream()))
        return d_b


class Plan:
    """A device solve captured once as a HIP graph (wraps camp_plan); the tensors are fixed
    in the plan and read at every replay."""

    def __init__(self, mech: Mech, denv: DeviceEnv, d_state, dt, rtol, atol,
                 opts: Optional[Opts] = None, d_status=None, d_stats=None):
        import torch
        n = d_state.shape[0]
        if d_status is None:
            d_status = torch.empty(n, dtype=torch.int32, device=d_state.device)
        self._keep = (mech, denv, d_state, d_status, d_stats, opts)
        self.d_status = d_status
        e = denv.c_env()
        h = C.c_void_p()
        _check(_lib.camp_plan_create(mech.h, n, _ptr(d_state), C.byref(e), dt, rtol, atol,
                                     None if opts is None else C.byref(opts), _ptr(d_status),
                                     _ptr(d_stats), _stream(), C.byref(h)))
        self.h = h

    def launch(self):
        _check(_lib.camp_plan_launch(self.h, _stream()))
        return self.d_status

    def close(self):
        if getattr(self, "h", None):
            _lib.camp_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_failed(d_status):
    n = C.c_int(0)
    _check(_lib.camp_count_failed(d_status.shape[0], _ptr(d_status), C.byref(n), _stream()))
    return n.value


def probe_copy(mib=2048, reps=10):
    """Sustained device copy bandwidth, GB/s (bytes read plus written)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    v = C.c_double(0)
    _check(_lib.camp_probe_copy(_ptr(a), _ptr(b), n, reps, _stream(), C.byref(v)))
    return v.value


def probe_fma(blocks=256 * 16, iters=20000):
    """Sustained FP64 FMA rate, TFLOP/s."""
    import torch
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    v = C.c_double(0)
    _check(_lib.camp_probe_fma(_ptr(sink), blocks, iters, _stream(), C.byref(v)))
    return v.value


def _host_env(env):
    def f(a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    ni = env.radius.shape[1] if env.radius is not None and env.radius.ndim == 2 else 0
    return [f(env.T), f(env.P), f(env.cos_sza), f(env.radius) if ni else None,
            f(env.mass) if ni else None, f(env.rate_override)]


class DeviceEnv:
    """Torch-device copies of an Environment (keeps the tensors alive)."""

    def __init__(self, env, device="cuda"):
        import torch
        arrs = _host_env(env)
        self.t = [None if a is None else torch.from_numpy(a).to(device) for a in arrs]

    def c_env(self):
        return Env(*[None if t is None else t.data_ptr() for t in self.t])

    def head(self, n):
        """The first n cells, sharing this environment's device memory."""
        v = DeviceEnv.__new__(DeviceEnv)
        v.t = [None if t is None else t[:n] for t in self.t]
        return v


class Server:
    """Continuous-batching request server (wraps camp_server)."""

    def __init__(self, max_bytes=0, max_inflight=8):
        h = C.c_void_p()
        _check(_lib.camp_serve_create(int(max_bytes), int(max_inflight), C.byref(h)))
        self.h = h

    def submit(self, mech: Mech, denv: DeviceEnv, d_state, dt, rtol, atol, d_status,
               opts: Optional[Opts] = None):
        e = denv.c_env()
        t = C.c_longlong(0)
        _check(_lib.camp_serve_submit(self.h, mech.h, d_state.shape[0], _ptr(d_state), C.byref(e),
                                      dt, rtol, atol, None if opts is None else C.byref(opts),
                                      _ptr(d_status), C.byref(t)))
        return t.value

    def poll(self, ticket):
        done, nf, lat = C.c_int(0), C.c_int(0), C.c_double(0)
        _check(_lib.camp_serve_poll(self.h, ticket, C.byref(done), C.byref(nf), C.byref(lat)))
        return bool(done.value), nf.value, lat.value

    def wait(self, ticket):
        _check(_lib.camp_serve_wait(self.h, ticket))

    def progress(self):
        a, b = C.c_int(0), C.c_int(0)
        _check(_lib.camp_serve_progress(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "h", None):
            _lib.camp_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
