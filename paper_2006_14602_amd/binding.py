"""Thin Python binding of libpma.so (include/pma.h): argument marshalling only.

Every step of the mesh computation runs in the HIP library; PyTorch is used for device memory
(the arena comes from torch's caching allocator) and for caller-owned device buffers and
streams.  There is no fallback: if the built library is missing, load() raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref
from ctypes import POINTER, c_double, c_int, c_size_t, c_uint64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpma.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pma.h")

PMA_OK, PMA_E_INVAL, PMA_E_NOMEM, PMA_E_HIP, PMA_E_TANGLED, PMA_E_NONFINITE, PMA_E_BUDGET, \
    PMA_E_NOTFOUND, PMA_E_BUSY = 0, -1, -2, -3, -4, -5, -6, -7, -8
PRECISION = {"fp64": 0, "fp32": 1, "split16": 2}
EXEC = {"batched": 0, "plain": 1}
PENDING, RUNNING, DONE, FAILED = 0, 1, 2, 3
MON_KIND = {"const": 0, "sech2_radial": 1, "sech2_sine": 2, "gauss_sum": 3, "separable_sech2": 4,
            "arclen_front": 5, "arclen_spiral": 6, "arclen_spheres": 7}


class PmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pma error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int * 3), ("lo", c_double * 3), ("hi", c_double * 3)]


class Monitor(ctypes.Structure):
    _fields_ = [("kind", c_int), ("nbumps", c_int), ("amp", c_double), ("k", c_double), ("r0", c_double),
                ("c", c_double * 3), ("amp_axes", c_double * 3), ("k_axes", c_double * 3),
                ("bamp", c_double * 9), ("bw", c_double * 9), ("bc", (c_double * 3) * 9), ("twist", c_double),
                ("theta", c_double)]


class Time(ctypes.Structure):
    _fields_ = [("dt", c_double), ("gamma", c_double), ("tol", c_double), ("max_steps", c_int),
                ("precision", c_int), ("resid_every", c_int), ("exec", c_int)]


class DD(ctypes.Structure):
    _fields_ = [("parts", c_int * 3), ("overlap_cells", c_int * 3), ("mode", c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("steps_done", c_int), ("status", c_int), ("final_resid", c_double), ("min_det", c_double),
                ("min_cell", c_double), ("theta", c_double), ("ms_total", c_double), ("ms_queue", c_double),
                ("quality_e2", c_double), ("quality_emax", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("march", c_int), ("persistent", c_int), ("eight_max", c_int), ("lbasis_max", c_int),
                ("step_ms", c_double), ("from_cache", c_int), ("candidates", c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("grid", Grid), ("dd", DD), ("mon", Monitor), ("time", Time), ("arrival_s", c_double),
                ("psi0", POINTER(c_double)), ("want_psi", c_int)]


ALLOC_CB = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
FREE_CB = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)

_lib = None


def declared_symbols():
    """Function names declared in include/pma.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(pma_\w+)\s*\(", text, flags=re.M)))


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with __graft_entry__.build()")
    # torch first: it brings its own HIP runtime under the same soname as the one the library links,
    # and a process holds one of them, whichever loads first; torch's CUDA state fails to come up on
    # the other one
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.pma_last_error.restype = ctypes.c_char_p
    L.pma_create.argtypes = [c_int, c_size_t, POINTER(c_void_p)]
    L.pma_destroy.argtypes = [c_void_p]
    L.pma_set_allocator.argtypes = [c_void_p, ALLOC_CB, FREE_CB, c_void_p]
    L.pma_solve_subdomain.argtypes = [c_void_p, POINTER(Grid), POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                      POINTER(Monitor), POINTER(Time), c_void_p, c_void_p, POINTER(Stats)]
    L.pma_solve_subdomain_noalloc.argtypes = L.pma_solve_subdomain.argtypes
    L.pma_dd_mesh.argtypes = [c_void_p, POINTER(Grid), POINTER(DD), POINTER(Monitor), POINTER(Time),
                              POINTER(c_double), POINTER(c_double), POINTER(c_double), POINTER(Stats)]
    L.pma_dd_mesh_batch.argtypes = [c_void_p, c_int, POINTER(Request), POINTER(POINTER(c_double)), POINTER(Stats)]
    L.pma_submit.argtypes = [c_void_p, POINTER(Request), POINTER(c_uint64)]
    L.pma_poll.argtypes = [c_void_p, c_uint64, POINTER(c_int), POINTER(c_double), POINTER(Stats)]
    L.pma_poll_psi.argtypes = [c_void_p, c_uint64, POINTER(c_int), POINTER(c_double), POINTER(c_double),
                               POINTER(Stats)]
    L.pma_server_info.argtypes = [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_size_t)]
    L.pma_request_bytes.argtypes = [POINTER(Request), POINTER(c_size_t)]
    L.pma_partition.argtypes = [POINTER(Grid), POINTER(DD), c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int)]
    L.pma_sweep_levels.argtypes = [POINTER(Grid), POINTER(DD), c_int, POINTER(c_int), POINTER(c_int)]
    L.pma_theta.argtypes = [POINTER(Grid), POINTER(Monitor), POINTER(c_double)]
    L.pma_plan_create.argtypes = [c_void_p, c_int, POINTER(Request), POINTER(c_void_p)]
    L.pma_plan_step.argtypes = [c_void_p, c_int]
    L.pma_plan_sync.argtypes = [c_void_p]
    L.pma_plan_phase_times.argtypes = [c_void_p, c_int, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                       c_int, POINTER(c_int)]
    L.pma_plan_autotune.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_double), c_int, POINTER(c_int)]
    L.pma_plan_set_march.argtypes = [c_void_p, c_int]
    L.pma_plan_set_fusion.argtypes = [c_void_p, c_int]
    L.pma_plan_set_wide_strips.argtypes = [c_void_p, c_int]
    L.pma_plan_set_persistent.argtypes = [c_void_p, c_int]
    L.pma_plan_tune.argtypes = [c_void_p, c_int, ctypes.c_char_p, POINTER(Tuning)]
    L.pma_plan_mesh.argtypes = [c_void_p, c_int, POINTER(c_double), POINTER(Stats)]
    L.pma_plan_destroy.argtypes = [c_void_p]
    for f in declared_symbols():
        if f != "pma_last_error":
            getattr(L, f).restype = c_int
    _lib = L
    return L


def _check(rc):
    if rc != PMA_OK:
        raise PmaError(rc, load().pma_last_error().decode())


# ---------------------------------------------------------------------------------------------
# conversions from the workload dictionaries
# ---------------------------------------------------------------------------------------------

def make_grid(g: dict) -> Grid:
    G = Grid()
    G.dim = g["dim"]
    for k in range(g["dim"]):
        G.n[k] = int(g["n"][k])
        G.lo[k] = float(g["lo"][k])
        G.hi[k] = float(g["hi"][k])
    for k in range(g["dim"], 3):
        G.n[k] = 1
    return G


def make_monitor(m: dict, theta: float = 0.0) -> Monitor:
    M = Monitor()
    M.kind = MON_KIND[m["kind"]]
    M.amp = float(m.get("amp", 1.0)) if m["kind"] in ("const", "sech2_radial", "sech2_sine", "arclen_spiral") else 0.0
    M.k = float(m.get("k", 0.0))
    M.r0 = float(m.get("r0", 0.0))
    if m["kind"] == "arclen_front":
        M.k = float(m["eps"])
        M.r0 = float(m.get("offset", 1.0))
    if m["kind"] == "arclen_spiral":
        M.twist = float(m["twist"])
    if m["kind"] == "arclen_spheres":
        M.nbumps = len(m["bc"])
        for b in range(M.nbumps):
            for i, v in enumerate(m["bc"][b][:3]):
                M.bc[b][i] = float(v)
    for i, v in enumerate(m.get("c", [])[:3]):
        M.c[i] = float(v)
    if m["kind"] == "separable_sech2":
        for i in range(len(m["amp_axes"])):
            M.amp_axes[i] = float(m["amp_axes"][i])
            M.k_axes[i] = float(m["k_axes"][i])
    if m["kind"] == "gauss_sum":
        M.nbumps = len(m["bamp"])
        for b in range(M.nbumps):
            M.bamp[b] = float(m["bamp"][b])
            M.bw[b] = float(m["bw"][b])
            for i, v in enumerate(m["bc"][b][:3]):
                M.bc[b][i] = float(v)
    M.theta = float(theta or m.get("theta", 0.0) or 0.0)
    return M


def make_time(t: dict, precision="fp32", exec_="batched", tol=0.0, resid_every=10) -> Time:
    T = Time()
    T.dt = float(t["dt"])
    T.gamma = float(t["gamma"])
    T.tol = float(t.get("tol", tol))
    T.max_steps = int(t["steps"])
    T.precision = PRECISION[precision]
    T.resid_every = int(t.get("resid_every", resid_every))
    T.exec = EXEC[exec_]
    return T


DD_MODE = {"parallel": 0, "alternating": 1, "coloured": 2}


def make_dd(dd, dim) -> DD:
    D = DD()
    for k in range(3):
        D.parts[k] = 1
        D.overlap_cells[k] = 0
    if dd:
        for k in range(dim):
            D.parts[k] = int(dd["parts"][k])
            D.overlap_cells[k] = int(dd["overlap"][k])
    D.mode = DD_MODE[(dd or {}).get("mode", "parallel")]
    return D


def make_request(w: dict, precision="fp32", exec_="batched", psi0=None, want_psi=False) -> Request:
    """psi0: optional float64 array of the grid's shape (warm start); the caller keeps it alive
    for the duration of the call that reads it."""
    R = Request()
    R.grid = make_grid(w["grid"])
    R.dd = make_dd(w.get("dd"), w["grid"]["dim"])
    R.mon = make_monitor(w["monitor"])
    R.time = make_time(w["time"], precision, exec_)
    R.arrival_s = float(w.get("arrival_s", 0.0))
    if psi0 is not None:
        assert psi0.dtype == np.float64 and psi0.flags.c_contiguous and psi0.shape == tuple(w["grid"]["n"])
        R.psi0 = _dptr(psi0)
    R.want_psi = 1 if want_psi else 0
    return R


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


# ---------------------------------------------------------------------------------------------
# host-only helpers
# ---------------------------------------------------------------------------------------------

def partition(grid: dict, dd: dict | None):
    L = load()
    G = make_grid(grid)
    D = make_dd(dd, grid["dim"])
    n = c_int()
    _check(L.pma_partition(ctypes.byref(G), ctypes.byref(D), 0, ctypes.byref(n), None, None))
    ranges = (c_int * (6 * n.value))()
    faces = (c_int * (6 * n.value))()
    _check(L.pma_partition(ctypes.byref(G), ctypes.byref(D), n.value, ctypes.byref(n), ranges, faces))
    return np.array(ranges[:], dtype=np.int64).reshape(n.value, 6), np.array(faces[:], dtype=np.int64).reshape(n.value, 6)


def sweep_levels(grid: dict, dd: dict) -> np.ndarray:
    L = load()
    G = make_grid(grid)
    D = make_dd(dd, grid["dim"])
    n = c_int()
    _check(L.pma_sweep_levels(ctypes.byref(G), ctypes.byref(D), 0, ctypes.byref(n), None))
    out = (c_int * n.value)()
    _check(L.pma_sweep_levels(ctypes.byref(G), ctypes.byref(D), n.value, ctypes.byref(n), out))
    return np.array(out[:], dtype=np.int64)


def request_bytes(w: dict, precision="fp32") -> int:
    """Device bytes the request occupies while served (state plus every DCT basis it uses)."""
    L = load()
    R = make_request(w, precision, "batched")
    out = c_size_t()
    _check(L.pma_request_bytes(ctypes.byref(R), ctypes.byref(out)))
    return out.value


def theta(grid: dict, mon: dict) -> float:
    L = load()
    out = c_double()
    G, M = make_grid(grid), make_monitor(mon)
    _check(L.pma_theta(ctypes.byref(G), ctypes.byref(M), ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------------------------

_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    # release device memory while torch's allocator is still alive
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A library context on one GPU.  The device arena (budget bytes) comes from torch's caching
    allocator unless use_torch_allocator is False."""

    def __init__(self, device: int = 0, budget_bytes: int = 8 << 30, use_torch_allocator: bool = True):
        L = load()
        self._L = L
        self.device = device
        if use_torch_allocator:
            import torch
            # torch's CUDA state is set up here, on the caller's thread: the library's serving
            # thread may be the first to allocate through the callbacks below
            torch.cuda.init()
        h = c_void_p()
        _check(L.pma_create(device, budget_bytes, ctypes.byref(h)))
        self.h = h
        self._cbs = None
        if use_torch_allocator:
            alloc = torch.cuda.caching_allocator_alloc
            delete = torch.cuda.caching_allocator_delete

            def _alloc(size, stream, user):
                try:
                    return alloc(int(size), device=device)
                except Exception:
                    return None

            def _free(ptr, stream, user):
                try:
                    delete(int(ptr))
                except Exception:  # interpreter shutdown: torch may already be torn down
                    pass

            self._cbs = (ALLOC_CB(_alloc), FREE_CB(_free))
            _check(L.pma_set_allocator(self.h, self._cbs[0], self._cbs[1], None))
        _LIVE.add(self)

    def close(self):
        if self.h:
            _check(self._L.pma_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- whole mesh ------------------------------------------------------------------------
    def dd_mesh(self, w: dict, precision="fp32", exec_="batched", psi0=None, want_psi=False, tol=0.0,
                resid_every=10, theta_override=0.0):
        """Adaptive mesh of workload w: returns (mesh[d, *n], psi or None, stats dict)."""
        g = w["grid"]
        n = tuple(g["n"])
        G = make_grid(g)
        D = make_dd(w.get("dd"), g["dim"])
        M = make_monitor(w["monitor"], theta_override)
        T = make_time(w["time"], precision, exec_, tol, resid_every)
        mesh = np.empty((g["dim"],) + n, dtype=np.float64)
        psi = np.empty(n, dtype=np.float64) if want_psi else None
        p0 = None
        if psi0 is not None:
            p0 = np.ascontiguousarray(psi0, dtype=np.float64)
            assert p0.shape == n
        st = Stats()
        _check(self._L.pma_dd_mesh(self.h, ctypes.byref(G), ctypes.byref(D), ctypes.byref(M), ctypes.byref(T),
                                   _dptr(p0) if p0 is not None else None, _dptr(mesh),
                                   _dptr(psi) if psi is not None else None, ctypes.byref(st)))
        return mesh, psi, st.as_dict()

    def dd_mesh_batch(self, ws, precision="fp32", exec_="batched", psi0s=None):
        """Many meshes advanced together; returns (list of meshes, list of stats dicts).
        psi0s: optional list of warm starts (None entries: Psi^0 = |xi|^2/2)."""
        count = len(ws)
        reqs = (Request * count)()
        outs = []
        keep = [None if p is None else np.ascontiguousarray(p, dtype=np.float64) for p in (psi0s or [None] * count)]
        for i, w in enumerate(ws):
            reqs[i] = make_request(w, precision, exec_, psi0=keep[i])
            outs.append(np.empty((w["grid"]["dim"],) + tuple(w["grid"]["n"]), dtype=np.float64))
        ptrs = (POINTER(c_double) * count)(*[_dptr(o) for o in outs])
        stats = (Stats * count)()
        _check(self._L.pma_dd_mesh_batch(self.h, count, reqs, ptrs, stats))
        return outs, [s.as_dict() for s in stats]

    # -- one subdomain ---------------------------------------------------------------------
    def solve_subdomain(self, grid: dict, lo, hi, faces, mon: dict, time: dict, psi_dev, stream=None,
                        precision="fp32", exec_="batched", noalloc=False):
        """Advance one subdomain in place.  psi_dev: a contiguous float64 CUDA tensor of the
        subdomain's nodes holding Psi (artificial faces hold the Dirichlet data).  noalloc: through
        pma_solve_subdomain_noalloc (state in the library's fixed device scratch)."""
        import torch
        assert psi_dev.is_cuda and psi_dev.dtype == torch.float64 and psi_dev.is_contiguous()
        d = grid["dim"]
        shape = tuple(hi[k] - lo[k] + 1 for k in range(d))
        assert tuple(psi_dev.shape) == shape, (psi_dev.shape, shape)
        G = make_grid(grid)
        lo3 = (c_int * 3)(*(list(lo) + [0] * (3 - d)))
        hi3 = (c_int * 3)(*(list(hi) + [0] * (3 - d)))
        f6 = (c_int * 6)(*(list(faces) + [0] * (6 - len(faces))))
        M = make_monitor(mon)
        T = make_time(time, precision, exec_)
        st = Stats()
        s = stream if stream is not None else torch.cuda.current_stream(psi_dev.device)
        fn = self._L.pma_solve_subdomain_noalloc if noalloc else self._L.pma_solve_subdomain
        _check(fn(self.h, ctypes.byref(G), lo3, hi3, f6, ctypes.byref(M), ctypes.byref(T),
                  c_void_p(psi_dev.data_ptr()), c_void_p(s.cuda_stream), ctypes.byref(st)))
        return st.as_dict()

    # -- serving ---------------------------------------------------------------------------
    def submit(self, w: dict, precision="fp32", psi0=None, want_psi=False) -> int:
        """psi0: optional warm start (float64 array of the grid's shape, copied by the call);
        want_psi: keep the final Psi for poll_psi."""
        if psi0 is not None:
            psi0 = np.ascontiguousarray(psi0, dtype=np.float64)
        R = make_request(w, precision, "batched", psi0=psi0, want_psi=want_psi)
        t = c_uint64()
        _check(self._L.pma_submit(self.h, ctypes.byref(R), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, shape=None):
        """(state, mesh or None, stats or None).  shape = (dim, *n) to receive the mesh."""
        stt = c_int()
        mesh = np.empty(shape, dtype=np.float64) if shape is not None else None
        st = Stats()
        _check(self._L.pma_poll(self.h, ticket, ctypes.byref(stt), _dptr(mesh) if mesh is not None else None,
                                ctypes.byref(st)))
        if stt.value in (DONE, FAILED):
            d = st.as_dict()
            if stt.value == FAILED:
                d["error"] = self._L.pma_last_error().decode()
            return stt.value, (mesh if stt.value == DONE else None), d
        return stt.value, None, None

    def poll_psi(self, ticket: int, shape):
        """(state, mesh or None, psi or None, stats or None) of a request submitted with
        want_psi; shape = (dim, *n)."""
        stt = c_int()
        mesh = np.empty(shape, dtype=np.float64)
        psi = np.empty(shape[1:], dtype=np.float64)
        st = Stats()
        _check(self._L.pma_poll_psi(self.h, ticket, ctypes.byref(stt), _dptr(mesh), _dptr(psi), ctypes.byref(st)))
        if stt.value == DONE:
            return stt.value, mesh, psi, st.as_dict()
        if stt.value == FAILED:
            return stt.value, None, None, st.as_dict()
        return stt.value, None, None, None

    def server_info(self):
        q, r, f = c_int(), c_int(), c_int()
        b = c_size_t()
        _check(self._L.pma_server_info(self.h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f), ctypes.byref(b)))
        return {"queued": q.value, "running": r.value, "finished": f.value, "bytes_in_use": b.value}


PHASES = ["transmit", "stencil", "euler", "fwd_last", "fwd_mid", "pair0", "inv_mid", "inv_last", "resid"]


class Plan:
    """Requests kept resident on the device, stepped on demand (pma_plan_*)."""

    def __init__(self, ctx: Context, ws, precision="fp32", exec_="batched"):
        self._L = ctx._L
        self.ctx = ctx
        self.ws = list(ws)
        reqs = (Request * len(self.ws))()
        for i, w in enumerate(self.ws):
            reqs[i] = make_request(w, precision, exec_)
        h = c_void_p()
        _check(self._L.pma_plan_create(ctx.h, len(self.ws), reqs, ctypes.byref(h)))
        self.h = h

    def step(self, n: int):
        _check(self._L.pma_plan_step(self.h, int(n)))

    def sync(self):
        _check(self._L.pma_plan_sync(self.h))

    def phase_times(self, n: int):
        ms = (c_double * 9)()
        fl = (c_double * 9)()
        by = (c_double * 9)()
        nph = c_int()
        _check(self._L.pma_plan_phase_times(self.h, int(n), ms, fl, by, 9, ctypes.byref(nph)))
        return {PHASES[i]: {"ms": ms[i], "flops": fl[i], "bytes": by[i]} for i in range(nph.value)}

    def autotune(self, reps: int = 10):
        """Stencil march length picked by timing (pma_plan_autotune): (choice, [ms per candidate
        march 1, 2, 4, .. capped at the longest useful one])."""
        march = c_int()
        ms = (c_double * 8)()
        nc = c_int()
        _check(self._L.pma_plan_autotune(self.h, int(reps), ctypes.byref(march), ms, 8, ctypes.byref(nc)))
        return march.value, [ms[k] for k in range(nc.value)]

    def set_march(self, march: int):
        _check(self._L.pma_plan_set_march(self.h, int(march)))

    def set_fusion(self, on: bool):
        _check(self._L.pma_plan_set_fusion(self.h, 1 if on else 0))

    def set_wide_strips(self, on: bool):
        _check(self._L.pma_plan_set_wide_strips(self.h, 1 if on else 0))

    def tune(self, reps: int = 10, cache_path=None):
        """Launch configuration picked by timing whole steps (pma_plan_tune); cache_path: the
        tuning cache file (None: no cache)."""
        t = Tuning()
        _check(self._L.pma_plan_tune(self.h, int(reps), None if cache_path is None else str(cache_path).encode(),
                                     ctypes.byref(t)))
        return t.as_dict()

    def set_persistent(self, on: bool):
        _check(self._L.pma_plan_set_persistent(self.h, 1 if on else 0))

    def mesh(self, i: int = 0):
        w = self.ws[i]
        out = np.empty((w["grid"]["dim"],) + tuple(w["grid"]["n"]), dtype=np.float64)
        st = Stats()
        _check(self._L.pma_plan_mesh(self.h, i, _dptr(out), ctypes.byref(st)))
        return out, st.as_dict()

    def close(self):
        if self.h:
            _check(self._L.pma_plan_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
