"""Binding of the continuous-batching engine (``include/richards_serve.h``).

Argument marshalling only: admission, scheduling, the per-request state
machine and every arithmetic step run in the native library.  PyTorch supplies
the device arena, the engine's stream and the request state tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import RS_EBUSY, check, constitutive, grid_desc, lib

RS_REQ_RUNNING, RS_REQ_FINISHED, RS_REQ_FAILED = 1, 3, 4


class EngineOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("max_slots", C.c_int),
                ("max_wide_levels", C.c_int), ("tail_nodes", C.c_int), ("nu1", C.c_int),
                ("nu2", C.c_int), ("nu_coarse", C.c_int), ("max_corrections", C.c_int),
                ("tol_abs", C.c_double), ("tol_rel", C.c_double), ("stagnation", C.c_int),
                ("rounds_per_tick", C.c_int), ("use_graph", C.c_int)]


class RequestStats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("state", C.c_int), ("status", C.c_int),
                ("steps", C.c_int), ("corrections", C.c_int),
                ("max_step_corrections", C.c_int), ("res", C.c_double)]


_bound = False


def _lib():
    global _bound
    L = lib()
    if not _bound:
        vp, I, Z = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_size_t)
        O = C.POINTER(EngineOpts)
        L.rs_engine_default_opts.argtypes = [O]
        L.rs_engine_default_opts.restype = None
        L.rs_engine_control_bytes.argtypes = [O, Z]
        L.rs_engine_request_bytes.argtypes = [O, vp, Z]
        L.rs_engine_create.argtypes = [O, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.rs_engine_submit.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, C.c_int, I]
        L.rs_engine_tick.argtypes = [vp, I, C.c_int, I, I]
        L.rs_engine_fetch.argtypes = [vp, C.c_int, vp, C.POINTER(RequestStats)]
        L.rs_engine_capacity.argtypes = [vp, Z, I]
        L.rs_engine_destroy.argtypes = [vp]
        L.rs_engine_destroy.restype = None
        _bound = True
    return L


def engine_opts(**kw) -> EngineOpts:
    o = EngineOpts()
    _lib().rs_engine_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def control_bytes(opts: EngineOpts) -> int:
    out = C.c_size_t()
    check(_lib().rs_engine_control_bytes(C.byref(opts), C.byref(out)))
    return out.value


def request_bytes(opts: EngineOpts, grid) -> int:
    out = C.c_size_t()
    d = grid_desc(grid)
    check(_lib().rs_engine_request_bytes(C.byref(opts), C.byref(d), C.byref(out)))
    return out.value


class Engine:
    """A continuous-batching engine over one device arena.

    ``submit`` admits a request (``None`` when it does not fit right now),
    ``tick`` runs correction rounds and returns the tickets that finished,
    ``fetch`` returns a finished request's final state and statistics and
    releases its memory.
    """

    def __init__(self, arena_bytes: int, opts: EngineOpts | None = None, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda" if device is None else device)
        self.opts = opts if opts is not None else engine_opts()
        self.stream = torch.cuda.Stream(self.device)   # default priority
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        self._arena_ptr = base + (-base) % 256
        self.arena_bytes = arena_bytes
        h = C.c_void_p()
        torch.cuda.current_stream(self.device).synchronize()
        check(_lib().rs_engine_create(C.byref(self.opts), C.c_void_p(self._arena_ptr),
                                      arena_bytes, C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)))
        self.h = h
        self._pending = []
        self._shape = {}
        self._done = (C.c_int * 4096)()

    def close(self):
        if getattr(self, "h", None):
            _lib().rs_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, w, nsteps=None):
        """Admit workload w (its grid, law, psi0, dt, order); the ticket, or
        None when no slot or arena space is free."""
        torch = self.torch
        d = grid_desc(w.grid)
        c, keep = constitutive(w.law, w.Ks_field, w.soils, w.soil_id)
        with torch.cuda.stream(self.stream):
            psi0 = torch.as_tensor(np.ascontiguousarray(w.psi0, dtype=np.float64)).to(
                self.device)
        t = C.c_int()
        code = _lib().rs_engine_submit(self.h, C.byref(d), C.byref(c), C.c_void_p(psi0.data_ptr()),
                                       w.dt, w.order, w.steps if nsteps is None else nsteps,
                                       C.byref(t))
        del keep
        if code == RS_EBUSY:
            return None
        check(code)
        self._pending.append(psi0)
        self._shape[t.value] = tuple(w.grid.shape)
        return t.value

    def tick(self):
        """Run the configured correction rounds; (finished tickets, running)."""
        nd, na = C.c_int(), C.c_int()
        check(_lib().rs_engine_tick(self.h, self._done, len(self._done), C.byref(nd),
                                    C.byref(na)))
        self._pending.clear()
        return [self._done[i] for i in range(nd.value)], na.value

    def fetch(self, ticket, want_psi=True):
        """(final psi as a device tensor or None, stats) of a finished request."""
        torch = self.torch
        st = RequestStats()
        st.struct_size = C.sizeof(RequestStats)
        out = None
        if want_psi:
            with torch.cuda.stream(self.stream):
                out = torch.empty(self._shape[ticket], dtype=torch.float64, device=self.device)
        check(_lib().rs_engine_fetch(self.h, ticket,
                                     C.c_void_p(out.data_ptr()) if out is not None else None,
                                     C.byref(st)))
        del self._shape[ticket]
        return out, st

    def capacity(self):
        fb, fs = C.c_size_t(), C.c_int()
        check(_lib().rs_engine_capacity(self.h, C.byref(fb), C.byref(fs)))
        return fb.value, fs.value

    def synchronize(self):
        self.stream.synchronize()


def run_stream(E: Engine, reqs, arrivals=None, keep=()):
    """Serve ``reqs`` in arrival order (FCFS admission) against the wall clock.

    ``arrivals``: seconds after the start at which request q arrives (all at 0
    when None).  A request is submitted once it has arrived and the requests
    before it are admitted; it waits while the engine has no room.  Returns
    (arrival, completion, stats, kept): completion times in seconds after the
    start (taken when the tick that reports the request returns), per-request
    (status, steps, corrections, max corrections in a step), and the final
    states of the requests listed in ``keep`` as device tensors."""
    import time
    n = len(reqs)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    comp = np.full(n, np.nan)
    stats = [None] * n
    kept = {}
    keep = set(keep)
    ticket_of = {}
    nxt = 0
    finished = 0
    t0 = time.perf_counter()
    while finished < n:
        now = time.perf_counter() - t0
        while nxt < n and arr[nxt] <= now:
            t = E.submit(reqs[nxt])
            if t is None:
                if not ticket_of:
                    raise RuntimeError("request %d does not fit an empty engine" % nxt)
                break
            ticket_of[t] = nxt
            nxt += 1
        if not ticket_of:
            time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
            continue
        done, _ = E.tick()
        tdone = time.perf_counter() - t0
        for t in done:
            q = ticket_of.pop(t)
            psi, st = E.fetch(t, want_psi=q in keep)
            if psi is not None:
                kept[q] = psi
            comp[q] = tdone
            stats[q] = (st.status, st.steps, st.corrections, st.max_step_corrections)
            finished += 1
    E.synchronize()
    return arr, comp, stats, kept
