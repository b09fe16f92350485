"""Python binding of ``libocm.so`` (the C ABI of include/ocm.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  Tensors must be contiguous device tensors on the current
GPU; calls are enqueued on torch's current stream.  There is no CPU fallback:
if the library is missing every call raises.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
from fractions import Fraction

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libocm.so")

OCM_OK = 0
OCM_E_INVALID_ARG = -1
OCM_E_BAD_CSR = -2
OCM_E_NO_OUT_EDGE = -3
OCM_E_NOT_STRONGLY_CONNECTED = -4
OCM_E_OVERFLOW = -5
OCM_E_CAPACITY = -6
OCM_E_NOT_CONVERGED = -7
OCM_E_WORKSPACE = -8
OCM_E_HIP = -9

OCM_W_I32, OCM_W_I64 = 0, 1
OCM_F_TIE, OCM_F_TIE_UNCHECKED, OCM_F_TIGHT_EDGES, OCM_F_INT128 = 1, 2, 4, 8

PHASES = ("validate", "sweep", "tiescan", "cycles", "select", "conn_pull", "conn_mark",
          "conn_claim", "reverse", "values", "fast", "result")


class OCMError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        super().__init__(f"ocm status {status}: {message}")
        self.status = status
        self.message = message


class Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("w", C.c_void_p), ("wtype", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("p", C.c_int64), ("q", C.c_int64), ("cycle_len", C.c_int64),
                ("source", C.c_int32), ("iterations", C.c_int32), ("flags", C.c_uint32),
                ("connect_rounds", C.c_int32), ("jump_rounds", C.c_int32),
                ("fast_iters", C.c_int32), ("W", C.c_int64), ("L", C.c_int64),
                ("tight_edges", C.c_int64), ("push_frontier", C.c_int64),
                ("push_in_edges", C.c_int64), ("general_iters", C.c_int32),
                ("value_rounds", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * len(PHASES)), ("launches", C.c_int32 * len(PHASES)),
                ("bytes", C.c_double * len(PHASES))]

    def as_dict(self):
        """{class: (milliseconds, launches, algorithmic bytes)}"""
        return {p: (self.ms[i], self.launches[i], self.bytes[i]) for i, p in enumerate(PHASES)}


class Options(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("validate", C.c_int32), ("schedule", C.c_int32),
                ("tie_check", C.c_int32), ("fast_path", C.c_int32),
                ("connect_mode", C.c_int32), ("tile", C.c_int32), ("init_policy", C.c_void_p),
                ("policy_out", C.c_void_p), ("potential_out", C.c_void_p),
                ("profile", C.POINTER(Profile)), ("int128_values", C.c_int32),
                ("multichain", C.c_int32)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OCMError(OCM_E_HIP, f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1111_0627_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        G, O = C.POINTER(Graph), C.POINTER(Options)
        L.ocm_default_options.argtypes = [O]
        L.ocm_workspace_size.argtypes = [G, O]
        L.ocm_workspace_size.restype = C.c_size_t
        for f in (L.ocm_min, L.ocm_max):
            f.argtypes = [G, O, P, C.c_size_t, P, i64, C.POINTER(_Result), P]
            f.restype = C.c_int
        L.ocm_min_noalloc.argtypes = [G, O, P, i64, C.POINTER(_Result), P]
        L.ocm_min_noalloc.restype = C.c_int
        for f in (L.ocm_ratio_min, L.ocm_ratio_max):
            f.argtypes = [G, P, O, P, C.c_size_t, P, i64, C.POINTER(_Result), P]
            f.restype = C.c_int
        L.ocm_general_workspace_size.argtypes = [G]
        L.ocm_general_workspace_size.restype = C.c_size_t
        for f in (L.ocm_min_general, L.ocm_max_general):
            f.argtypes = [G, O, P, C.c_size_t, P, i64, C.POINTER(_Result), C.POINTER(i64), P]
            f.restype = C.c_int
        L.ocm_phase_sweep.argtypes = [G, i32, i32, P, i64, i64, P, i32, P, C.c_size_t,
                                      C.POINTER(i64), P]
        L.ocm_phase_cycles.argtypes = [G, P, P, P, P, C.c_size_t, C.POINTER(i64), P]
        L.ocm_phase_select.argtypes = [G, i32, P, P, P, P, C.c_size_t, C.POINTER(i32),
                                       C.POINTER(i64), C.POINTER(i64), P]
        L.ocm_phase_connect.argtypes = [G, P, i32, P, P, P, C.c_size_t, C.POINTER(i32), P]
        L.ocm_phase_values.argtypes = [G, i32, P, i32, i64, i64, P, P, C.c_size_t,
                                       C.POINTER(i32), P]
        for f in (L.ocm_phase_sweep, L.ocm_phase_cycles, L.ocm_phase_select,
                  L.ocm_phase_connect, L.ocm_phase_values):
            f.restype = C.c_int
        L.ocm_batched_workspace_size.argtypes = [i64, P, P, G, O]
        L.ocm_batched_workspace_size.restype = C.c_size_t
        for f in (L.ocm_min_batched, L.ocm_max_batched):
            f.argtypes = [i64, P, P, G, O, P, C.c_size_t, P, P, P, P, i64, P, P, P, P]
            f.restype = C.c_int
        L.ocm_batched_last_schedule.argtypes = [P, P, P]
        L.ocm_weights_from_f64.argtypes = [i64, P, P, P, C.c_size_t, P]
        L.ocm_weights_from_f64.restype = C.c_int
        L.ocm_adjoint_scatter.argtypes = [i64, P, i64, P, P, P]
        L.ocm_adjoint_scatter.restype = C.c_int
        L.ocm_status_string.argtypes = [C.c_int]
        L.ocm_status_string.restype = C.c_char_p
        L.ocm_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OCM_OK:
        raise OCMError(rc, lib().ocm_last_error().decode())


def _dev(t: torch.Tensor, dtypes, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def make_graph(row_ptr: torch.Tensor, col: torch.Tensor, w: torch.Tensor) -> Graph:
    _dev(row_ptr, (torch.int32,), "row_ptr")
    _dev(col, (torch.int32,), "col")
    _dev(w, (torch.int32, torch.int64), "w")
    if w.numel() != col.numel():
        raise ValueError("w and col must have the same length")
    return Graph(row_ptr.numel() - 1, col.numel(), row_ptr.data_ptr(), col.data_ptr(),
                 w.data_ptr(), OCM_W_I64 if w.dtype == torch.int64 else OCM_W_I32)


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_ws_cache: dict = {}


def workspace(g: Graph, device) -> torch.Tensor:
    """A cached device workspace of at least ocm_workspace_size bytes."""
    need = lib().ocm_workspace_size(C.byref(g), None)
    if need == 0:
        _check(OCM_E_INVALID_ARG)
    key = torch.device(device)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need:
        _ws_cache.pop(key, None)
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def release_workspace():
    _ws_cache.clear()
    _bws_cache.clear()
    _gws_cache.clear()


@dataclasses.dataclass
class Result:
    p: int
    q: int
    cycle_edges: torch.Tensor      # int32 CSR edge positions from the source
    source: int
    iterations: int
    flags: int
    W: int
    L: int
    tight_edges: int
    connect_rounds: int
    jump_rounds: int
    fast_iters: int
    counters: dict = dataclasses.field(default_factory=dict)
    policy: torch.Tensor | None = None
    potential: torch.Tensor | None = None
    profile: dict | None = None

    @property
    def value(self) -> Fraction:
        return Fraction(self.p, self.q)

    @property
    def int128(self) -> bool:
        """True when the solve carried its values in int128."""
        return bool(self.flags & OCM_F_INT128)

    @property
    def tie(self):
        """True / False, or None when the uniqueness test did not decide."""
        if self.flags & OCM_F_TIE:
            return True
        if self.flags & OCM_F_TIE_UNCHECKED:
            return None
        return False


CONNECT_MODES = {"auto": 0, "pull": 1, "push": 2}


def options(max_iters=0, validate=True, schedule=0, tie_check=True, fast_path=True,
            connect="auto", init_policy=None, tile=0, int128=False,
            multichain=False) -> Options:
    o = Options()
    lib().ocm_default_options(C.byref(o))
    o.max_iters, o.validate, o.schedule, o.tile = max_iters, int(validate), schedule, tile
    o.int128_values = int(int128)
    o.multichain = int(multichain)
    o.tie_check, o.fast_path = int(tie_check), int(fast_path)
    o.connect_mode = CONNECT_MODES[connect]
    if init_policy is not None:
        _dev(init_policy, (torch.int32,), "init_policy")
        o.init_policy = init_policy.data_ptr()
    return o


def _solve(fn, row_ptr, col, w, want_policy, want_potential, profile, times=None,
           **opt) -> Result:
    g = make_graph(row_ptr, col, w)
    if times is not None:
        _dev(times, (torch.int32,), "t")
        if times.numel() != g.m:
            raise ValueError("t and col must have the same length")
    dev = col.device
    o = options(**opt)
    pol = torch.empty(g.n, dtype=torch.int32, device=dev) if want_policy else None
    pot = torch.empty(g.n, dtype=torch.int64, device=dev) if want_potential else None
    o.policy_out = pol.data_ptr() if want_policy else None
    o.potential_out = pot.data_ptr() if want_potential else None
    prof = Profile() if profile else None
    if prof is not None:
        o.profile = C.pointer(prof)
    ws = workspace(g, dev)
    cyc = torch.empty(g.n, dtype=torch.int32, device=dev)
    res = _Result()
    if times is None:
        _check(fn(C.byref(g), C.byref(o), C.c_void_p(ws.data_ptr()), ws.numel(),
                  C.c_void_p(cyc.data_ptr()), g.n, C.byref(res), _stream()))
    else:
        _check(fn(C.byref(g), C.c_void_p(times.data_ptr()), C.byref(o),
                  C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(cyc.data_ptr()), g.n,
                  C.byref(res), _stream()))
    counters = dict(push_frontier=res.push_frontier, push_in_edges=res.push_in_edges,
                    general_iters=res.general_iters, value_rounds=res.value_rounds)
    return Result(res.p, res.q, cyc[:res.cycle_len], res.source, res.iterations, res.flags,
                  res.W, res.L, res.tight_edges, res.connect_rounds, res.jump_rounds,
                  res.fast_iters, counters, pol, pot,
                  prof.as_dict() if prof is not None else None)


def min_cycle_mean(row_ptr, col, w, *, want_policy=False, want_potential=False,
                   profile=False, **opt) -> Result:
    """Exact minimum cycle mean and one critical cycle (ocm_min)."""
    return _solve(lib().ocm_min, row_ptr, col, w, want_policy, want_potential, profile, **opt)


# ocm_min_noalloc's scratch per GPU (OCM_NOALLOC_SCRATCH_BYTES in ocm.h)
NOALLOC_SCRATCH_BYTES = 256 << 20


def min_cycle_mean_noalloc(row_ptr, col, w, cycle_out: torch.Tensor, **opt) -> Result:
    """ocm_min without a workspace (ocm_min_noalloc): the library's static
    per-GPU scratch array is used, so the call allocates no device memory.
    ``cycle_out``: caller-owned int32 device tensor for the cycle's edges."""
    g = make_graph(row_ptr, col, w)
    _dev(cycle_out, (torch.int32,), "cycle_out")
    o = options(**opt)
    res = _Result()
    _check(lib().ocm_min_noalloc(C.byref(g), C.byref(o), C.c_void_p(cycle_out.data_ptr()),
                                 cycle_out.numel(), C.byref(res), _stream()))
    counters = dict(push_frontier=res.push_frontier, push_in_edges=res.push_in_edges,
                    general_iters=res.general_iters, value_rounds=res.value_rounds)
    return Result(res.p, res.q, cycle_out[:res.cycle_len], res.source, res.iterations, res.flags,
                  res.W, res.L, res.tight_edges, res.connect_rounds, res.jump_rounds,
                  res.fast_iters, counters)


def max_cycle_mean(row_ptr, col, w, *, want_policy=False, want_potential=False,
                   profile=False, **opt) -> Result:
    """Exact maximum cycle mean and one critical cycle (ocm_max)."""
    return _solve(lib().ocm_max, row_ptr, col, w, want_policy, want_potential, profile, **opt)


def min_cycle_ratio(row_ptr, col, w, t, *, want_policy=False, want_potential=False,
                    profile=False, **opt) -> Result:
    """Exact minimum cycle ratio cost/time and one critical cycle
    (ocm_ratio_min); ``t``: int32 edge times >= 1.  ``W`` and ``L`` of the
    result are the critical cycle's cost and time."""
    return _solve(lib().ocm_ratio_min, row_ptr, col, w, want_policy, want_potential, profile,
                  times=t, **opt)


def max_cycle_ratio(row_ptr, col, w, t, *, want_policy=False, want_potential=False,
                    profile=False, **opt) -> Result:
    """Exact maximum cycle ratio (ocm_ratio_max)."""
    return _solve(lib().ocm_ratio_max, row_ptr, col, w, want_policy, want_potential, profile,
                  times=t, **opt)


_gws_cache: dict = {}


def cycle_mean_general(row_ptr, col, w, mode: str = "min", **opt) -> Result:
    """Optimum of a graph that need not be strongly connected (its vertices
    may even lack out-edges): the best optimum over its strongly connected
    components (ocm_min_general / ocm_max_general).  ``counters["components"]``
    is the number of components that hold a cycle."""
    if mode not in ("min", "max"):
        raise ValueError("mode must be 'min' or 'max'")
    g = make_graph(row_ptr, col, w)
    need = lib().ocm_general_workspace_size(C.byref(g))
    if need == 0:
        _check(OCM_E_INVALID_ARG)
    key = torch.device(col.device)
    ws = _gws_cache.get(key)
    if ws is None or ws.numel() < need:
        _gws_cache.pop(key, None)
        ws = torch.empty(need, dtype=torch.uint8, device=col.device)
        _gws_cache[key] = ws
    o = options(**opt)
    cyc = torch.empty(g.n, dtype=torch.int32, device=col.device)
    res = _Result()
    nc = C.c_int64()
    fn = lib().ocm_min_general if mode == "min" else lib().ocm_max_general
    _check(fn(C.byref(g), C.byref(o), C.c_void_p(ws.data_ptr()), ws.numel(),
              C.c_void_p(cyc.data_ptr()), g.n, C.byref(res), C.byref(nc), _stream()))
    return Result(res.p, res.q, cyc[:res.cycle_len], res.source, res.iterations, res.flags,
                  res.W, res.L, res.tight_edges, res.connect_rounds, res.jump_rounds,
                  res.fast_iters, {"components": nc.value})


def cycle_mean(row_ptr, col, w, mode: str = "min", **kw) -> Result:
    if mode not in ("min", "max"):
        raise ValueError("mode must be 'min' or 'max'")
    return (min_cycle_mean if mode == "min" else max_cycle_mean)(row_ptr, col, w, **kw)


@dataclasses.dataclass
class BatchResult:
    p: list
    q: list
    cycle_ptr: list
    cycle_edges: torch.Tensor     # int32 union CSR positions, graph by graph
    iterations: list
    flags: list
    status: list

    def value(self, g: int) -> Fraction:
        return Fraction(self.p[g], self.q[g])

    def cycle(self, g: int) -> torch.Tensor:
        return self.cycle_edges[self.cycle_ptr[g]:self.cycle_ptr[g + 1]]

    def tie(self, g: int):
        f = self.flags[g]
        if f & OCM_F_TIE:
            return True
        if f & OCM_F_TIE_UNCHECKED:
            return None
        return False


_bws_cache: dict = {}


def batched_last_schedule():
    """(lanes, tile, tuned_now) of the last batched call on this thread."""
    a, b, t = C.c_int32(), C.c_int32(), C.c_int32()
    lib().ocm_batched_last_schedule(C.byref(a), C.byref(b), C.byref(t))
    return a.value, b.value, bool(t.value)


def cycle_mean_batched(row_ptr, col, w, vptr, eptr, mode: str = "min", **opt) -> BatchResult:
    """Every graph of a disjoint-union CSR solved concurrently
    (ocm_min_batched / ocm_max_batched).  vptr, eptr: host int64 sequences."""
    import numpy as np
    if mode not in ("min", "max"):
        raise ValueError("mode must be 'min' or 'max'")
    g = make_graph(row_ptr, col, w)
    vp = np.ascontiguousarray(vptr, dtype=np.int64)
    ep = np.ascontiguousarray(eptr, dtype=np.int64)
    G = len(vp) - 1
    o = options(**opt)
    P = C.c_void_p
    need = lib().ocm_batched_workspace_size(G, vp.ctypes.data_as(P), ep.ctypes.data_as(P),
                                            C.byref(g), C.byref(o))
    if need == 0:
        _check(OCM_E_INVALID_ARG)
    key = torch.device(col.device)
    ws = _bws_cache.get(key)
    if ws is None or ws.numel() < need:
        _bws_cache.pop(key, None)
        ws = torch.empty(need, dtype=torch.uint8, device=col.device)
        _bws_cache[key] = ws
    p = np.zeros(G, np.int64)
    q = np.zeros(G, np.int64)
    cptr = np.zeros(G + 1, np.int64)
    iters = np.zeros(G, np.int32)
    flags = np.zeros(G, np.uint32)
    status = np.zeros(G, np.int32)
    cyc = torch.empty(g.n, dtype=torch.int32, device=col.device)
    fn = lib().ocm_min_batched if mode == "min" else lib().ocm_max_batched
    rc = fn(G, vp.ctypes.data_as(P), ep.ctypes.data_as(P), C.byref(g), C.byref(o),
            C.c_void_p(ws.data_ptr()), ws.numel(), p.ctypes.data_as(P), q.ctypes.data_as(P),
            cptr.ctypes.data_as(P), C.c_void_p(cyc.data_ptr()), g.n, iters.ctypes.data_as(P),
            flags.ctypes.data_as(P), status.ctypes.data_as(P), _stream())
    res = BatchResult(p.tolist(), q.tolist(), cptr.tolist(), cyc[:int(cptr[-1])],
                      iters.tolist(), flags.tolist(), status.tolist())
    if rc != OCM_OK and all(x == OCM_OK for x in res.status):
        _check(rc)
    return res


_small_ws: dict = {}


def weights_from_f64(w: torch.Tensor) -> torch.Tensor:
    """int64 copy of float64 weights; raises unless every weight is an integer
    with |w| < 2^53 (ocm_weights_from_f64)."""
    _dev(w, (torch.float64,), "w")
    out = torch.empty(w.numel(), dtype=torch.int64, device=w.device)
    key = torch.device(w.device)
    if key not in _small_ws:
        _small_ws[key] = torch.empty(256, dtype=torch.uint8, device=w.device)
    ws = _small_ws[key]
    _check(lib().ocm_weights_from_f64(w.numel(), C.c_void_p(w.data_ptr()),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                      ws.numel(), _stream()))
    return out


def adjoint_scatter(m: int, cycle_edges: torch.Tensor, grad_out: torch.Tensor) -> torch.Tensor:
    """float64[m] gradient: grad_out / |C| on the cycle's edges, 0 elsewhere
    (ocm_adjoint_scatter); grad_out is a one-element float64 GPU tensor."""
    _dev(cycle_edges, (torch.int32,), "cycle_edges")
    g = grad_out.reshape(1).to(torch.float64).contiguous()
    _dev(g, (torch.float64,), "grad_out")
    grad = torch.empty(m, dtype=torch.float64, device=cycle_edges.device)
    _check(lib().ocm_adjoint_scatter(m, C.c_void_p(cycle_edges.data_ptr()), cycle_edges.numel(),
                                     C.c_void_p(g.data_ptr()), C.c_void_p(grad.data_ptr()),
                                     _stream()))
    return grad


# -------------------------------------------------------------------------
# single phases (ocm_phase_*), driven from a given state
# -------------------------------------------------------------------------
def phase_sweep(row_ptr, col, w, pi, V=None, W=0, L=1, first=False, neg=False, schedule=0):
    g = make_graph(row_ptr, col, w)
    _dev(pi, (torch.int32,), "pi")
    if V is not None:
        _dev(V, (torch.int64,), "V")
    ws = workspace(g, col.device)
    ch = C.c_int64()
    _check(lib().ocm_phase_sweep(C.byref(g), int(neg), int(first),
                                 None if V is None else C.c_void_p(V.data_ptr()), W, L,
                                 C.c_void_p(pi.data_ptr()), schedule, C.c_void_p(ws.data_ptr()),
                                 ws.numel(), C.byref(ch), _stream()))
    return ch.value


def phase_cycles(row_ptr, col, w, pi):
    g = make_graph(row_ptr, col, w)
    _dev(pi, (torch.int32,), "pi")
    rep = torch.empty(g.n, dtype=torch.int32, device=col.device)
    onc = torch.empty(g.n, dtype=torch.uint8, device=col.device)
    ws = workspace(g, col.device)
    nc = C.c_int64()
    _check(lib().ocm_phase_cycles(C.byref(g), C.c_void_p(pi.data_ptr()),
                                  C.c_void_p(rep.data_ptr()), C.c_void_p(onc.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(nc), _stream()))
    return rep, onc, nc.value


def phase_select(row_ptr, col, w, pi, rep, onc, neg=False):
    g = make_graph(row_ptr, col, w)
    ws = workspace(g, col.device)
    s, W, L = C.c_int32(), C.c_int64(), C.c_int64()
    _check(lib().ocm_phase_select(C.byref(g), int(neg), C.c_void_p(pi.data_ptr()),
                                  C.c_void_p(rep.data_ptr()), C.c_void_p(onc.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(s), C.byref(W),
                                  C.byref(L), _stream()))
    return s.value, W.value, L.value


def phase_connect(row_ptr, col, w, rep, s, pi):
    """Rewires ``pi`` in place; returns (layer, rounds)."""
    g = make_graph(row_ptr, col, w)
    _dev(pi, (torch.int32,), "pi")
    layer = torch.empty(g.n, dtype=torch.int32, device=col.device)
    ws = workspace(g, col.device)
    r = C.c_int32()
    _check(lib().ocm_phase_connect(C.byref(g), C.c_void_p(rep.data_ptr()), s,
                                   C.c_void_p(pi.data_ptr()), C.c_void_p(layer.data_ptr()),
                                   C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(r), _stream()))
    return layer, r.value


def phase_values(row_ptr, col, w, pi, s, W, L, neg=False):
    g = make_graph(row_ptr, col, w)
    V = torch.empty(g.n, dtype=torch.int64, device=col.device)
    ws = workspace(g, col.device)
    r = C.c_int32()
    _check(lib().ocm_phase_values(C.byref(g), int(neg), C.c_void_p(pi.data_ptr()), s, W, L,
                                  C.c_void_p(V.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                  C.byref(r), _stream()))
    return V, r.value
