"""ctypes wrapper of ``liboracle.so`` (Karp, sequential policy iteration,
exact tie test, optimality certificate).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK = 0
ORC_E_INVALID_ARG = -1
ORC_E_BAD_CSR = -2
ORC_E_NO_OUT_EDGE = -3
ORC_E_NOT_STRONGLY_CONNECTED = -4
ORC_E_OVERFLOW = -5
ORC_E_CAPACITY = -6
ORC_E_NOT_CONVERGED = -7
ORC_E_CERT_CYCLE = -20
ORC_E_CERT_MEAN = -21
ORC_E_CERT_POTENTIAL = -22


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"oracle status {code} {what}")
        self.code = code


class _Result(C.Structure):
    _fields_ = [("p", C.c_int64), ("q", C.c_int64), ("cycle_len", C.c_int64),
                ("source", C.c_int32), ("iterations", C.c_int32),
                ("tie", C.c_int32), ("ncycles_first", C.c_int32),
                ("W", C.c_int64), ("L", C.c_int64), ("tight", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        L.orc_karp.argtypes = [i64, i64, P, P, P, P, P]
        L.orc_karp.restype = C.c_int
        L.orc_solve.argtypes = [i64, i64, P, P, P, C.c_int, i32, C.c_int,
                                C.POINTER(_Result), P, i64, P, P]
        L.orc_solve.restype = C.c_int
        L.orc_solve_ratio.argtypes = [i64, i64, P, P, P, P, C.c_int, i32, C.c_int,
                                      C.POINTER(_Result), P, i64, P, P]
        L.orc_solve_ratio.restype = C.c_int
        L.orc_solve_mc.argtypes = [i64, i64, P, P, P, C.c_int, i32, C.c_int,
                                   C.POINTER(_Result), P, i64, P, P]
        L.orc_solve_mc.restype = C.c_int
        L.orc_certify_ratio.argtypes = [i64, i64, P, P, P, P, C.c_int, i64, i64, P, i64, P,
                                        i64]
        L.orc_certify_ratio.restype = C.c_int
        L.orc_state_new_ratio.argtypes = [i64, i64, P, P, P, P, C.c_int, C.POINTER(C.c_int)]
        L.orc_state_new_ratio.restype = P
        L.orc_certify.argtypes = [i64, i64, P, P, P, C.c_int, i64, i64, P, i64, P, i64]
        L.orc_certify.restype = C.c_int
        L.orc_state_new.argtypes = [i64, i64, P, P, P, C.c_int, C.POINTER(C.c_int)]
        L.orc_state_new.restype = P
        L.orc_state_free.argtypes = [P]
        L.orc_state_sweep.argtypes = [P]
        L.orc_state_sweep.restype = i64
        L.orc_state_cycles.argtypes = [P]
        L.orc_state_cycles.restype = i64
        L.orc_state_select.argtypes = [P, P, P, P]
        L.orc_state_select.restype = C.c_int
        L.orc_state_connect.argtypes = [P]
        L.orc_state_connect.restype = C.c_int
        L.orc_state_values.argtypes = [P]
        L.orc_state_tie.argtypes = [P]
        L.orc_state_tie.restype = C.c_int
        for nm in ("pi", "rep", "on_cycle", "layer"):
            getattr(L, f"orc_state_get_{nm}").argtypes = [P, P]
        L.orc_state_get_val.argtypes = [P, P]
        L.orc_state_get_val.restype = C.c_int
        L.orc_state_rounds.argtypes = [P]
        L.orc_state_rounds.restype = i32
        L.orc_state_iter.argtypes = [P]
        L.orc_state_iter.restype = i32
        L.orc_state_set.argtypes = [P, P, P, i64, i64, i32, i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(row_ptr, col, w):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int64)
    return rp, cl, ww


def karp(row_ptr, col, w) -> Fraction:
    """Minimum cycle mean by Karp's theorem (value only)."""
    rp, cl, ww = _csr(row_ptr, col, w)
    p, q = C.c_int64(), C.c_int64()
    rc = lib().orc_karp(len(rp) - 1, len(cl), _ptr(rp), _ptr(cl), _ptr(ww),
                        C.byref(p), C.byref(q))
    if rc:
        raise OracleError(rc, "karp")
    return Fraction(p.value, q.value)


@dataclasses.dataclass
class Solution:
    p: int
    q: int
    cycle: np.ndarray        # CSR edge positions, starting at pi(source)
    source: int
    iterations: int
    tie: int                 # 1 another critical cycle exists, 0 unique, -1 not checked
    ncycles_first: int
    W: int
    L: int
    tight: int               # tight non-policy edges at the optimum
    V: np.ndarray | None     # potential scaled by L (int64), if requested
    pi: np.ndarray | None = None   # final policy (CSR positions), if requested

    @property
    def value(self) -> Fraction:
        return Fraction(self.p, self.q)


def solve(row_ptr, col, w, mode: str = "min", max_iters: int = 0,
          tie: bool = True, want_V: bool = False, want_pi: bool = False,
          t=None) -> Solution:
    """Sequential policy iteration (Alg. 2 with readings R1-R10).  With edge
    times ``t`` (integers >= 1) it solves the optimal cycle ratio cost/time;
    then ``L`` is the critical cycle's time and ``len(cycle)`` its length."""
    rp, cl, ww = _csr(row_ptr, col, w)
    n, m = len(rp) - 1, len(cl)
    res = _Result()
    cyc = np.zeros(max(n, 1), np.int32)
    V = np.zeros(n, np.int64) if want_V else None
    pi = np.zeros(n, np.int32) if want_pi else None
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.int64)
    rc = lib().orc_solve_ratio(n, m, _ptr(rp), _ptr(cl), _ptr(ww),
                               None if tt is None else _ptr(tt), int(mode == "max"),
                               max_iters, int(tie), C.byref(res), _ptr(cyc), n,
                               _ptr(V) if want_V else None, _ptr(pi) if want_pi else None)
    if rc:
        raise OracleError(rc, "solve")
    return Solution(res.p, res.q, cyc[:res.cycle_len].copy(), res.source,
                    res.iterations, res.tie, res.ncycles_first, res.W, res.L, res.tight, V, pi)


def solve_multichain(row_ptr, col, w, mode: str = "min", max_iters: int = 0,
                     tie: bool = True, want_V: bool = False,
                     want_pi: bool = False) -> Solution:
    """Multichain policy iteration (every policy cycle keeps its own gain; no
    rebuild): same optimum, its own trajectory and critical cycle.  ``V``:
    each vertex's value scaled by the length of the cycle it reaches."""
    rp, cl, ww = _csr(row_ptr, col, w)
    n, m = len(rp) - 1, len(cl)
    res = _Result()
    cyc = np.zeros(max(n, 1), np.int32)
    V = np.zeros(n, np.int64) if want_V else None
    pi = np.zeros(n, np.int32) if want_pi else None
    rc = lib().orc_solve_mc(n, m, _ptr(rp), _ptr(cl), _ptr(ww), int(mode == "max"), max_iters,
                            int(tie), C.byref(res), _ptr(cyc), n,
                            _ptr(V) if want_V else None, _ptr(pi) if want_pi else None)
    if rc:
        raise OracleError(rc, "solve_multichain")
    return Solution(res.p, res.q, cyc[:res.cycle_len].copy(), res.source, res.iterations,
                    res.tie, res.ncycles_first, res.W, res.L, res.tight, V, pi)


def certify(row_ptr, col, w, p, q, cycle, V, K, mode: str = "min", t=None) -> int:
    """Optimality certificate; returns ORC_OK (0) or a negative code.  With
    edge times ``t`` it certifies the optimal cost-to-time ratio p/q."""
    rp, cl, ww = _csr(row_ptr, col, w)
    cy = np.ascontiguousarray(cycle, dtype=np.int32)
    VV = np.ascontiguousarray(V, dtype=np.int64)
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.int64)
    return lib().orc_certify_ratio(len(rp) - 1, len(cl), _ptr(rp), _ptr(cl), _ptr(ww),
                                   None if tt is None else _ptr(tt), int(mode == "max"),
                                   int(p), int(q), _ptr(cy), len(cy), _ptr(VV), int(K))


class Stepper:
    """Phase-by-phase sequential policy iteration, for trace comparisons.

    The phases are the steps of Alg. 2 in order: ``sweep`` (policy
    improvement), ``cycles`` (policy-graph cycles), ``select`` (minimum-mean
    cycle and its source), ``connect`` (break every other cycle) and
    ``values`` (value update from the source).
    """

    def __init__(self, row_ptr, col, w, mode: str = "min", t=None):
        self.rp, self.cl, self.ww = _csr(row_ptr, col, w)
        self.tt = None if t is None else np.ascontiguousarray(t, dtype=np.int64)
        self.n, self.m = len(self.rp) - 1, len(self.cl)
        rc = C.c_int()
        self.h = lib().orc_state_new_ratio(self.n, self.m, _ptr(self.rp), _ptr(self.cl),
                                           _ptr(self.ww),
                                           None if self.tt is None else _ptr(self.tt),
                                           int(mode == "max"), C.byref(rc))
        if not self.h:
            raise OracleError(rc.value, "state")

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_state_free(self.h)
            self.h = None

    def sweep(self) -> int:
        return int(lib().orc_state_sweep(self.h))

    def cycles(self) -> int:
        return int(lib().orc_state_cycles(self.h))

    def select(self):
        s, W, L = C.c_int32(), C.c_int64(), C.c_int64()
        rc = lib().orc_state_select(self.h, C.byref(s), C.byref(W), C.byref(L))
        if rc:
            raise OracleError(rc, "select")
        return s.value, W.value, L.value

    def connect(self) -> int:
        return int(lib().orc_state_connect(self.h))

    def values(self):
        lib().orc_state_values(self.h)

    def tie(self) -> int:
        return int(lib().orc_state_tie(self.h))

    def get(self, name: str) -> np.ndarray:
        if name == "val":
            out = np.zeros(self.n, np.int64)
            rc = lib().orc_state_get_val(self.h, _ptr(out))
            if rc:
                raise OracleError(rc, "val")
            return out
        dt = np.uint8 if name == "on_cycle" else np.int32
        out = np.zeros(self.n, dt)
        getattr(lib(), f"orc_state_get_{name}")(self.h, _ptr(out))
        return out

    @property
    def rounds(self) -> int:
        return int(lib().orc_state_rounds(self.h))

    @property
    def iter(self) -> int:
        return int(lib().orc_state_iter(self.h))

    def set(self, pi=None, val=None, W=0, L=1, s=-1, it=0):
        pp = None if pi is None else np.ascontiguousarray(pi, np.int32)
        vv = None if val is None else np.ascontiguousarray(val, np.int64)
        lib().orc_state_set(self.h, None if pp is None else _ptr(pp),
                            None if vv is None else _ptr(vv), W, L, s, it)
