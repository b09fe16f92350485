"""Optimal cycle mean of graphs that are not strongly connected.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Prop. 2.2: every cycle lies inside one strongly connected component, so the
optimum of a graph is the best optimum among its components that hold a
cycle (two or more vertices, or one vertex with a self-loop).  Section 2.5
names the SCC decomposition as the alternative to making the graph strongly
connected.  Here: Tarjan's components (``orc_scc``), then each component
solved alone by the sequential policy iteration of ``native``, with

* the component's vertices numbered in increasing original index and its
  edges (those with both ends inside it) in original CSR order;
* the result taken from the best component, ties broken by the smallest
  component id (its smallest vertex index), the cycle mapped back to the
  original edge positions;
* the tie flag set when the chosen component has a second critical cycle or
  another component reaches the same optimum.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
from fractions import Fraction

import numpy as np

from . import native


def components(row_ptr, col) -> np.ndarray:
    """comp[v] = smallest vertex index of v's strongly connected component."""
    L = native.lib()
    if not getattr(L, "_scc_typed", False):
        L.orc_scc.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_scc.restype = C.c_int
        L._scc_typed = True
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    n = len(rp) - 1
    comp = np.empty(n, np.int32)
    rc = L.orc_scc(n, len(cl), rp.ctypes.data_as(C.c_void_p), cl.ctypes.data_as(C.c_void_p),
                   comp.ctypes.data_as(C.c_void_p))
    if rc:
        raise native.OracleError(rc, "scc")
    return comp


@dataclasses.dataclass
class Part:
    comp: int                 # component id (smallest vertex)
    verts: np.ndarray         # original vertex of each local vertex (ascending)
    row_ptr: np.ndarray
    col: np.ndarray
    emap: np.ndarray          # original edge position of each local edge


def parts(row_ptr, col, comp) -> list:
    """The components that hold a cycle, each as its own CSR graph."""
    rp = np.asarray(row_ptr, np.int64)
    cl = np.asarray(col, np.int64)
    n = len(rp) - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    inside = comp[src] == comp[cl]
    out = []
    order = np.argsort(comp, kind="stable")
    ids, starts = np.unique(comp[order], return_index=True)
    bounds = list(starts) + [n]
    local = np.empty(n, np.int64)
    for k, cid in enumerate(ids):
        verts = order[bounds[k]:bounds[k + 1]]
        local[verts] = np.arange(len(verts))
        edges = np.concatenate([np.arange(rp[v], rp[v + 1])[inside[rp[v]:rp[v + 1]]]
                                for v in verts])
        if len(edges) == 0:
            continue            # a single vertex without a self-loop: no cycle
        deg = np.array([int(inside[rp[v]:rp[v + 1]].sum()) for v in verts])
        sub_rp = np.zeros(len(verts) + 1, np.int64)
        np.cumsum(deg, out=sub_rp[1:])
        out.append(Part(int(cid), verts.astype(np.int64), sub_rp.astype(np.int32),
                        local[cl[edges]].astype(np.int32), edges.astype(np.int64)))
    return out


@dataclasses.dataclass
class GeneralSolution:
    p: int
    q: int
    cycle: np.ndarray         # original edge positions, from the source's edge
    source: int               # original vertex
    iterations: int           # of the chosen component's solve
    tie: int
    comp: int                 # chosen component id
    ncomp: int                # components that hold a cycle

    @property
    def value(self) -> Fraction:
        return Fraction(self.p, self.q)


def solve(row_ptr, col, w, mode: str = "min") -> GeneralSolution:
    comp = components(row_ptr, col)
    ps = parts(row_ptr, col, comp)
    if not ps:
        raise native.OracleError(native.ORC_E_INVALID_ARG, "the graph has no cycle")
    w = np.asarray(w, np.int64)
    best = None
    sols = []
    for part in ps:
        s = native.solve(part.row_ptr, part.col, w[part.emap], mode=mode)
        sols.append((part, s))
        if best is None or (s.value < best[1].value if mode == "min" else s.value > best[1].value):
            best = (part, s)
    part, s = best
    same = sum(1 for _, x in sols if x.value == s.value)
    return GeneralSolution(s.p, s.q, part.emap[s.cycle].astype(np.int64),
                           int(part.verts[s.source]), s.iterations,
                           1 if (s.tie == 1 or same > 1) else 0, part.comp, len(ps))
