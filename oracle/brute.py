"""Brute-force optimal cycle mean by simple-cycle enumeration, in exact
rationals, for tiny graphs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The definition of Section 2.1: the cycle mean of a cycle is its weight divided
by its length, and the optimal cycle mean is the minimum over all cycles.  Any
cycle splits into simple cycles and its mean is their length-weighted average,
so the minimum over simple cycles is the same number.  Cycles are sequences of
edges, so parallel edges give distinct cycles and a self-loop is a cycle of
length one.

Each simple cycle is enumerated once, starting from its smallest vertex and
continuing only through larger vertices, and is recorded as the tuple of its
CSR edge positions starting with the edge that leaves the smallest vertex.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def simple_cycles(row_ptr, col):
    """All simple cycles, each a tuple of edge positions from its min vertex."""
    n = len(row_ptr) - 1
    rp = [int(x) for x in row_ptr]
    cl = [int(x) for x in col]
    out = []
    for s in range(n):
        # depth-first over vertices > s; path holds edge positions
        on_path = [False] * n
        on_path[s] = True
        stack = [(s, rp[s])]
        path = []
        while stack:
            v, e = stack[-1]
            if e >= rp[v + 1]:
                stack.pop()
                if path:
                    on_path[v] = False
                    path.pop()
                continue
            stack[-1] = (v, e + 1)
            u = cl[e]
            if u == s:
                out.append(tuple(path + [e]))
            elif u > s and not on_path[u]:
                on_path[u] = True
                path.append(e)
                stack.append((u, rp[u]))
    return out


def optimum(row_ptr, col, w, mode: str = "min"):
    """(optimal mean as Fraction, sorted list of optimal simple cycles)."""
    cycles = simple_cycles(row_ptr, col)
    if not cycles:
        raise ValueError("graph has no cycle")
    ww = [int(x) for x in w]
    best = None
    crit = []
    for c in cycles:
        mu = Fraction(sum(ww[e] for e in c), len(c))
        better = best is None or (mu < best if mode == "min" else mu > best)
        if better:
            best, crit = mu, [c]
        elif mu == best:
            crit.append(c)
    return best, sorted(crit)


def random_tiny(rng: np.random.Generator, n: int, dmax: int, wlo: int, whi: int,
                ring: bool = True):
    """A tiny random digraph, optionally with a Hamiltonian ring, that may hold
    self-loops, parallel edges and equal weights."""
    rp = [0]
    col = []
    for v in range(n):
        d = int(rng.integers(0, dmax + 1)) if ring else int(rng.integers(1, dmax + 1))
        tg = [int(t) for t in rng.integers(0, n, d)]
        if ring:
            tg.insert(int(rng.integers(0, d + 1)), (v + 1) % n)
        col.extend(tg)
        rp.append(len(col))
    w = rng.integers(wlo, whi + 1, len(col))
    return (np.array(rp, np.int32), np.array(col, np.int32), np.array(w, np.int64))
