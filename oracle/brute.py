"""Brute-force optimal cycle mean (and cycle ratio) by simple-cycle
enumeration, in exact rationals, for tiny graphs.

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


def optimum(row_ptr, col, w, mode: str = "min", t=None):
    """(optimal mean as Fraction, sorted list of optimal simple cycles).

    With edge times ``t`` (all >= 1) the value of a cycle is its cost over its
    time (the optimal cycle ratio of Section 2.2).  A cycle's ratio is the
    time-weighted average of the ratios of the simple cycles it splits into,
    so simple cycles again suffice."""
    cycles = simple_cycles(row_ptr, col)
    if not cycles:
        raise ValueError("graph has no cycle")
    ww = [int(x) for x in w]
    tt = [1] * len(ww) if t is None else [int(x) for x in t]
    if min(tt, default=1) < 1:
        raise ValueError("times must be >= 1")
    best = None
    crit = []
    for c in cycles:
        mu = Fraction(sum(ww[e] for e in c), sum(tt[e] for e in c))
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


def has_negative_cycle(row_ptr, col, cost) -> bool:
    """Bellman-Ford from a virtual source joined to every vertex: does some
    cycle have negative total cost?  (Exact, any integer or Fraction costs.)"""
    n = len(row_ptr) - 1
    rp = [int(x) for x in row_ptr]
    cl = [int(x) for x in col]
    d = [0] * n
    for _ in range(n):
        changed = False
        for v in range(n):
            for e in range(rp[v], rp[v + 1]):
                u = cl[e]
                x = d[v] + cost[e]
                if x < d[u]:
                    d[u] = x
                    changed = True
        if not changed:
            return False
    return True


def ratio_by_parametric_check(row_ptr, col, w, t, lam: Fraction) -> bool:
    """lam is the minimum cycle ratio iff no cycle is negative under the costs
    q*w - p*t (lam = p/q, so lam <= every ratio) while some cycle is negative
    under q*w - p*t - 1 scaled appropriately; the second test uses
    (q*w - p*t)*D - t with D larger than any cycle time, which is negative on
    a cycle exactly when that cycle's ratio equals lam."""
    p, q = lam.numerator, lam.denominator
    base = [q * int(a) - p * int(b) for a, b in zip(w, t)]
    if has_negative_cycle(row_ptr, col, base):
        return False
    D = sum(int(b) for b in t) + 1
    tight = [x * D - int(b) for x, b in zip(base, t)]
    return has_negative_cycle(row_ptr, col, tight)
