"""The general-graph oracle (strongly connected components, Prop. 2.2)
against brute-force cycle enumeration over the whole graph, brute-force
reachability, Karp per component and the Fig. 1 graph of Section 2.1."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, general, native
from paper_1111_0627_amd import synth


def reach_sets(rp, cl):
    n = len(rp) - 1
    out = []
    for s in range(n):
        seen = {s}
        st = [s]
        while st:
            v = st.pop()
            for e in range(rp[v], rp[v + 1]):
                u = int(cl[e])
                if u not in seen:
                    seen.add(u)
                    st.append(u)
        out.append(seen)
    return out


def random_general(rng, n, dmax, wlo, whi):
    rp = [0]
    col = []
    for v in range(n):
        d = int(rng.integers(0, dmax + 1))
        col.extend(int(t) for t in rng.integers(0, n, d))
        rp.append(len(col))
    return (np.array(rp, np.int32), np.array(col, np.int32),
            rng.integers(wlo, whi + 1, len(col)).astype(np.int64))


def test_components_against_reachability():
    rng = np.random.default_rng(1)
    for _ in range(400):
        n = int(rng.integers(1, 12))
        rp, cl, _ = random_general(rng, n, 3, 0, 1)
        comp = general.components(rp, cl)
        R = reach_sets(rp, cl)
        for v in range(n):
            members = [u for u in range(n) if u in R[v] and v in R[u]]
            assert comp[v] == min(members)


def test_general_against_brute_force():
    rng = np.random.default_rng(2)
    done = 0
    for it in range(3000):
        n = int(rng.integers(1, 9))
        rp, cl, w = random_general(rng, n, 3, -5, 5)
        mode = "max" if it % 3 == 0 else "min"
        if not brute.simple_cycles(rp, cl):
            with pytest.raises(native.OracleError):
                general.solve(rp, cl, w, mode)
            continue
        best, crit = brute.optimum(rp, cl, w, mode)
        s = general.solve(rp, cl, w, mode)
        assert s.value == best, it
        cyc = tuple(int(e) for e in s.cycle)
        assert cyc in [tuple(c) for c in crit], it
        assert s.tie == (1 if len(crit) > 1 else 0), it
        # the source is the smallest vertex of the cycle, its edge comes first
        srcs = [int(np.searchsorted(rp, e, side="right") - 1) for e in cyc]
        assert s.source == min(srcs) == srcs[0]
        done += 1
    assert done > 2000


def test_fig1_graph_min_over_components():
    """Fig. 1 (Section 2.1): components {a}, {b, e, f}, {c, d}, {g}; the
    optimum is the best one among those holding a cycle (a's self-loop, the
    cycle b-c... is not one: b->c leaves the component)."""
    a, b, c, d, e, f, g = range(7)
    adj = {a: [b, f, a], b: [c, e], c: [d], d: [c], e: [f], f: [b], g: [e]}
    rp = np.cumsum([0] + [len(adj[v]) for v in range(7)]).astype(np.int32)
    cl = np.array([t for v in range(7) for t in adj[v]], np.int32)
    comp = general.components(rp, cl)
    assert comp.tolist() == [a, b, c, c, b, b, g]
    rng = np.random.default_rng(4)
    for _ in range(200):
        w = rng.integers(-9, 10, len(cl))
        s = general.solve(rp, cl, w)
        loop = Fraction(int(w[2]), 1)                     # a -> a
        cd = Fraction(int(w[5] + w[6]), 2)                # c -> d -> c
        bef = Fraction(int(w[4] + w[7] + w[8]), 3)        # b -> e -> f -> b
        assert s.value == min(loop, cd, bef)


def test_midsize_components_against_karp():
    rng = np.random.default_rng(3)
    for k in range(6):
        parts = [synth.random_digraph(int(rng.integers(5, 300)), 1, 4, -50, 50, np.int64,
                                      seed=[3, k, j]) for j in range(int(rng.integers(2, 6)))]
        u, vptr, eptr = synth.disjoint_union(parts)
        # forward edges between components (a DAG of components) plus sinks
        rp, cl, w = u.row_ptr.astype(np.int64), u.col.astype(np.int64), u.w.astype(np.int64)
        extra_src = rng.integers(0, u.n, 40)
        rows = [list(cl[rp[v]:rp[v + 1]]) for v in range(u.n)]
        wts = [list(w[rp[v]:rp[v + 1]]) for v in range(u.n)]
        for v in extra_src:
            gi = int(np.searchsorted(vptr, v, side="right") - 1)
            if gi + 1 < len(parts):
                rows[v].append(int(rng.integers(vptr[gi + 1], u.n)))
                wts[v].append(int(rng.integers(-50, 50)))
        nrp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
        ncl = np.array([x for r in rows for x in r], np.int32)
        nw = np.array([x for r in wts for x in r], np.int64)
        s = general.solve(nrp, ncl, nw)
        want = min(native.karp(p.row_ptr, p.col, p.w) for p in parts)
        assert s.value == want
        assert s.ncomp == len(parts)
