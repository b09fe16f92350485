"""The multichain policy iteration oracle (every policy cycle keeps its own
gain; no rebuild) against what pins it: a hand-derived run, brute-force
simple-cycle enumeration (value, critical-cycle membership, tie flag), Karp
and the invariants."""

import json
import os

import numpy as np
import pytest

from oracle import brute, native
from paper_1111_0627_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_multichain_hand_trace():
    with open(os.path.join(GOLD, "multichain_traces.json")) as f:
        traces = json.load(f)["traces"]
    for tr in traces:
        rp, cl, w = (np.array(tr[k]) for k in ("row_ptr", "col", "w"))
        r = tr["multichain"]
        s = native.solve_multichain(rp, cl, w, want_V=True, want_pi=True)
        assert (s.p, s.q, s.cycle.tolist(), s.source, s.iterations, s.tie, s.tight) == \
            (r["p"], r["q"], r["cycle"], r["source"], r["iterations"], r["tie"], r["tight"])
        assert s.V.tolist() == r["V"] and s.pi.tolist() == r["pi"]
        u = tr["unichain"]
        su = native.solve(rp, cl, w)
        assert (su.p, su.q, su.cycle.tolist(), su.source, su.iterations) == \
            (u["p"], u["q"], u["cycle"], u["source"], u["iterations"])


def test_multichain_tight_edges_closed_form():
    """Equal weights: every cycle is critical, every value is 0 and every
    non-policy edge is tight (m - n of them)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        rp, cl, w = brute.random_tiny(rng, n, 4, 0, 0)
        w = np.full(len(cl), 7, np.int64)
        s = native.solve_multichain(rp, cl, w, want_V=True)
        assert s.value == 7 and s.tight == len(cl) - n
        assert not s.V.any()


def test_multichain_tight_edges_cover_critical_cycles():
    """Every edge of every critical cycle is tight at the optimum (reduced
    costs are non-negative and sum to zero around it), so the tight
    non-policy edges number at least the critical cycles' edges outside the
    policy."""
    rng = np.random.default_rng(31)
    for it in range(2000):
        n = int(rng.integers(1, 7))
        rp, cl, w = brute.random_tiny(rng, n, 3, -3, 3)
        best, crit = brute.optimum(rp, cl, w)
        s = native.solve_multichain(rp, cl, w, want_pi=True)
        pol = set(s.pi.tolist())
        on_crit = {e for c in crit for e in c} - pol
        assert s.tight >= len(on_crit), it


def test_multichain_against_brute_force():
    rng = np.random.default_rng(23)
    for it in range(4000):
        n = int(rng.integers(1, 8))
        rp, cl, w = brute.random_tiny(rng, n, 3, -6, 6)
        mode = "max" if it % 3 == 0 else "min"
        best, crit = brute.optimum(rp, cl, w, mode)
        s = native.solve_multichain(rp, cl, w, mode)
        assert s.value == best, it
        assert tuple(int(e) for e in s.cycle) in [tuple(c) for c in crit], it
        assert s.tie == (1 if len(crit) > 1 else 0), it


@pytest.mark.parametrize("seed", range(6))
def test_multichain_against_karp_and_unichain(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(100, 3000))
    g = synth.random_digraph(n, 1, 5, -100, 100, np.int64, seed=[11, seed])
    s = native.solve_multichain(g.row_ptr, g.col, g.w)
    assert s.value == native.karp(g.row_ptr, g.col, g.w)
    assert s.value == native.solve(g.row_ptr, g.col, g.w).value
    # shift and scale move the value, not the trajectory
    sh = native.solve_multichain(g.row_ptr, g.col, g.w + 7)
    sc = native.solve_multichain(g.row_ptr, g.col, 3 * g.w)
    assert sh.value == s.value + 7 and sc.value == 3 * s.value
    assert (sh.cycle.tolist(), sh.iterations) == (s.cycle.tolist(), s.iterations)
    assert (sc.cycle.tolist(), sc.iterations) == (s.cycle.tolist(), s.iterations)
    mx = native.solve_multichain(g.row_ptr, g.col, g.w, mode="max")
    mn = native.solve_multichain(g.row_ptr, g.col, -g.w)
    assert mx.value == -mn.value and mx.cycle.tolist() == mn.cycle.tolist()
