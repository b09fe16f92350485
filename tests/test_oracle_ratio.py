"""The optimal cycle ratio oracle (cost over time per cycle, Section 2.2;
the (v, w, t) edge record of Fig. 2) against what pins it without the oracle
itself: hand-derived runs, brute-force simple-cycle enumeration, an exact
parametric negative-cycle test, closed forms and invariants."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, native
from paper_1111_0627_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _traces():
    with open(os.path.join(GOLD, "ratio_traces.json")) as f:
        return json.load(f)["traces"]


@pytest.mark.parametrize("tr", _traces(), ids=lambda t: t["name"])
def test_ratio_hand_traces(tr):
    rp, cl, w, t = (np.array(tr[k]) for k in ("row_ptr", "col", "w", "t"))
    r = tr["result"]
    s = native.solve(rp, cl, w, t=t)
    assert (s.p, s.q, s.L, s.cycle.tolist(), s.source, s.iterations, s.tie, s.tight) == \
        (r["p"], r["q"], r["T"], r["cycle"], r["source"], r["iterations"], r["tie"], r["tight"])
    if "mean_result" in tr:
        mr = tr["mean_result"]
        sm = native.solve(rp, cl, w)
        assert (sm.p, sm.q, sm.cycle.tolist(), sm.source) == \
            (mr["p"], mr["q"], mr["cycle"], mr["source"])


def _tiny(rng, n):
    rp, cl, w = brute.random_tiny(rng, n, 3, -6, 6)
    t = rng.integers(1, 6, len(cl))
    return rp, cl, w, t


def test_ratio_against_brute_force_and_certificate():
    rng = np.random.default_rng(11)
    for it in range(3000):
        n = int(rng.integers(1, 8))
        rp, cl, w, t = _tiny(rng, n)
        mode = "max" if it % 3 == 0 else "min"
        best, crit = brute.optimum(rp, cl, w, mode, t=t)
        s = native.solve(rp, cl, w, mode=mode, t=t, want_V=True)
        assert s.value == best, it
        assert tuple(int(e) for e in s.cycle) in [tuple(c) for c in crit] or \
            tuple(sorted(int(e) for e in s.cycle)) in [tuple(sorted(c)) for c in crit], it
        assert s.tie == (1 if len(crit) > 1 else 0), it
        assert sum(int(t[e]) for e in s.cycle) == s.L
        assert native.certify(rp, cl, w, s.p, s.q, s.cycle, s.V, s.L, mode, t=t) == 0


def test_ratio_parametric_check_midsize():
    rng = np.random.default_rng(5)
    for k in range(12):
        n = int(rng.integers(20, 120))
        g = synth.random_digraph(n, 1, 4, -50, 50, np.int64, seed=[7, k])
        t = rng.integers(1, 20, g.m)
        s = native.solve(g.row_ptr, g.col, g.w, t=t)
        assert brute.ratio_by_parametric_check(g.row_ptr, g.col, g.w, t, s.value)
        # dropping the times (the mean) is a different, wrong answer here
        sm = native.solve(g.row_ptr, g.col, g.w)
        if sm.value != s.value:
            assert not brute.ratio_by_parametric_check(g.row_ptr, g.col, g.w, t, sm.value)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_constant_time_is_the_mean_over_k(k):
    for seed in range(5):
        g = synth.random_digraph(400, 1, 5, -40, 40, np.int32, seed=seed)
        t = np.full(g.m, k, np.int64)
        s = native.solve(g.row_ptr, g.col, g.w, t=t)
        m = native.solve(g.row_ptr, g.col, g.w)
        assert s.value == m.value / k
        assert (s.cycle.tolist(), s.source, s.iterations, s.tie, s.tight) == \
            (m.cycle.tolist(), m.source, m.iterations, m.tie, m.tight)


def test_shift_by_multiple_of_time_and_scaling():
    rng = np.random.default_rng(9)
    for seed in range(5):
        g = synth.random_digraph(300, 1, 4, -30, 30, np.int64, seed=seed)
        t = rng.integers(1, 9, g.m)
        s = native.solve(g.row_ptr, g.col, g.w, t=t)
        # cost + c * time shifts every cycle's ratio by c (the first sweep,
        # which minimises plain cost, may then start elsewhere)
        for c in (-5, 17):
            sh = native.solve(g.row_ptr, g.col, g.w + c * t, t=t)
            assert sh.value == s.value + c
        sc = native.solve(g.row_ptr, g.col, 3 * g.w, t=2 * t)
        assert sc.value == s.value * Fraction(3, 2)
        assert (sc.cycle.tolist(), sc.iterations) == (s.cycle.tolist(), s.iterations)


def test_ring_closed_form_and_max_is_minus_min():
    rng = np.random.default_rng(2)
    n = 37
    rp = np.arange(n + 1, dtype=np.int32)
    cl = ((np.arange(n) + 1) % n).astype(np.int32)
    w = rng.integers(-100, 100, n)
    t = rng.integers(1, 10, n)
    s = native.solve(rp, cl, w, t=t)
    assert s.value == Fraction(int(w.sum()), int(t.sum()))
    g = synth.random_digraph(500, 1, 5, -20, 20, np.int64, seed=4)
    t = rng.integers(1, 7, g.m)
    mx = native.solve(g.row_ptr, g.col, g.w, mode="max", t=t)
    mn = native.solve(g.row_ptr, g.col, -g.w, t=t)
    assert mx.value == -mn.value
    assert (mx.cycle.tolist(), mx.iterations) == (mn.cycle.tolist(), mn.iterations)


def test_ratio_rejects_nonpositive_times_and_planted_mistakes():
    g = synth.random_digraph(50, 1, 3, 1, 9, np.int64, seed=1)
    t = np.ones(g.m, np.int64)
    t[7] = 0
    with pytest.raises(native.OracleError):
        native.solve(g.row_ptr, g.col, g.w, t=t)
    t = np.random.default_rng(3).integers(1, 5, g.m)
    s = native.solve(g.row_ptr, g.col, g.w, t=t, want_V=True)
    assert native.certify(g.row_ptr, g.col, g.w, s.p, s.q, s.cycle, s.V, s.L, t=t) == 0
    # a wrong value, or the same potential judged without the times, fails
    assert native.certify(g.row_ptr, g.col, g.w, s.p + 1, s.q, s.cycle, s.V, s.L, t=t) != 0
    if len(set(int(t[e]) for e in s.cycle)) > 1 or int(t[s.cycle[0]]) != 1:
        assert native.certify(g.row_ptr, g.col, g.w, s.p, s.q, s.cycle, s.V, s.L) != 0
