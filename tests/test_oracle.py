"""Pins of the CPU oracle against facts that do not come from the oracle itself:
hand-derived traces of Alg. 2, brute-force enumeration of simple cycles
(the definition of Section 2.1), Karp's theorem, closed forms, invariants of
the cycle mean, and the optimality certificate (Prop. 2.1, Eq. (1))."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, closed, native
from paper_1111_0627_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_traces():
    with open(os.path.join(GOLD, "hand_traces.json")) as f:
        return json.load(f)["traces"]


@pytest.mark.parametrize("tr", _load_traces(), ids=lambda t: t["name"])
def test_hand_traces_phase_by_phase(tr):
    rp, cl, w = (np.array(tr[k]) for k in ("row_ptr", "col", "w"))
    st = native.Stepper(rp, cl, w)
    for it in tr["iterations"]:
        assert st.sweep() == it["changed"]
        assert st.get("pi").tolist() == it["pi"]
        if "rep" not in it:
            break
        st.cycles()
        assert st.get("rep").tolist() == it["rep"]
        assert st.get("on_cycle").tolist() == it["on_cycle"]
        assert st.select() == (it["s"], it["W"], it["L"])
        assert st.connect() == 0
        assert st.rounds == it["rounds"]
        assert st.get("layer").tolist() == it["layer"]
        assert st.get("pi").tolist() == it["pi_connected"]
        st.values()
        assert st.get("val").tolist() == it["V"]
    r = tr["result"]
    sol = native.solve(rp, cl, w, want_V=True)
    assert (sol.p, sol.q, sol.cycle.tolist(), sol.source, sol.iterations, sol.tie, sol.tight) == \
        (r["p"], r["q"], r["cycle"], r["source"], r["iterations"], r["tie"], r["tight"])
    val, crit = brute.optimum(rp, cl, w)
    assert val == Fraction(r["p"], r["q"]) == native.karp(rp, cl, w)
    assert tuple(r["cycle"]) in crit
    assert (len(crit) > 1) == bool(r["tie"])


def test_brute_enumerates_known_cycles():
    # complete digraph on 3 vertices with self-loops: 3 loops, 3 two-cycles,
    # 2 three-cycles
    rp = np.array([0, 3, 6, 9])
    cl = np.array([0, 1, 2, 0, 1, 2, 0, 1, 2])
    assert len(brute.simple_cycles(rp, cl)) == 8
    # parallel edges double the 2-cycle count
    rp = np.array([0, 2, 3])
    cl = np.array([1, 1, 0])
    assert sorted(brute.simple_cycles(rp, cl)) == [(0, 2), (1, 2)]


def _check_tiny(rp, cl, w, mode):
    val, crit = brute.optimum(rp, cl, w, mode)
    sol = native.solve(rp, cl, w, mode=mode, want_V=True, want_pi=True)
    assert sol.value == val
    assert tuple(sol.cycle.tolist()) in crit
    assert sol.tie == int(len(crit) > 1)
    # Every edge of a critical cycle is tight at the optimum (its reduced
    # costs are >= 0 under a feasible potential and sum to zero around it),
    # so the tight non-policy count is at least the number of non-policy
    # edges lying on some critical simple cycle; a second critical cycle
    # needs at least one non-policy edge (the policy graph holds one cycle).
    on_crit = set(e for c in crit for e in c)
    assert sol.tight >= len(on_crit - set(sol.pi.tolist()))
    if len(crit) > 1:
        assert sol.tight >= 1
    assert sol.source == min(int(np.searchsorted(rp, e, side="right") - 1) for e in sol.cycle)
    assert native.certify(rp, cl, w, sol.p, sol.q, sol.cycle, sol.V, sol.L, mode) == 0
    kv = native.karp(rp, cl, w if mode == "min" else -w)
    assert (kv if mode == "min" else -kv) == val
    return sol


def test_random_tiny_graphs_against_brute_force_and_karp():
    rng = np.random.default_rng(12345)
    ties = 0
    for i in range(10_000):
        n = int(rng.integers(1, 8))
        rp, cl, w = brute.random_tiny(rng, n, 3, -3 if i % 3 == 0 else 1, 4 if i % 2 else 9)
        sol = _check_tiny(rp, cl, w, "min" if i % 4 else "max")
        ties += sol.tie
    assert 100 < ties < 9_900   # both branches of the tie test are exercised


def test_tiny_graphs_without_ring_are_certified_or_rejected():
    rng = np.random.default_rng(7)
    rejected = 0
    for _ in range(3000):
        n = int(rng.integers(2, 8))
        rp, cl, w = brute.random_tiny(rng, n, 3, 0, 6, ring=False)
        val, crit = brute.optimum(rp, cl, w)
        try:
            sol = native.solve(rp, cl, w, want_V=True)
        except native.OracleError as e:
            assert e.code == native.ORC_E_NOT_STRONGLY_CONNECTED
            rejected += 1
            continue
        assert sol.value == val and tuple(sol.cycle.tolist()) in crit
        assert native.certify(rp, cl, w, sol.p, sol.q, sol.cycle, sol.V, sol.L) == 0
    assert rejected > 100


@pytest.mark.parametrize("seed", range(6))
def test_tight_count_closed_form(seed):
    # A ring whose edges all weigh c plus chords weighing c or more.  The
    # weight-c edges then form a strongly connected subgraph (it holds the
    # ring), every weight-c edge lies on a cycle of mean c = the optimum, so
    # all of them are tight and the potential is constant; a heavier edge has
    # reduced cost L * (w - c) > 0.  Hence exactly (#weight-c edges) - n
    # non-policy edges are tight, whatever trajectory the iteration took.
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    c = int(rng.integers(-20, 20))
    rp, cl, ww = [0], [], []
    for v in range(n):
        d = int(rng.integers(0, 5))
        tg = [int(t) for t in rng.integers(0, n, d)]
        wt = [c + (int(rng.integers(1, 4)) if rng.random() < 0.6 else 0) for _ in tg]
        k = int(rng.integers(0, d + 1))
        tg.insert(k, (v + 1) % n)
        wt.insert(k, c)
        cl.extend(tg)
        ww.extend(wt)
        rp.append(len(cl))
    rp, cl, ww = np.array(rp), np.array(cl), np.array(ww)
    for mode, sign in (("min", 1), ("max", -1)):
        sol = native.solve(rp, cl, sign * ww, mode=mode, want_V=True, want_pi=True)
        assert sol.value == sign * c
        assert sol.tight == int((ww == c).sum()) - n
        assert (sol.V == 0).all()


def test_fig1_graph_not_strongly_connected():
    # Fig. 1 (Section 2.1): a..g, SCCs {a}, {b,e,f}, {c,d}, {g}; a has a self-loop
    a, b, c, d, e, f, g = range(7)
    adj = {a: [b, f, a], b: [c, e], c: [d], d: [c], e: [f], f: [b], g: [e]}
    rp = np.cumsum([0] + [len(adj[v]) for v in range(7)])
    cl = np.array([t for v in range(7) for t in adj[v]])
    rng = np.random.default_rng(3)
    for _ in range(200):
        w = rng.integers(-5, 6, len(cl))
        val, crit = brute.optimum(rp, cl, w)
        try:
            sol = native.solve(rp, cl, w, want_V=True)
        except native.OracleError as ex:
            assert ex.code == native.ORC_E_NOT_STRONGLY_CONNECTED
            continue
        assert sol.value == val
        assert native.certify(rp, cl, w, sol.p, sol.q, sol.cycle, sol.V, sol.L) == 0


def test_fig2b_offsets_zero_out_degree():
    # Fig. 2b: offsets 0, 3, 5, 5, 7: vertex 2 has no out-edge
    rp = np.array([0, 3, 5, 5, 7])
    cl = np.array([1, 2, 3, 0, 3, 1, 0])
    w = np.ones(7, np.int64)
    with pytest.raises(native.OracleError) as ex:
        native.solve(rp, cl, w)
    assert ex.value.code == native.ORC_E_NO_OUT_EDGE
    with pytest.raises(native.OracleError) as ex:
        native.solve(np.array([0, 3, 2, 7, 7]), cl, w)
    assert ex.value.code == native.ORC_E_BAD_CSR


def test_ring_closed_form():
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 17, 1000):
        w = rng.integers(-50, 50, n)
        rp = np.arange(n + 1)
        cl = (np.arange(n) + 1) % n
        sol = native.solve(rp, cl, w)
        assert sol.value == closed.ring_mean(w)
        assert sol.cycle.tolist() == list(range(n)) and sol.source == 0
        assert sol.iterations == 2 and sol.tie == 0


def test_self_loops_closed_form():
    # one vertex, several self-loops: the optimum is the smallest loop weight,
    # reached at its lowest position
    w = np.array([5, 3, 7, 3])
    sol = native.solve(np.array([0, 4]), np.zeros(4, np.int32), w)
    assert sol.value == 3 and sol.cycle.tolist() == [1] and sol.tie == 1
    sol = native.solve(np.array([0, 4]), np.zeros(4, np.int32), w, mode="max")
    assert sol.value == 7 and sol.cycle.tolist() == [2] and sol.tie == 0


@pytest.mark.parametrize("procs,states,seed", [(2, 4, 0), (3, 8, 1), (4, 16, 2), (3, 16, 0)])
def test_product_graph_closed_form(procs, states, seed):
    g = synth.product_graph(procs, states, 0.3, 1, 1000, seed)
    has2, t2, cost = synth.product_tables(procs, states, 0.3, 1, 1000, seed)
    locals_ = [synth.local_automaton(has2, t2, cost, i) for i in range(procs)]
    for mode in ("min", "max"):
        sol = native.solve(g.row_ptr, g.col, g.w, mode=mode, want_V=True)
        assert sol.value == closed.product_optimum(locals_, mode)
        assert native.certify(g.row_ptr, g.col, g.w, sol.p, sol.q, sol.cycle,
                              sol.V, sol.L, mode) == 0


@pytest.mark.slow
def test_full_product_graph_closed_form():
    g = synth.workload("product16x6")
    has2, t2, cost = synth.product_tables(6, 16, 0.3, 1, 1000, 0)
    locals_ = [synth.local_automaton(has2, t2, cost, i) for i in range(6)]
    sol = native.solve(g.row_ptr, g.col, g.w, tie=False, want_V=True)
    assert sol.value == closed.product_optimum(locals_)
    assert native.certify(g.row_ptr, g.col, g.w, sol.p, sol.q, sol.cycle, sol.V, sol.L) == 0


def _mid_graphs():
    return [synth.random_digraph(n, 1, 4, lo, hi, np.int64, seed)
            for n, lo, hi, seed in ((300, 1, 20, 0), (1000, 1, 100, 1), (2000, -1000, 1000, 2),
                                    (500, 7, 7, 3))]


@pytest.mark.parametrize("gi", range(4))
def test_karp_agrees_on_midsize_graphs(gi):
    g = _mid_graphs()[gi]
    for mode in ("min", "max"):
        sol = native.solve(g.row_ptr, g.col, g.w, mode=mode, want_V=True)
        k = native.karp(g.row_ptr, g.col, g.w if mode == "min" else -g.w)
        assert sol.value == (k if mode == "min" else -k)
        assert native.certify(g.row_ptr, g.col, g.w, sol.p, sol.q, sol.cycle,
                              sol.V, sol.L, mode) == 0
        assert int(g.w.min()) <= sol.value <= int(g.w.max())


@pytest.mark.parametrize("gi", range(4))
def test_invariants_shift_scale_negate_relabel(gi):
    g = _mid_graphs()[gi]
    base = native.solve(g.row_ptr, g.col, g.w)
    for c in (-17, 0, 5, 1000):
        s = native.solve(g.row_ptr, g.col, g.w + c)
        assert s.value == base.value + c
        assert (s.cycle.tolist(), s.iterations, s.source, s.tie) == \
            (base.cycle.tolist(), base.iterations, base.source, base.tie)
    for k in (1, 2, 7):
        s = native.solve(g.row_ptr, g.col, g.w * k)
        assert s.value == base.value * k
        assert (s.cycle.tolist(), s.iterations) == (base.cycle.tolist(), base.iterations)
    s = native.solve(g.row_ptr, g.col, -g.w, mode="max")
    assert s.value == -base.value
    assert (s.cycle.tolist(), s.iterations, s.tie) == (base.cycle.tolist(), base.iterations, base.tie)
    # relabel vertices: the value is unchanged
    rng = np.random.default_rng(gi)
    perm = rng.permutation(g.n)          # old -> new
    inv = np.argsort(perm)
    rp = [0]
    cl, ww = [], []
    for newv in range(g.n):
        oldv = inv[newv]
        a, b = g.row_ptr[oldv], g.row_ptr[oldv + 1]
        cl.extend(perm[g.col[a:b]].tolist())
        ww.extend(g.w[a:b].tolist())
        rp.append(len(cl))
    s = native.solve(np.array(rp), np.array(cl), np.array(ww))
    assert s.value == base.value


def test_certificate_rejects_planted_mistakes():
    g = _mid_graphs()[1]
    sol = native.solve(g.row_ptr, g.col, g.w, want_V=True)
    args = (g.row_ptr, g.col, g.w)
    assert native.certify(*args, sol.p, sol.q, sol.cycle, sol.V, sol.L) == 0
    # a claimed mean that the cycle does not have
    assert native.certify(*args, sol.p + 1, sol.q, sol.cycle, sol.V, sol.L) != 0
    # an edge with a violated potential inequality
    V = sol.V.copy()
    bad = int(np.argmax(V))
    V[bad] += 10**6
    assert native.certify(*args, sol.p, sol.q, sol.cycle, V, sol.L) == native.ORC_E_CERT_POTENTIAL
    # a walk that does not close
    if len(sol.cycle) > 1:
        assert native.certify(*args, sol.p, sol.q, sol.cycle[:-1], sol.V, sol.L) != 0
    # a non-optimal cycle: the ring, with the optimum's potential
    ring = g.row_ptr[1:] - 1
    wr = Fraction(int(g.w[ring].sum()), g.n)
    assert native.certify(*args, wr.numerator, wr.denominator, ring, sol.V, sol.L) != 0


def test_max_iters_and_bounds():
    g = _mid_graphs()[1]
    with pytest.raises(native.OracleError) as ex:
        native.solve(g.row_ptr, g.col, g.w, max_iters=1)
    assert ex.value.code == native.ORC_E_NOT_CONVERGED
    full = native.solve(g.row_ptr, g.col, g.w)
    ok = native.solve(g.row_ptr, g.col, g.w, max_iters=full.iterations)
    assert ok.value == full.value


@pytest.mark.parametrize("ring,tail,extra,hlo,hhi,seed",
                         [(700, 800, 2, 2**47, 2**48, 1), (128, 3000, 3, 2**47, 2**48, 2),
                          (300, 3000, 1, 2**46, 2**47, 4)])
def test_deep_tail_values_leave_int64(ring, tail, extra, hlo, hhi, seed):
    """The int128 instances: the optimum is the light ring's mean (closed form,
    and Karp's value), every weight passes the 2 n max|w| < 2^62 bound, yet the
    optimum's potential does not fit int64 (the oracle keeps it in int128 and
    refuses to export it as int64)."""
    g = synth.deep_tail_graph(ring, tail, extra, 10, hlo, hhi, seed)
    assert 2 * g.n * int(np.abs(g.w).max()) < 2**62
    ring_w = g.w[g.row_ptr[:ring]]
    want = Fraction(int(ring_w.sum()), ring)
    sol = native.solve(g.row_ptr, g.col, g.w)
    assert sol.value == want == native.karp(g.row_ptr, g.col, g.w)
    assert sorted(int(e) for e in sol.cycle) == sorted(int(e) for e in g.row_ptr[:ring])
    with pytest.raises(native.OracleError) as ei:
        native.solve(g.row_ptr, g.col, g.w, want_V=True)
    assert ei.value.code == native.ORC_E_OVERFLOW
