"""Parity of the multichain variant (ocm_options.multichain) with the
multichain oracle: the optimum, C, the source, the sweep count, the tight
non-policy edge count, the tie flag, the final policy and every vertex's
value (scaled by the length of the cycle it reaches) must be identical."""

import json
import os

import numpy as np
import pytest
import torch

from oracle import brute, native
from paper_1111_0627_amd import ocm, synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ocm.lib()
    yield
    ocm.release_workspace()


def to_dev(rp, cl, w, wdtype=np.int64):
    return (torch.from_numpy(np.ascontiguousarray(rp, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(cl, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(np.asarray(w).astype(wdtype))).cuda())


def check(rp, cl, w, mode="min", wdtype=np.int64, values=True, **kw):
    sol = native.solve_multichain(rp, cl, w, mode, want_V=values, want_pi=values)
    res = ocm.cycle_mean(*to_dev(rp, cl, w, wdtype), mode=mode, multichain=True,
                         want_policy=values, want_potential=values, **kw)
    got = (res.p, res.q, res.cycle_edges.cpu().tolist(), res.source, res.iterations,
           res.tight_edges, res.tie)
    exp = (sol.p, sol.q, sol.cycle.tolist(), sol.source, sol.iterations, sol.tight,
           bool(sol.tie))
    assert got == exp
    if values:
        assert np.array_equal(res.policy.cpu().numpy(), sol.pi)
        assert np.array_equal(res.potential.cpu().numpy(), sol.V)
    return res, sol


def test_hand_trace():
    with open(os.path.join(GOLD, "multichain_traces.json")) as f:
        for tr in json.load(f)["traces"]:
            rp, cl, w = (np.array(tr[k]) for k in ("row_ptr", "col", "w"))
            res, _ = check(rp, cl, w)
            r = tr["multichain"]
            assert (res.p, res.q, res.iterations) == (r["p"], r["q"], r["iterations"])
            assert res.potential.cpu().tolist() == r["V"]


def test_tiny_graphs_against_oracle():
    rng = np.random.default_rng(77)
    for it in range(300):
        n = int(rng.integers(1, 9))
        rp, cl, w = brute.random_tiny(rng, n, 3, -4, 4)
        check(rp, cl, w, "max" if it % 3 == 0 else "min")


@pytest.mark.parametrize("n,dlo,dhi,wlo,whi,seed", [
    (1, 1, 3, -5, 5, 1), (257, 1, 4, -50, 50, 2), (3000, 1, 6, 1, 100, 3),
    (20001, 2, 9, -1000, 1000, 4), (70000, 1, 3, 0, 3, 5), (100003, 4, 12, 1, 10**6, 6)])
@pytest.mark.parametrize("mode", ["min", "max"])
def test_random_graphs(n, dlo, dhi, wlo, whi, seed, mode):
    g = synth.random_digraph(n, dlo, dhi, wlo, whi, np.int64, seed=[13, seed])
    for wdtype in (np.int32, np.int64):
        check(g.row_ptr, g.col, g.w, mode, wdtype)


@pytest.mark.parametrize("G", [1, 4, 16, 64])
def test_lane_counts_agree(G):
    g = synth.random_digraph(30000, 1, 40, -20, 20, np.int64, seed=[14, G])
    check(g.row_ptr, g.col, g.w, schedule=G)


def test_equal_weights_all_tight():
    g = synth.random_digraph(5000, 1, 5, 3, 3, np.int64, seed=[15, 0])
    res, sol = check(g.row_ptr, g.col, g.w)
    assert res.tight_edges == g.m - g.n and res.tie


def test_ties_and_small_weight_ranges():
    for seed in range(6):
        g = synth.random_digraph(4000, 1, 4, 0, 2, np.int64, seed=[16, seed])
        check(g.row_ptr, g.col, g.w)
        check(g.row_ptr, g.col, g.w, "max")


def test_product_graph():
    g = synth.product_graph(5, 16, 0.3, 1, 1000, 0)
    res, sol = check(g.row_ptr, g.col, g.w, wdtype=np.int32)
    uni = native.solve(g.row_ptr, g.col, g.w)
    assert (res.p, res.q) == (uni.p, uni.q)


def test_values_overflow_is_reported():
    """Values stay int64 here: a deep heavy tail makes one leave 2^62."""
    g = synth.deep_tail_graph(700, 800, 2, 10, 2**47, 2**48, seed=1)
    with pytest.raises(ocm.OCMError) as ei:
        ocm.cycle_mean(*to_dev(g.row_ptr, g.col, g.w), multichain=True)
    assert ei.value.status == ocm.OCM_E_OVERFLOW


def test_rejected_combinations():
    g = synth.random_digraph(100, 1, 3, 1, 9, np.int64, seed=[17, 0])
    rp, cl, w = to_dev(g.row_ptr, g.col, g.w)
    t = torch.ones(g.m, dtype=torch.int32, device="cuda")
    for call in (lambda: ocm.cycle_mean(rp, cl, w, multichain=True, int128=True),
                 lambda: ocm.min_cycle_ratio(rp, cl, w, t, multichain=True),
                 lambda: ocm.cycle_mean(rp, cl, w, multichain=True,
                                        init_policy=rp[:-1].clone())):
        with pytest.raises(ocm.OCMError) as ei:
            call()
        assert ei.value.status == ocm.OCM_E_INVALID_ARG


def test_noalloc_entry_point():
    g = synth.random_digraph(20000, 1, 5, -30, 30, np.int64, seed=[18, 0])
    rp, cl, w = to_dev(g.row_ptr, g.col, g.w)
    a = ocm.cycle_mean(rp, cl, w, multichain=True)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    b = ocm.min_cycle_mean_noalloc(rp, cl, w, out, multichain=True)
    assert (a.p, a.q, a.iterations, a.tight_edges, a.tie) == \
        (b.p, b.q, b.iterations, b.tight_edges, b.tie)
    assert a.cycle_edges.cpu().tolist() == b.cycle_edges.cpu().tolist()


def test_giant_rows():
    """The first sweep takes giant rows (more than 8192 edges) through the
    multi-workgroup path; the later sweeps use lanes per vertex."""
    g = synth.hub_graph(5000, 3, 20000, 1, 4, -10, 10, np.int64, seed=[19, 0])
    check(g.row_ptr, g.col, g.w)
    check(g.row_ptr, g.col, g.w, "max")
