"""Differentiation of the exact optimum through the C ABI: the adjoint
scatter, the exact uniqueness test it relies on, warm starts, and exact
finite differences (each perturbed solve certified by the oracle)."""

from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import brute, native
from paper_1111_0627_amd import autograd, gradcheck, ocm, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ocm.lib()
    yield
    ocm.release_workspace()


def dev_graph(g):
    return (torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.w, np.int64)).cuda())


def test_weights_from_f64_checks_integrality():
    w = torch.tensor([1.0, -3.0, 2.0**52, -(2.0**52)], dtype=torch.float64, device="cuda")
    assert ocm.weights_from_f64(w).cpu().tolist() == [1, -3, 2**52, -(2**52)]
    for bad in (0.5, 2.0**53, float("nan"), float("inf")):
        with pytest.raises(ocm.OCMError):
            ocm.weights_from_f64(torch.tensor([1.0, bad], dtype=torch.float64, device="cuda"))


def test_adjoint_scatter_pattern():
    m = 1000
    cyc = torch.tensor([5, 17, 999], dtype=torch.int32, device="cuda")
    g = torch.tensor(2.0, dtype=torch.float64, device="cuda")
    grad = ocm.adjoint_scatter(m, cyc, g).cpu().numpy()
    exp = np.zeros(m)
    exp[[5, 17, 999]] = 2.0 / 3.0
    assert np.array_equal(grad, exp)


@pytest.mark.parametrize("mode", ["min", "max"])
def test_cycle_mean_autograd_matches_analytic_gradient(mode):
    g = synth.random_digraph(20000, 2, 6, 1, 2**20, np.int64, 3)
    rp, cl, wi = dev_graph(g)
    w = wi.to(torch.float64).requires_grad_(True)
    val = autograd.cycle_mean(w, rp, cl, mode=mode)
    sol = native.solve(g.row_ptr, g.col, g.w, mode=mode)
    assert sol.tie == 0
    assert val.item() == float(Fraction(sol.p, sol.q))
    val.backward()
    grad = w.grad.cpu().numpy()
    exp = np.zeros(g.m)
    exp[sol.cycle] = 1.0 / len(sol.cycle)
    assert np.array_equal(grad, exp)


def test_backward_raises_on_ties():
    # two disjoint critical cycles joined by heavy edges
    rp = np.array([0, 1, 3, 4, 6], np.int32)
    cl = np.array([1, 0, 2, 3, 2, 0], np.int32)
    w = torch.tensor([1.0, 1.0, 5.0, 1.0, 1.0, 5.0], dtype=torch.float64, device="cuda",
                     requires_grad=True)
    rpt, clt = torch.from_numpy(rp).cuda(), torch.from_numpy(cl).cuda()
    val = autograd.cycle_mean(w, rpt, clt)
    with pytest.raises(autograd.TieError):
        val.backward()
    w.grad = None
    val = autograd.cycle_mean(w, rpt, clt, on_tie="ignore")
    val.backward()
    assert w.grad.cpu().tolist() == [0.5, 0.5, 0, 0, 0, 0]


def test_exact_tie_flag_against_brute_force():
    rng = np.random.default_rng(77)
    seen = {True: 0, False: 0}
    for i in range(300):
        n = int(rng.integers(2, 9))
        rp, cl, w = brute.random_tiny(rng, n, 3, 1, 6)
        val, crit = brute.optimum(rp, cl, w)
        res = ocm.min_cycle_mean(torch.from_numpy(rp).cuda(), torch.from_numpy(cl).cuda(),
                                 torch.from_numpy(w).cuda())
        assert res.value == val
        assert res.tie == (len(crit) > 1)
        seen[res.tie] += 1
    assert seen[True] > 20 and seen[False] > 20


def test_exact_tie_flag_on_larger_graphs():
    for seed in range(4):
        g = synth.random_digraph(30000, 1, 5, 1, 30, np.int32, 40 + seed)
        sol = native.solve(g.row_ptr, g.col, g.w)
        res = ocm.min_cycle_mean(*dev_graph(g))
        assert res.tight_edges == sol.tight
        assert res.tie == bool(sol.tie)


def test_warm_start_same_optimum_and_bad_policy_rejected():
    g = synth.random_digraph(50000, 2, 6, 1, 1000, np.int32, 5)
    rp, cl, w = dev_graph(g)
    cold = ocm.min_cycle_mean(rp, cl, w, want_policy=True)
    again = ocm.min_cycle_mean(rp, cl, w, init_policy=cold.policy)
    assert again.value == cold.value and again.iterations == 1
    w2 = w.clone()
    w2[123] -= 50
    warm = ocm.min_cycle_mean(rp, cl, w2, init_policy=cold.policy)
    ref = native.solve(g.row_ptr, g.col, w2.cpu().numpy())
    assert warm.value == ref.value
    bad = cold.policy.clone()
    bad[7] = int(g.row_ptr[9])
    with pytest.raises(ocm.OCMError) as ex:
        ocm.min_cycle_mean(rp, cl, w, init_policy=bad)
    assert ex.value.status == ocm.OCM_E_INVALID_ARG


@pytest.mark.parametrize("mode", ["min", "max"])
def test_exact_finite_differences(mode):
    g = synth.random_digraph(20000, 2, 6, 1, 2**20, np.int64, 11)
    rp, cl, w = dev_graph(g)
    base = ocm.cycle_mean(rp, cl, w, mode=mode, want_policy=True)
    edges = gradcheck.stratified_edges(base.cycle_edges.cpu().numpy(), g.row_ptr, g.m, total=120)
    assert set(base.cycle_edges.cpu().tolist()) <= set(edges.tolist())
    certified = []

    def certify(e, delta, r):
        ww = g.w.astype(np.int64).copy()
        ww[e] += delta
        pot = ocm.cycle_mean(rp, cl, torch.from_numpy(ww).cuda(), mode=mode,
                             want_potential=True, init_policy=base.policy)
        assert (pot.p, pot.q) == (r.p, r.q)
        certified.append(native.certify(g.row_ptr, g.col, ww, pot.p, pot.q,
                                        pot.cycle_edges.cpu().numpy(),
                                        pot.potential.cpu().numpy(), pot.L, mode) == 0)

    rep = gradcheck.fd_check(rp, cl, w, edges, mode=mode, base=base, w_host=g.w, on_solve=certify)
    assert rep.checked == 2 * len(edges)
    assert rep.failed == 0, rep.details
    assert rep.exact > 0.9 * rep.checked
    assert all(certified)
