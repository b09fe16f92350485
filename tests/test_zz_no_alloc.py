"""ocm_min_noalloc (the entry point for callers that cannot allocate) gives
the same bytes as ocm_min with a caller workspace, through the C ABI, on
consecutive calls that reuse the library's static per-GPU scratch array (the
second call smaller than the first, so stale contents of the first are
present), and rejects graphs whose scratch would exceed the array."""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_1111_0627_amd import ocm, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ocm.lib()
    yield
    ocm.release_workspace()


def _dev(g):
    return (torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(),
            torch.from_numpy(g.w).cuda())


def _raw_min(G, n):
    """ocm_min through the C ABI with a workspace of exactly the needed size."""
    L = ocm.lib()
    need = L.ocm_workspace_size(C.byref(G), None)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    cyc = torch.empty(n, dtype=torch.int32, device="cuda")
    res = ocm._Result()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.ocm_min(C.byref(G), None, C.c_void_p(ws.data_ptr()), need, C.c_void_p(cyc.data_ptr()),
                   n, C.byref(res), st)
    assert rc == ocm.OCM_OK, L.ocm_last_error()
    return res, cyc[:res.cycle_len].cpu().tolist()


def _raw_noalloc(G, n):
    L = ocm.lib()
    cyc = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    res = ocm._Result()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.ocm_min_noalloc(C.byref(G), None, C.c_void_p(cyc.data_ptr()), n, C.byref(res), st)
    assert rc == ocm.OCM_OK, L.ocm_last_error()
    return res, cyc[:res.cycle_len].cpu().tolist()


def _key(res, cyc):
    return (res.p, res.q, cyc, res.source, res.iterations, res.flags, res.W, res.L,
            res.tight_edges, res.connect_rounds, res.jump_rounds, res.fast_iters)


def _case(g):
    rp, cl, w = _dev(g)
    G = ocm.make_graph(rp, cl, w)
    assert ocm.lib().ocm_workspace_size(C.byref(G), None) <= ocm.NOALLOC_SCRATCH_BYTES
    want = _key(*_raw_min(G, g.n))
    got = _key(*_raw_noalloc(G, g.n))
    assert got == want
    return got


def test_noalloc_matches_ocm_min_on_consecutive_calls():
    big = synth.random_digraph(1 << 20, 2, 10, 1, 10000, np.int32, seed=0)
    small = synth.random_digraph(3001, 1, 4, 1, 100, np.int32, seed=5)
    a = _case(big)
    b = _case(small)
    assert a != b
    # the small graph again after the large one, and int64 weights
    w64 = synth.random_digraph(4099, 1, 8, 1, 1 << 20, np.int64, seed=9)
    _case(w64)
    _case(small)


def test_noalloc_binding_and_rejections():
    g = synth.random_digraph(777, 1, 3, -50, 50, np.int32, seed=2)
    rp, cl, w = _dev(g)
    cyc = torch.empty(g.n, dtype=torch.int32, device="cuda")
    r = ocm.min_cycle_mean_noalloc(rp, cl, w, cyc)
    e = ocm.min_cycle_mean(rp, cl, w)
    assert (r.p, r.q, r.cycle_edges.cpu().tolist(), r.iterations) == \
        (e.p, e.q, e.cycle_edges.cpu().tolist(), e.iterations)
    # a graph whose scratch exceeds the array is refused before any device work
    L = ocm.lib()
    huge = ocm.Graph(1 << 24, 1 << 27, rp.data_ptr(), cl.data_ptr(), w.data_ptr(), 0)
    res = ocm._Result()
    rc = L.ocm_min_noalloc(C.byref(huge), None, C.c_void_p(cyc.data_ptr()), g.n, C.byref(res),
                           None)
    assert rc == ocm.OCM_E_WORKSPACE
    assert b"scratch" in L.ocm_last_error()
    # profile is refused
    o = ocm.options()
    prof = ocm.Profile()
    o.profile = C.pointer(prof)
    G = ocm.make_graph(rp, cl, w)
    rc = L.ocm_min_noalloc(C.byref(G), C.byref(o), C.c_void_p(cyc.data_ptr()), g.n,
                           C.byref(res), None)
    assert rc == ocm.OCM_E_INVALID_ARG
    # the array still works after the refusals
    r2 = ocm.min_cycle_mean_noalloc(rp, cl, w, cyc)
    assert (r2.p, r2.q, r2.iterations) == (e.p, e.q, e.iterations)
