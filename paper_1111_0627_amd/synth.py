"""Seeded synthetic graph generators.

This module only builds inputs: CSR arrays (``row_ptr``, ``col``) and integer
edge weights ``w``.  It contains none of the cycle-mean arithmetic, so both the
HIP path and the CPU oracle can consume the same arrays without sharing code.

Graphs are stored in the adjacency-list form of Section 2.3 (Fig. 2b): an
offsets array of n+1 entries and a target array of m entries ordered by source
vertex.  Edge weights are a separate array in the same order as the targets.

Every draw uses ``numpy.random.Generator(PCG64(seed))`` in a fixed order, so a
(recipe, seed) pair always yields identical arrays.

Recipes
-------
``random_digraph(n, dlo, dhi, wlo, whi, wdtype, seed)``
    1. ``deg = integers(dlo, dhi + 1, n)``
    2. ``tgt = integers(0, n, deg.sum())``
    3. vertex v gets its ``deg[v]`` random targets in draw order, then the
       ring edge v -> (v + 1) mod n, which makes the graph strongly connected
       (the Hamiltonian-cycle augmentation of Section 2.5).  Self-loops and
       duplicate targets are kept.
    4. ``w = integers(wlo, whi + 1, m)`` in final CSR order, cast to wdtype.

``deep_tail_graph(ring, tail, extra, wlight, hlo, hhi, seed)``
    A light ring 0 .. ring-1 fed by a long heavy tail, so that the optimum's
    values grow like tail * ring * hhi (beyond int64 for large weights) while
    every single weight stays small.
    1. ``xt = integers(max(j - 8, 0), tail)`` for tail index j, ``extra``
       draws per tail vertex in one call (shape (tail, extra)): extra targets
       at most 8 steps nearer the ring, so every way to the ring crosses at
       least tail / 8 heavy edges;
    2. out-edges, in CSR order: ring vertex i -> (i + 1) mod ring, and ring
       vertex 0 also -> ring + tail - 1 (the tail's far end); tail vertex
       ring + j -> ring + j - 1 (ring vertex 0 for j = 0), then its extra
       targets ring + xt[j];
    3. ``w = integers(hlo, hhi + 1, m)`` in CSR order, then the ring edges'
       weights are redrawn as ``integers(0, wlight + 1, ring)`` (int64).
    Strongly connected; the minimum cycle mean is the ring's mean whenever
    hlo exceeds wlight.

``product_graph(procs, states, p2, wlo, whi, seed)``
    Interleaving product of ``procs`` local automata with ``states`` local
    states each, the shape of a model checker's state space (Section 4).
    1. ``has2 = random((procs, states)) < p2``
    2. ``t2 = integers(0, states - 1, (procs, states))``; values at or above
       the ring target (s + 1) mod states are shifted up by one, so the
       second target differs from the ring target (a local self-loop is
       allowed).
    3. ``cost = integers(wlo, whi + 1, (procs, states, states))`` int32
    4. global state v = sum_i s_i * states**i (process 0 least significant).
    5. out-edges of v, for i = 0 .. procs-1: the ring step s_i -> s_i + 1,
       then the second step s_i -> t2[i, s_i] if ``has2[i, s_i]``.  The
       weight of a step of process i from s to t is ``cost[i, s, t]``.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Graph:
    """A CSR digraph with integer edge weights (host numpy arrays)."""

    row_ptr: np.ndarray  # int32 [n + 1]
    col: np.ndarray      # int32 [m]
    w: np.ndarray        # int32 or int64 [m]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_digraph(n: int, dlo: int, dhi: int, wlo: int, whi: int,
                   wdtype=np.int32, seed=0, name: str = "") -> Graph:
    """Random digraph with a Hamiltonian ring; recipe in the module docstring."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    deg = rng.integers(dlo, dhi + 1, n)
    tgt = rng.integers(0, n, int(deg.sum()))
    outdeg = deg + 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(outdeg, out=row_ptr[1:])
    m = int(row_ptr[-1])
    if m >= 2**31:
        raise ValueError("edge count must stay below 2^31")
    col = np.empty(m, dtype=np.int32)
    ring_pos = row_ptr[1:] - 1
    is_ring = np.zeros(m, dtype=bool)
    is_ring[ring_pos] = True
    col[~is_ring] = tgt.astype(np.int32)
    col[ring_pos] = ((np.arange(n, dtype=np.int64) + 1) % n).astype(np.int32)
    w = rng.integers(wlo, whi + 1, m).astype(wdtype)
    return Graph(row_ptr.astype(np.int32), col, w, name)


def hub_graph(n: int, hubs: int, hub_deg: int, dlo: int, dhi: int, wlo: int, whi: int,
              wdtype=np.int64, seed=0, name: str = "") -> Graph:
    """random_digraph(n, dlo, dhi, ...) whose vertices 0, n/hubs, 2n/hubs, ...
    (``hubs`` of them) get ``hub_deg`` extra out-edges to uniform targets: a
    few rows far longer than the rest (power-law-like hubs)."""
    base = random_digraph(n, dlo, dhi, wlo, whi, wdtype, seed)
    rng = _rng([seed, 1] if isinstance(seed, int) else [*seed, 1])
    deg = np.diff(base.row_ptr.astype(np.int64))
    hub_ids = (np.arange(hubs, dtype=np.int64) * n) // max(hubs, 1)
    extra = np.zeros(n, np.int64)
    extra[hub_ids] = hub_deg
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(deg + extra, out=row_ptr[1:])
    m = int(row_ptr[-1])
    if m >= 2**31:
        raise ValueError("edge count must stay below 2^31")
    col = np.empty(m, np.int32)
    w = np.empty(m, wdtype)
    # each row: its base edges (ring edge last), then the hub's extra edges
    src_base = np.repeat(np.arange(n), deg)
    off_base = np.arange(base.row_ptr[-1]) - np.repeat(base.row_ptr[:-1].astype(np.int64), deg)
    pos_base = row_ptr[:-1][src_base] + off_base
    col[pos_base] = base.col
    w[pos_base] = base.w
    src_x = np.repeat(np.arange(n), extra)
    off_x = np.arange(int(extra.sum())) - np.repeat(np.cumsum(extra) - extra, extra)
    pos_x = row_ptr[:-1][src_x] + deg[src_x] + off_x
    col[pos_x] = rng.integers(0, n, len(pos_x)).astype(np.int32)
    w[pos_x] = rng.integers(wlo, whi + 1, len(pos_x)).astype(wdtype)
    return Graph(row_ptr.astype(np.int32), col, w, name)


def deep_tail_graph(ring: int, tail: int, extra: int = 2, wlight: int = 10,
                    hlo: int = 2**47, hhi: int = 2**48, seed=0, name: str = "") -> Graph:
    """Light ring fed by a long heavy tail; recipe in the module docstring."""
    if ring < 1 or tail < 1:
        raise ValueError("ring and tail must be >= 1")
    rng = _rng(seed)
    xt = rng.integers(np.maximum(np.arange(tail) - 8, 0)[:, None], tail, (tail, extra))
    n = ring + tail
    deg = np.ones(n, np.int64)
    deg[0] += 1
    deg[ring:] += extra
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    m = int(row_ptr[-1])
    col = np.empty(m, np.int32)
    rs = row_ptr[:ring]
    col[rs] = (np.arange(ring) + 1) % ring
    col[rs[0] + 1] = ring + tail - 1
    ts = row_ptr[ring:n]
    j = np.arange(tail)
    col[ts] = np.where(j == 0, 0, ring + j - 1)
    for k in range(extra):
        col[ts + 1 + k] = ring + xt[:, k]
    w = rng.integers(hlo, hhi + 1, m).astype(np.int64)
    w[rs] = rng.integers(0, wlight + 1, ring)
    return Graph(row_ptr.astype(np.int32), col, w, name)


def product_tables(procs: int, states: int, p2: float, wlo: int, whi: int,
                   seed=0):
    """The local automata of ``product_graph``: (has2, t2, cost)."""
    rng = _rng(seed)
    has2 = rng.random((procs, states)) < p2
    t2 = rng.integers(0, states - 1, (procs, states))
    ring_t = (np.arange(states) + 1) % states
    t2 = t2 + (t2 >= ring_t[None, :])
    cost = rng.integers(wlo, whi + 1, (procs, states, states)).astype(np.int32)
    return has2, t2.astype(np.int64), cost


def local_automaton(has2, t2, cost, i: int) -> Graph:
    """Process i's own automaton as a CSR graph (ring step, then second step)."""
    states = has2.shape[1]
    rp = [0]
    col, w = [], []
    for s in range(states):
        r = (s + 1) % states
        col.append(r)
        w.append(int(cost[i, s, r]))
        if has2[i, s]:
            col.append(int(t2[i, s]))
            w.append(int(cost[i, s, t2[i, s]]))
        rp.append(len(col))
    return Graph(np.array(rp, np.int32), np.array(col, np.int32),
                 np.array(w, np.int32), f"local{i}")


def product_graph(procs: int = 6, states: int = 16, p2: float = 0.3,
                  wlo: int = 1, whi: int = 1000, seed=0,
                  name: str = "") -> Graph:
    """Interleaving product of local automata; recipe in the module docstring."""
    has2, t2, cost = product_tables(procs, states, p2, wlo, whi, seed)
    n = states ** procs
    if n >= 2**31:
        raise ValueError("vertex count must stay below 2^31")
    v = np.arange(n, dtype=np.int64)
    digits = [(v // states**i) % states for i in range(procs)]
    extra = [has2[i][digits[i]].astype(np.int64) for i in range(procs)]
    deg = procs + sum(extra)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    m = int(row_ptr[-1])
    if m >= 2**31:
        raise ValueError("edge count must stay below 2^31")
    col = np.empty(m, dtype=np.int32)
    w = np.empty(m, dtype=np.int32)
    off = row_ptr[:-1].copy()
    for i in range(procs):
        s = digits[i]
        stride = states ** i
        r = (s + 1) % states
        col[off] = (v + (r - s) * stride).astype(np.int32)
        w[off] = cost[i, s, r]
        off += 1
        sel = extra[i].astype(bool)
        o2 = off[sel]
        s2 = s[sel]
        t = t2[i][s2]
        col[o2] = (v[sel] + (t - s2) * stride).astype(np.int32)
        w[o2] = cost[i, s2, t]
        off += extra[i]
        del s, r, sel, o2, s2, t
    return Graph(row_ptr.astype(np.int32), col, w, name)


def batch_sizes(G: int = 4096, lo: int = 100, hi: int = 100_000, seed=0):
    """Log-uniform graph sizes of the batched workload."""
    rng = _rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi), G)
    return np.clip(np.round(np.exp(u)), lo, hi).astype(np.int64)


def batch_graphs(G: int = 4096, lo: int = 100, hi: int = 100_000,
                 dlo: int = 1, dhi: int = 8, wlo: int = 1, whi: int = 10_000,
                 seed=0):
    """The batched workload: G independent random digraphs (seed [seed, g])."""
    sizes = batch_sizes(G, lo, hi, seed)
    return [random_digraph(int(sizes[g]), dlo, dhi, wlo, whi, np.int32,
                           seed=[seed, g], name=f"b{g}") for g in range(G)]


def disjoint_union(graphs):
    """Concatenate graphs into one CSR with global vertex ids.

    Returns (Graph, vptr, eptr) where graph g owns vertices
    [vptr[g], vptr[g+1]) and edges [eptr[g], eptr[g+1]).
    """
    G = len(graphs)
    vptr = np.zeros(G + 1, np.int64)
    eptr = np.zeros(G + 1, np.int64)
    vptr[1:] = np.cumsum([g.n for g in graphs])
    eptr[1:] = np.cumsum([g.m for g in graphs])
    if vptr[-1] >= 2**31 or eptr[-1] >= 2**31:
        raise ValueError("union must stay below 2^31 vertices and edges")
    row_ptr = np.empty(int(vptr[-1]) + 1, np.int64)
    col = np.empty(int(eptr[-1]), np.int32)
    wdt = np.result_type(*[g.w.dtype for g in graphs])
    w = np.empty(int(eptr[-1]), wdt)
    for k, g in enumerate(graphs):
        v0, e0 = int(vptr[k]), int(eptr[k])
        row_ptr[v0:v0 + g.n] = g.row_ptr[:-1].astype(np.int64) + e0
        col[e0:e0 + g.m] = g.col.astype(np.int64) + v0
        w[e0:e0 + g.m] = g.w
    row_ptr[-1] = eptr[-1]
    return Graph(row_ptr.astype(np.int32), col, w, "union"), vptr, eptr


# The five measured workloads, by name.
def workload(name: str) -> Graph:
    if name == "rand1k":
        return random_digraph(1000, 1, 4, 1, 100, np.int32, 0, name)
    if name == "rand1m_max":
        return random_digraph(2**20, 2, 10, 1, 10_000, np.int32, 0, name)
    if name == "product16x6":
        return product_graph(6, 16, 0.3, 1, 1000, 0, name)
    if name == "rand4m_i64":
        return random_digraph(2**22, 2, 6, 1, 2**20, np.int64, 0, name)
    if name == "hub1m":
        return hub_graph(2**20, 8, 2**20, 2, 6, 1, 1000, np.int64, 0, name)
    raise KeyError(name)


WORKLOADS = {
    "rand1k": dict(mode="min", desc="random digraph n=1000, deg 1-4 + ring, w int32 in [1,100], seed 0"),
    "rand1m_max": dict(mode="max", desc="random digraph n=2^20, deg 2-10 + ring, w int32 in [1,10000], seed 0, maximum"),
    "product16x6": dict(mode="min", desc="interleaving product of 6 automata x 16 states (n=16^6), p2=0.3, w int32 in [1,1000], seed 0"),
    "batch4096": dict(mode="min", desc="4096 random digraphs, n log-uniform in [100,1e5], deg 1-8 + ring, w int32 in [1,10000]"),
    "rand4m_i64": dict(mode="min", desc="random digraph n=2^22, deg 2-6 + ring, w int64 in [1,2^20], seed 0"),
    "hub1m": dict(mode="min", desc="random digraph n=2^20, deg 2-6 + ring, plus 8 hubs of 2^20 extra out-edges, "
                                   "w int64 in [1,1000], seed 0"),
}
