"""Writes the sequential policy-iteration oracle's results on the full-size
workloads: tests/golden/workloads.json (single graphs) and
tests/golden/batch4096.json (every graph of the batched workload).

Calls only ``oracle/`` (and the seeded generators).  Run from the repo root:
    python tests/golden/make_golden.py [name ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import native  # noqa: E402
from paper_1111_0627_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "workloads.json")
BATCH_OUT = os.path.join(HERE, "batch4096.json")
NAMES = ["rand1k", "rand1m_max", "product16x6", "rand4m_i64", "hub1m", "batch4096"]


def _batch_one(k):
    g = _BATCH[k]
    s = native.solve(g.row_ptr, g.col, g.w, mode="min", tie=True)
    return dict(n=g.n, m=g.m, p=s.p, q=s.q, cycle=s.cycle.tolist(), source=s.source,
                iterations=s.iterations, tie=s.tie, tight=s.tight)


_BATCH = None


def batch_golden(procs=6):
    """Every graph of the batched workload, one oracle solve each (cycles as
    CSR positions local to the graph)."""
    global _BATCH
    import multiprocessing as mp
    t = time.time()
    _BATCH = synth.batch_graphs()
    with mp.get_context("fork").Pool(procs) as pool:
        per = pool.map(_batch_one, range(len(_BATCH)), chunksize=16)
    dt = time.time() - t
    out = dict(recipe=synth.WORKLOADS["batch4096"]["desc"], mode="min", graphs=len(per),
               oracle_seconds_wall=round(dt, 1), oracle_processes=procs, per_graph=per)
    with open(BATCH_OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("batch4096", len(per), "graphs", round(dt, 1), "s", flush=True)


def main(names):
    if "batch4096" in names:
        batch_golden()
        names = [x for x in names if x != "batch4096"]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        mode = synth.WORKLOADS[name]["mode"]
        g = synth.workload(name)
        t = time.time()
        s = native.solve(g.row_ptr, g.col, g.w, mode=mode, tie=True)
        dt = time.time() - t
        data[name] = dict(mode=mode, n=g.n, m=g.m, p=s.p, q=s.q, W=s.W, L=s.L,
                          cycle=s.cycle.tolist(), source=s.source, iterations=s.iterations,
                          tie=s.tie, tight=s.tight, oracle_seconds=round(dt, 2),
                          recipe=synth.WORKLOADS[name]["desc"])
        print(name, data[name]["p"], data[name]["q"], data[name]["iterations"], round(dt, 1),
              flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
