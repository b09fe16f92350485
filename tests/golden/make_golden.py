"""Writes tests/golden/workloads.json: the sequential policy-iteration
oracle's results on the full-size workloads.

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
NAMES = ["rand1k", "rand1m_max", "product16x6", "rand4m_i64"]


def main(names):
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
