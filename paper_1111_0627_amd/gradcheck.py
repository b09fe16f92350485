"""Exact finite-difference check of d(optimum)/d(w).

For a sampled edge e the forward differences with unit steps,
    FD+ = mu*(w + 1_e) - mu*(w),   FD- = mu*(w) - mu*(w - 1_e),
are computed exactly (each mu* is a rational p/q from an exact solve).
Expected: 1/|C| for e in the critical cycle C, 0 otherwise.  A unit step
moves the mean of a simple cycle through e by exactly 1/|cycle|, so FD+- can
differ from the gradient only if another cycle C' is within
max(1/|C|, 1/|C'|) of mu* before the step; such a mismatch is flagged (with
C' as the witness the perturbed solve returned) instead of failed.  For
e not in C, FD+ = 0 always.

Each perturbed solve is warm-started from the unperturbed optimal policy.
It ends with a full sweep finding no improving edge, i.e. its potential is
feasible, so it certifies its own optimum.
"""

from __future__ import annotations

import dataclasses
from fractions import Fraction

import numpy as np
import torch

from . import ocm


def stratified_edges(cycle_edges: np.ndarray, row_ptr: np.ndarray, m: int, total: int = 1000,
                     seed: int = 0) -> np.ndarray:
    """All edges of C (at most half the sample), up to a quarter of the
    sample from C's vertices' other out-edges, the rest uniform over E."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cyc = np.asarray(cycle_edges, dtype=np.int64)
    chosen = list(cyc[: total // 2])
    cset = set(int(e) for e in cyc)
    srcs = np.searchsorted(row_ptr, cyc, side="right") - 1
    near = [e for v in srcs for e in range(int(row_ptr[v]), int(row_ptr[v + 1])) if e not in cset]
    near = sorted(set(near))
    k = min(len(near), total // 4)
    if k:
        chosen += list(rng.choice(np.array(near, np.int64), size=k, replace=False))
    have = set(int(e) for e in chosen)
    want = min(total, m) - len(chosen)
    while want > 0:
        cand = rng.integers(0, m, size=2 * want + 16)
        for e in cand:
            e = int(e)
            if e not in have:
                have.add(e)
                chosen.append(e)
                want -= 1
                if want == 0:
                    break
    return np.array(chosen, dtype=np.int64)


@dataclasses.dataclass
class FDReport:
    checked: int = 0
    exact: int = 0
    flagged: int = 0
    failed: int = 0
    details: list = dataclasses.field(default_factory=list)

    def as_dict(self):
        return dict(checked=self.checked, exact=self.exact, flagged=self.flagged,
                    failed=self.failed)


def fd_check(row_ptr: torch.Tensor, col: torch.Tensor, w: torch.Tensor, edges, mode: str = "min",
             base=None, w_host: np.ndarray | None = None, on_solve=None) -> FDReport:
    """Checks the analytic gradient against exact unit finite differences on
    `edges` (int64 weights on the GPU).  on_solve(e, delta, result), if
    given, sees every perturbed solve (e.g. to certify it)."""
    if base is None:
        base = ocm.cycle_mean(row_ptr, col, w, mode=mode, want_policy=True)
    if w_host is None:
        w_host = w.cpu().numpy()
    mu = Fraction(base.p, base.q)
    cyc = base.cycle_edges.cpu().numpy()
    cset = set(int(e) for e in cyc)
    L = len(cyc)
    rp_host = row_ptr.cpu().numpy()
    col_host = col.cpu().numpy()
    work = w.clone()
    rep = FDReport()
    for e in edges:
        e = int(e)
        expected = Fraction(1, L) if e in cset else Fraction(0)
        for delta in (1, -1):
            work[e] += delta
            r = ocm.cycle_mean(row_ptr, col, work, mode=mode, init_policy=base.policy)
            work[e] -= delta
            if on_solve is not None:
                on_solve(e, delta, r)
            fd = (Fraction(r.p, r.q) - mu) * delta
            rep.checked += 1
            if fd == expected:
                rep.exact += 1
                continue
            # explain the mismatch by the perturbed solve's cycle C'
            c2 = r.cycle_edges.cpu().numpy()
            ok = False
            if len(c2) and set(int(x) for x in c2) != cset:
                # C' must be a cycle whose perturbed mean is the new optimum
                pert = [int(w_host[x]) + (delta if int(x) == e else 0) for x in c2]
                closed = all(int(col_host[c2[i]]) ==
                             int(np.searchsorted(rp_host, c2[(i + 1) % len(c2)], side="right") - 1)
                             for i in range(len(c2)))
                mu2 = Fraction(int(sum(int(w_host[x]) for x in c2)), len(c2))
                if closed and Fraction(sum(pert), len(c2)) == Fraction(r.p, r.q):
                    gap = abs(mu2 - mu)
                    ok = gap <= max(Fraction(1, L), Fraction(1, len(c2)))
            if ok:
                rep.flagged += 1
            else:
                rep.failed += 1
            rep.details.append(dict(edge=e, delta=delta, fd=str(fd), expected=str(expected),
                                    witness_len=len(c2), explained=ok))
    return rep
