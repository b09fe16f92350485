"""Closed forms for the optimal cycle mean of structured graphs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* A graph that is a single directed ring has exactly one cycle, so its optimum
  is the ring's weight sum divided by its length.
* For the interleaving product of local automata P_1..P_k (every global edge
  moves one process along one of its local edges, at that local edge's cost),
  the minimum cycle mean equals the smallest minimum cycle mean among the P_i:
  a global cycle projects onto a closed walk in every P_i and its mean is the
  length-weighted average of those walks' means, each at least that process's
  optimum; and a local cycle of P_i, taken with every other process frozen,
  is itself a global cycle.  (Prop. 2.2 is the analogous statement for the
  strongly connected components of one graph.)  Each P_i is tiny, so its
  optimum comes from brute-force enumeration.
"""

from __future__ import annotations

from fractions import Fraction

from . import brute


def ring_mean(w) -> Fraction:
    return Fraction(int(sum(int(x) for x in w)), len(w))


def product_optimum(local_graphs, mode: str = "min") -> Fraction:
    vals = [brute.optimum(g.row_ptr, g.col, g.w, mode)[0] for g in local_graphs]
    return min(vals) if mode == "min" else max(vals)
