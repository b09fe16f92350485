"""Differentiable exact optimal cycle mean.

Away from ties the optimum mu*(w) equals the mean of its critical cycle C,
w(C)/|C|, on a neighbourhood of w, so d(mu*)/d(w_e) = 1/|C| for e in C and 0
for every other edge.  (The same holds for the maximum cycle mean.)  When C
is not the unique critical cycle the optimum is a minimum (maximum) of
several such linear functions and has no gradient there; the exact
uniqueness test of the forward pass reports this, and ``on_tie`` decides
what backward does.

torch cannot attach gradients to integer tensors, so weights come in as
float64 holding integers with |w| < 2^53; the device converts them to int64
(ocm_weights_from_f64) and the solve stays exact.
"""

from __future__ import annotations

import warnings
from fractions import Fraction

import torch

from . import ocm


class TieError(ocm.OCMError):
    """The critical cycle is not unique, so the optimum has no gradient."""


class CycleMean(torch.autograd.Function):
    """value, p, q = CycleMean.apply(w, row_ptr, col, mode, on_tie, init_policy)

    value is p/q as float64 (correctly rounded); p and q are int64 and not
    differentiable.  on_tie: "raise" (default), "warn" or "ignore" in
    backward when C is not unique (or uniqueness was not decided).
    """

    @staticmethod
    def forward(ctx, w, row_ptr, col, mode="min", on_tie="raise", init_policy=None):
        if on_tie not in ("raise", "warn", "ignore"):
            raise ValueError("on_tie must be 'raise', 'warn' or 'ignore'")
        wi = ocm.weights_from_f64(w.detach().contiguous())
        res = ocm.cycle_mean(row_ptr, col, wi, mode=mode, init_policy=init_policy)
        ctx.save_for_backward(res.cycle_edges)
        ctx.m = w.numel()
        ctx.tie = res.tie
        ctx.on_tie = on_tie
        dev = w.device
        value = torch.tensor(float(Fraction(res.p, res.q)), dtype=torch.float64, device=dev)
        p = torch.tensor(res.p, dtype=torch.int64, device=dev)
        q = torch.tensor(res.q, dtype=torch.int64, device=dev)
        ctx.mark_non_differentiable(p, q)
        return value, p, q

    @staticmethod
    def backward(ctx, g, gp=None, gq=None):
        (cyc,) = ctx.saved_tensors
        if ctx.tie is not False:
            msg = ("the critical cycle is not unique (or uniqueness was not decided): "
                   "the optimum has no gradient here")
            if ctx.on_tie == "raise":
                raise TieError(ocm.OCM_E_INVALID_ARG, msg)
            if ctx.on_tie == "warn":
                warnings.warn(msg, RuntimeWarning, stacklevel=2)
        grad = ocm.adjoint_scatter(ctx.m, cyc, g)
        return grad, None, None, None, None, None


def cycle_mean(w, row_ptr, col, mode: str = "min", on_tie: str = "raise", init_policy=None):
    """Differentiable optimum (float64 0-dim tensor) of float64 integral weights."""
    value, _, _ = CycleMean.apply(w, row_ptr, col, mode, on_tie, init_policy)
    return value
