"""torch.autograd binding of the CTMRG fixed point: (f, E, M) as functions of K.

The forward pass runs the library to its fixed point; the backward pass calls
ctmrg_backward (implicit differentiation through the fixed point, see
include/ctmrg.h), which gives df/dK, dE/dK = d2F/dK2 and dM/dK from one tangent
solve.  Torch only carries the scalars; all work runs in the library.
"""
from __future__ import annotations

import torch

from . import ctmrg


class CTMRGFixedPoint(torch.autograd.Function):
    """f, E, M = CTMRGFixedPoint.apply(K, V, m, tol, max_steps) for a 0-d float64 tensor K."""

    @staticmethod
    def forward(ctx, K, V, m, tol=1e-13, max_steps=3000):
        g = ctmrg.CTMRG(V, float(K.item()), int(m))
        steps, delta, conv = g.run_to_fixed_point(tol, max_steps)
        if not conv:
            g.close()
            raise ctmrg.CTMRGError(4, f"no fixed point after {steps} steps (Delta {delta:.3e})")
        o = g.observables()
        ctx.g = g
        return tuple(torch.tensor(o[k], dtype=torch.float64) for k in ("f", "E", "M"))

    @staticmethod
    def backward(ctx, grad_f, grad_E, grad_M):
        g = ctx.g
        try:
            bar = [float(grad_f) if grad_f is not None else 0.0,
                   float(grad_E) if grad_E is not None else 0.0,
                   float(grad_M) if grad_M is not None else 0.0]
            kb, _ = g.backward(bar)
        finally:
            g.close()
        return torch.tensor(kb, dtype=torch.float64), None, None, None, None
