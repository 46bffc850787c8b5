"""Differentiable forward simulation: traces(c) with a time-reversal backward.

``simulate(handle, c, src_sig, w)`` returns the sensor traces of the encoded
sources as a torch tensor that is differentiable with respect to the sound
speed ``c``.  The forward pass runs ``fwi_forward`` and keeps only the
pressure on the boundary layer dGamma (the tape); the backward pass runs
``fwi_backward``: the adjoint simulation driven by the incoming trace
gradient, interleaved with a time-reversed re-simulation of the forward field
from the tape (Sec. 3.1 and Alg. 1 of arXiv 2102.00755), so no wavefield
history is stored.  The gradient is restricted to Gamma (zero elsewhere), as
in the paper, where c outside Gamma is known.

The tape lives in the handle: a later forward or gradient call on the same
handle overwrites it, and a backward through an older graph then raises.
"""

from __future__ import annotations

import torch

from .fwi import Handle


class _Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c: torch.Tensor, handle: Handle, src_sig, w):
        traces = handle.forward(c, src_sig, w, save_tape=True)
        ctx.handle = handle
        ctx.token = handle.tape_token
        ctx.batched = c.dim() == 4
        ctx.save_for_backward(c)
        return traces if ctx.batched else traces[0]

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        (c,) = ctx.saved_tensors
        h: Handle = ctx.handle
        if h.tape_token != ctx.token:
            raise RuntimeError("the boundary tape of this forward was overwritten by a later call on the "
                               "same handle; run the forward again before backward")
        g = grad_traces if ctx.batched else grad_traces.unsqueeze(0)
        _, grad = h.backward(c, g.to(h.dtype).contiguous())
        return (grad if ctx.batched else grad[0]), None, None, None


def simulate(handle: Handle, c: torch.Tensor, src_sig, w) -> torch.Tensor:
    """Sensor traces [nt, n_rec] (or [B, nt, n_rec]) differentiable in c."""
    return _Traces.apply(c, handle, src_sig, w)
