"""torch.autograd wrapper of the adjoint mode of the C ABI.

``final_observable(coef, problem, psi0, t0, dt, n_steps, m)`` returns the sum
of the final expectation values selected by ``loss_kind`` (1 <x>, 2 <y>,
4 <p_x>, 8 <p_y>) as a 0-d tensor that is differentiable with respect to the
Fourier laser coefficients ``coef`` (pulse kind DL_PULSE_FOURIER_SIN2).
The forward call runs the library's whole adjoint (forward pass with
checkpoints, backward pass, gradient); ``backward`` only scales the stored
gradient, so an optimisation loop pays one adjoint per loss evaluation.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import Propagator

__all__ = ["FinalObservable", "final_observable"]


class FinalObservable(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coef, problem, psi0, t0, dt, n_steps, m, ckpt_every, loss_kind):
        c = coef.detach().to("cpu", torch.float64).numpy().copy()
        prob = dict(problem, pulse_kind=2, coef=c)
        prop = Propagator(prob, m, "fp64")
        try:
            loss, grad = prop.adjoint(psi0, t0, dt, n_steps, ckpt_every, loss_kind)
        finally:
            prop.close()
        ctx.save_for_backward(torch.as_tensor(np.asarray(grad), dtype=coef.dtype, device=coef.device))
        return coef.new_tensor(loss)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return (gout * g,) + (None,) * 8


def final_observable(coef, problem: dict, psi0, t0: float, dt: float, n_steps: int, m: int,
                     ckpt_every: int = 50, loss_kind: int = 9):
    """Differentiable final observable; see the module docstring."""
    return FinalObservable.apply(coef, problem, psi0, t0, dt, n_steps, m, ckpt_every, loss_kind)
