"""torch.autograd binding of the ensemble expectation and its adjoint gradient.

Pre-trajectory sampling fixes each trajectory's Kraus operators before
execution (Sec. 3), so E(theta) = sum_a w_a <psi_a(theta)|O|psi_a(theta)>, with
the trajectory set's ensemble weights w_a, is a smooth function of the circuit
parameters.  Forward runs the library's adjoint gradient call (one forward
preparation and one reverse sweep of every trajectory) when the parameters
require a gradient, else its expectation mode, which sums the weighted value on
the device; backward scales the stored gradient.
"""

import torch

from . import ptsbe_adjoint_grad, ptsbe_run_batch


class PTSBEExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, plan, ts, observable):
        pv = params.detach().to("cpu", torch.float64).numpy()
        if params.requires_grad:
            E, G = ptsbe_adjoint_grad(plan, ts, pv, observable)
            ctx.save_for_backward(G.to(params.device, params.dtype))
            return E[0].to(params.device, params.dtype)
        r = ptsbe_run_batch(plan, ts, mode="expectation", params=pv, observable=observable)
        return r["E"][0].to(params.device, params.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        return grad_out * G, None, None, None


def expectation(params, plan, ts, observable):
    """E(params) of the trajectory set ts under the Z-string observable
    [(coef, qubits), ...]; differentiable in params (1-D tensor, n_params)."""
    return PTSBEExpectation.apply(params, plan, ts, observable)
