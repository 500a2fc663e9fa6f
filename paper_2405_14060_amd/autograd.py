"""torch.autograd.Function around the device-side sum-product of libtn.

forward : log Z of the network whose factor tables are ``values`` (FP32,
          linear domain, laid out as in tn_load_network), contracted on the
          plan's stream by the library's kernels.
backward: d logZ / dT_f for every factor entry, produced by the library's
          adjoint kernels in the same call (theorem thm:diff: the derivative
          of the contraction with respect to one tensor is the contraction of
          the network without it, with that tensor's labels as output; the
          reverse pass of eq. einback computes all of them in one sweep).
"""
from __future__ import annotations

import torch


class TNLogZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, values, evidence=None):
        values = values.detach().contiguous()
        if values.dtype != torch.float32 or not values.is_cuda:
            raise TypeError("values must be a float32 device tensor")
        logz = torch.empty(1, dtype=torch.float64, device=values.device)
        grad = torch.empty_like(values) if ctx.needs_input_grad[1] else None
        plan.log_z_dev(values.data_ptr(), logz.data_ptr(),
                       grad.data_ptr() if grad is not None else None, evidence)
        plan.sync()
        ctx.save_for_backward(grad if grad is not None else torch.empty(0))
        return logz

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return None, (g.to(torch.float32) * grad), None


def log_z(plan, values, evidence=None):
    return TNLogZ.apply(plan, values, evidence)
