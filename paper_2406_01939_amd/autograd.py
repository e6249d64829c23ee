"""torch.autograd.Function around the library's REINFORCE kernel.

PicardReinforce.apply(params, prob, actions, advantages) returns the surrogate
L(theta) = sum_t A_t log pi_theta(a_t | s_t) at fixed actions (the states are those the
actions induce); its backward calls pk_policy_grad, which recomputes the activations
instead of storing them.  `actions` typically come from pk_picard_simulate with the same
parameters (the Picard rollout of Section 2, used inside the policy-gradient loop of
Section 4.2) and `advantages` from pk_reinforce_advantages.
"""
from __future__ import annotations

import dataclasses

import torch

from . import api


class PicardReinforce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, prob: "api.DeviceProblem", actions: torch.Tensor,
                advantages: torch.Tensor):
        p2 = dataclasses.replace(prob, params=params.detach().contiguous())
        r = api.pk_policy_grad(p2, actions, advantages, want_logp=False, want_grad=False)
        ctx.prob = p2
        ctx.save_for_backward(actions, advantages)
        return torch.tensor(r["objective"], dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        actions, advantages = ctx.saved_tensors
        r = api.pk_policy_grad(ctx.prob, actions, advantages, want_logp=False, want_grad=True)
        return grad_out * r["grad"], None, None, None

