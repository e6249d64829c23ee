"""torch.autograd.Function around the library's REINFORCE kernel.

PicardReinforce.apply(params, prob, actions, advantages) returns the surrogate
L(theta) = sum_t A_t log pi_theta(a_t | s_t) at fixed actions (the states are those the
actions induce); its backward calls pk_policy_grad, which recomputes the activations
instead of storing them.  `actions` typically come from pk_picard_simulate with the same
parameters (the Picard rollout of Section 2, used inside the policy-gradient loop of
Section 4.2).
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


def reward_to_go_advantages(prob: "api.DeviceProblem", actions: torch.Tensor,
                            shipped: torch.Tensor, lost_penalty: float = 200.0) -> torch.Tensor:
    """A_t = (reward-to-go of step t) - (its mean over the trajectory), with reward
    r_t = -cost[a_t][region_t] * shipped_t - lost_penalty * (q_t - shipped_t).  A helper
    for examples and tests: the advantages are an input of the gradient."""
    offs = torch.as_tensor(prob.traj_offsets, device=actions.device)
    traj = torch.repeat_interleave(torch.arange(prob.n_traj, device=actions.device),
                                   offs[1:] - offs[:-1])
    a = actions.long().clamp(min=0)
    c = prob.cost[traj, a, prob.region.long()].double()
    sh = shipped.double()
    rew = torch.where(actions >= 0, -c * sh, torch.zeros_like(sh)) - lost_penalty * (
        prob.qty.double() - sh)
    out = torch.empty_like(rew)
    for b in range(prob.n_traj):
        lo, hi = int(prob.traj_offsets[b]), int(prob.traj_offsets[b + 1])
        if hi == lo:
            continue
        rtg = torch.flip(torch.cumsum(torch.flip(rew[lo:hi], [0]), 0), [0])
        out[lo:hi] = rtg - rtg.mean()
    return out.float()
