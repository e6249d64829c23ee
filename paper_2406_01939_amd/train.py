"""Policy-gradient training around the Picard rollout (Section 4.2).

Each iteration
  1. rolls out the current policy on the batch's fixed sample paths (orders and Gumbel
     noise): Algorithm 1 warm-started from the previous iterate's actions (Section 5
     seeds the cache with the earlier policy's actions on the same sample path), or cold
     (lost sale everywhere), or the serial rollout as the baseline;
  2. forms REINFORCE advantages from that rollout (pk_reinforce_advantages);
  3. computes the gradient of sum_t A_t log pi(a_t | s_t) at the rolled-out actions
     (pk_policy_grad);
  4. takes one Adam step that ascends it (pk_adam_step, learning rate 3e-3 as in
     Section 4.2).
Every step runs in the library's kernels; this module only sequences the calls.  Any
cache gives the serial rollout at convergence (Proposition 2.1), so the three rollout
modes produce the same training run; they differ in passes and time.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import torch

from . import api

ROLLOUTS = ("picard", "serial")


@dataclasses.dataclass
class IterStats:
    it: int
    passes_max: int         # passes of the rollout (0 for the serial rollout)
    passes_mean: float
    rollout_ms: float       # wall time of the rollout call
    grad_ms: float          # advantages + gradient + Adam step
    objective: float        # sum_t A_t log pi(a_t | s_t) at this iterate
    mean_return: float      # mean over trajectories of the total margin reward


class PolicyGradient:
    """REINFORCE with Adam on a DeviceProblem whose `params` is the MLP pack (updated in
    place).  `warm_start` seeds each Picard rollout with the previous iterate's actions."""

    def __init__(self, prob: "api.DeviceProblem", lr: float = 3e-3, revenue: int = 200,
                 rollout: str = "picard", warm_start: bool = True, block_len: int = 0,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        if prob.params is None:
            raise ValueError("the problem carries no MLP parameters")
        if rollout not in ROLLOUTS:
            raise ValueError(f"rollout must be one of {ROLLOUTS}")
        self.prob = prob
        self.lr, self.revenue, self.rollout = lr, int(revenue), rollout
        self.warm_start, self.block_len = warm_start, block_len
        self.betas, self.eps = (beta1, beta2), eps
        self.m = torch.zeros_like(prob.params)
        self.v = torch.zeros_like(prob.params)
        self.t = 0
        self.prev_actions: Optional[torch.Tensor] = None
        self.out: Optional[dict] = None

    def _rollout(self) -> dict:
        if self.rollout == "serial":
            r = api.pk_serial_simulate(self.prob, "mlp", want_final=False)
            r["passes"] = None
            return r
        init = self.prev_actions if self.warm_start else None
        return api.pk_picard_simulate(self.prob, "mlp", block_len=self.block_len,
                                      init_cache=init, want_final=False)

    def step(self) -> IterStats:
        sync = torch.cuda.synchronize
        sync()
        t0 = time.perf_counter()
        out = self._rollout()
        sync()
        t1 = time.perf_counter()
        adv = api.pk_reinforce_advantages(self.prob, out["actions"], out["shipped"], self.revenue)
        g = api.pk_policy_grad(self.prob, out["actions"], adv["advantages"], want_logp=False)
        self.t += 1
        api.pk_adam_step(self.prob.params, g["grad"], self.m, self.v, self.t, self.lr,
                         self.betas[0], self.betas[1], self.eps, ascend=True)
        sync()
        t2 = time.perf_counter()
        self.prev_actions = out["actions"]
        self.out = out
        passes = out["passes"]
        return IterStats(
            it=self.t,
            passes_max=int(passes.max()) if passes is not None else 0,
            passes_mean=float(passes.mean()) if passes is not None else 0.0,
            rollout_ms=1e3 * (t1 - t0), grad_ms=1e3 * (t2 - t1),
            objective=float(g["objective"]),
            mean_return=float(adv["returns"].double().mean().item()))

    def run(self, iters: int, callback: Optional[Callable[[IterStats], None]] = None
            ) -> List[IterStats]:
        hist = []
        for _ in range(iters):
            s = self.step()
            hist.append(s)
            if callback:
                callback(s)
        return hist
