"""Pins of the oracle's policy-gradient pieces (Section 4.2): the REINFORCE advantages
of a rollout and the Adam step.

Advantages are pinned by facts other than their own formula: a brute-force double loop
for the reward-to-go on a tiny case; the difference of consecutive advantages is the
step's reward; advantages sum to zero over a trajectory; the total reward equals the
margin on shipped units aggregated per (warehouse, region) from the final inventory and
a count matrix; shifting the revenue shifts each reward-to-go by the shift times the
units shipped from then on; a trajectory of lost sales has zero advantages.

Adam is pinned against torch.optim.Adam (float64) on random gradient sequences, and by
two closed forms: the first step moves each coordinate by lr * g / (|g| + eps), and a
constant gradient moves it by that same amount at every step.
"""
import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import random_tiny

REV = 7


def _rollout(oracle, inst, b):
    return oracle.serial(inst, b, greedy=True)


@pytest.mark.parametrize("seed", range(4))
def test_reward_to_go_brute_force(oracle, seed):
    inst = random_tiny(300 + seed, N=5, K=3, R=4, T=40, qmax=3, inv_max=5, n_traj=2)
    for b in range(inst.n_traj):
        s = _rollout(oracle, inst, b)
        out = oracle.advantages(inst, s["actions"], s["shipped"], REV, b)
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        T = hi - lo
        r = []
        for t in range(T):
            a = int(s["actions"][t])
            if a < 0:
                r.append(0)
            else:
                r.append((REV - int(inst.cost[b][a][int(inst.region[lo + t])])) *
                         int(s["shipped"][t]))
        for t in range(T):
            assert int(out["rtg"][t]) == sum(r[t:])
        assert out["ret"] == sum(r)
        # A_t - A_{t+1} = r_t (to float32 rounding of each A), and sum_t A_t = 0
        A = out["advantages"].astype(np.float64)
        scale = max(1.0, float(np.abs(A).max()))
        np.testing.assert_allclose(A[:-1] - A[1:], np.asarray(r[:-1], np.float64),
                                   atol=4 * scale * 2**-24)
        assert abs(A.sum()) <= T * scale * 2**-23


@pytest.mark.parametrize("seed", range(3))
def test_total_reward_from_counts_and_final_inventory(oracle, seed):
    inst = random_tiny(400 + seed, N=6, K=4, R=5, T=60, qmax=2, inv_max=8, n_traj=1)
    s = _rollout(oracle, inst, 0)
    out = oracle.advantages(inst, s["actions"], s["shipped"], REV, 0)
    # units shipped in total, from the inventory that left the warehouses
    units = int(inst.x0[0].astype(np.int64).sum() - s["final_inv"].astype(np.int64).sum())
    # cost paid, from a (warehouse, region) count matrix of shipped units
    counts = np.zeros((inst.N, inst.R), np.int64)
    served = s["actions"] >= 0
    np.add.at(counts, (s["actions"][served], inst.region[served]), s["shipped"][served])
    paid = int((counts * inst.cost[0].astype(np.int64)).sum())
    assert out["ret"] == REV * units - paid


def test_revenue_shift(oracle):
    inst = random_tiny(500, N=4, K=2, R=3, T=50, qmax=3, inv_max=10)
    s = _rollout(oracle, inst, 0)
    a = oracle.advantages(inst, s["actions"], s["shipped"], REV, 0)
    d = oracle.advantages(inst, s["actions"], s["shipped"], REV + 5, 0)
    suffix_units = np.cumsum(s["shipped"][::-1].astype(np.int64))[::-1]
    np.testing.assert_array_equal(d["rtg"] - a["rtg"], 5 * suffix_units)


def test_lost_sales_and_single_order(oracle):
    inst = random_tiny(600, N=3, K=2, R=2, T=20, inv_max=0)
    s = _rollout(oracle, inst, 0)
    assert (s["actions"] == -1).all()
    out = oracle.advantages(inst, s["actions"], s["shipped"], REV, 0)
    assert (out["advantages"] == 0).all() and out["ret"] == 0
    one = random_tiny(601, N=3, K=1, R=2, T=1, inv_max=4)
    s1 = _rollout(oracle, one, 0)
    o1 = oracle.advantages(one, s1["actions"], s1["shipped"], REV, 0)
    assert o1["advantages"].tolist() == [0.0]


@pytest.mark.parametrize("ascend", [True, False])
def test_adam_matches_torch(oracle, ascend):
    rng = np.random.default_rng(7)
    n, steps, lr = 50, 6, 3e-3
    theta0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) * 10.0 ** rng.integers(-3, 2) for _ in range(steps)]
    p = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8, maximize=ascend)
    th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    for k, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = oracle.adam_step(th, g, m, v, k, lr, ascend=ascend)
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_closed_forms(oracle):
    g = np.array([2.0, -0.5, 1e-3, 0.0])
    lr, eps = 0.01, 1e-8
    th0 = np.array([1.0, 2.0, 3.0, 4.0])
    th1, m, v = oracle.adam_step(th0, g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    np.testing.assert_allclose(th1 - th0, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    th = th0
    m = v = np.zeros(4)
    for k in range(1, 6):
        th, m, v = oracle.adam_step(th, g, m, v, k, lr, eps=eps, ascend=False)
    np.testing.assert_allclose(th0 - th, 5 * lr * g / (np.abs(g) + eps), rtol=1e-10, atol=1e-15)
