"""Pins of the oracle's serial rollout (the definition every Picard result must equal).

Section 2 defines the answer as a_t = pi(s_t, w_t), s_{t+1} = f(s_t, a_t, w_t); Section 3
gives the fulfillment transition and Section 3.1 the greedy policy.  Pins:
hand-worked cases (tests/golden), an independent pure-Python brute force on a dense
state, numpy's first-minimum argmin as the per-step tie rule, and the invariants of the
transition (inventory never negative, shipped + lost = demand, x_final = x0 - shipped).
"""
import os

import numpy as np
import pytest

from paper_2406_01939_amd.instances import Instance, random_tiny, make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "greedy_handworked.txt")


def _golden_cases():
    cases, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, *rest = line.split()
        if head == "case":
            cur = {"name": rest[0]}
            cases.append(cur)
        elif "dims" not in cur:
            cur["dims"] = [int(head)] + [int(v) for v in rest]
        else:
            cur[head] = np.array([int(v) for v in rest], dtype=np.int32)
    return cases


def _inst_from_case(c):
    N, K, R = c["dims"]
    T = c["sku"].size
    return Instance(N=N, K=K, R=R, traj_offsets=np.array([0, T], np.int64), sku=c["sku"],
                    region=c["region"], qty=c["qty"], x0=c["x0"].reshape(1, K, N),
                    cost=c["cost"].reshape(1, N, R), rng_seed=0)


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_handworked(oracle, case):
    inst = _inst_from_case(case)
    r = oracle.serial(inst)
    np.testing.assert_array_equal(r["actions"], case["actions"])
    np.testing.assert_array_equal(r["shipped"], case["shipped"])
    np.testing.assert_array_equal(r["final_inv"].ravel(), case["final"])


def brute_force_greedy(inst: Instance, b: int = 0):
    """Independent dense-state rollout: dictionary state, min over (cost, index) pairs."""
    lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
    state = {(k, w): int(inst.x0[b, k, w]) for k in range(inst.K) for w in range(inst.N)}
    acts, ships = [], []
    for t in range(lo, hi):
        k, r, q = int(inst.sku[t]), int(inst.region[t]), int(inst.qty[t])
        options = [(int(inst.cost[b, w, r]), w) for w in range(inst.N) if state[(k, w)] > 0]
        if not options:
            acts.append(-1)
            ships.append(0)
            continue
        _, w = min(options)
        s = min(q, state[(k, w)])
        state[(k, w)] -= s
        acts.append(w)
        ships.append(s)
    fin = np.array([[state[(k, w)] for w in range(inst.N)] for k in range(inst.K)])
    return np.array(acts), np.array(ships), fin


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_greedy(oracle, seed):
    inst = random_tiny(seed, N=1 + seed % 6, K=1 + seed % 4, R=1 + seed % 3, T=30,
                       qmax=1 + seed % 3, inv_max=4)
    r = oracle.serial(inst)
    a, s, f = brute_force_greedy(inst)
    np.testing.assert_array_equal(r["actions"], a)
    np.testing.assert_array_equal(r["shipped"], s)
    np.testing.assert_array_equal(r["final_inv"], f)


def test_numpy_argmin_tie_rule(oracle):
    """Per step the greedy choice is numpy.argmin of the cost column masked to +inf at
    empty warehouses (argmin returns the first minimum: the lowest index)."""
    inst = random_tiny(123, N=7, K=2, R=4, T=200, inv_max=6)
    r = oracle.serial(inst)
    x = inst.x0[0].astype(np.int64).copy()
    for t in range(inst.total_orders):
        k, reg = inst.sku[t], inst.region[t]
        col = np.where(x[k] > 0, inst.cost[0, :, reg].astype(np.float64), np.inf)
        want = -1 if np.isinf(col).all() else int(np.argmin(col))
        assert r["actions"][t] == want
        if want >= 0:
            x[k, want] -= min(inst.qty[t], x[k, want])


@pytest.mark.parametrize("qmax", [1, 3])
def test_invariants_at_scale(oracle, qmax):
    inst = make_instance("greedy_batch256_n50_k2e4", n_traj=1, T=200_000, qmax=qmax)
    r = oracle.serial(inst)
    x0, fin = inst.x0[0].astype(np.int64), r["final_inv"].astype(np.int64)
    assert (fin >= 0).all()
    shipped = r["shipped"].astype(np.int64)
    lost = inst.qty.astype(np.int64) - shipped
    assert (lost >= 0).all() and (shipped >= 0).all()
    assert shipped.sum() + lost.sum() == inst.qty.sum()
    per = np.zeros_like(x0)
    m = r["actions"] >= 0
    np.add.at(per, (inst.sku[m], r["actions"][m]), shipped[m])
    assert (per <= x0).all()
    np.testing.assert_array_equal(fin, x0 - per)
    # a lost sale happens only when no warehouse of the SKU has stock (checked by eval_at)
    ev = oracle.eval_at(inst, r["actions"])
    assert ((r["actions"] == -1) == (ev["n_feasible"] == 0)).all()


def test_eval_at_reproduces_serial(oracle):
    inst = random_tiny(9, N=5, K=3, R=3, T=60, qmax=2)
    r = oracle.serial(inst)
    ev = oracle.eval_at(inst, r["actions"])
    np.testing.assert_array_equal(ev["choice"], r["actions"])


def test_bad_input_rejected(oracle):
    inst = random_tiny(1)
    inst.qty = inst.qty.copy()
    inst.qty[0] = 0
    with pytest.raises(ValueError):
        oracle.serial(inst)
