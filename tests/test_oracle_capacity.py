"""Pins of the oracle with node capacity (Section 3: state (x_t, c_t), an order may go to
node j only if c_{t,j} > 0 and x_{t,i,j} > 0, and shipping lowers both by one).

* Hand-worked tiny cases.
* Brute force: a dense pure-Python rollout, and numpy's argmin (first minimum) over the
  costs masked to +inf, per step.
* Reductions to the pinned no-capacity oracle: capacities that never bind; one SKU whose
  stock equals the capacities (the two counters move together); unbounded stock, where
  capacity plays the role of one shared SKU's stock.
* Invariants: capacities and stock never negative; what left a node equals its capacity
  drop.
* Algorithm 1: any fixed point equals the serial rollout; Proposition 2.1 (k* <= T for
  any partition and any initial cache); the time-block replay equals the brute-force
  algorithm pass by pass.
* Section 3.1, special case (stock never binds, greedy policy): Lemma 3.2's invariant
  (every cached action is the serial one or a node already out of capacity at that
  time) and the bound k* <= |Q_T| + 1, for any partition; Theorem 3.1 (Assumptions 1-3
  hold for greedy) for the product partition with binding stock.
"""
import numpy as np
import pytest

from paper_2406_01939_amd.instances import capacity, random_tiny


def _kstar(caches, serial_actions):
    if np.all(serial_actions == -1):
        return 0
    for k, c in enumerate(caches, start=1):
        if np.array_equal(c, serial_actions):
            return k
    raise AssertionError("never reached the serial trajectory")


def _tiny(seed, **kw):
    rng = np.random.default_rng(10_000 + seed)
    inst = random_tiny(seed, qmax=1, **kw)
    T = int(inst.traj_offsets[-1])
    cap0 = rng.integers(0, max(2, T // inst.N + 2), inst.N).astype(np.int32)
    return inst, cap0


def _brute_serial(inst, cap0):
    x = {(k, w): int(inst.x0[0][k, w]) for k in range(inst.K) for w in range(inst.N)}
    c = [int(v) for v in cap0]
    out = []
    for t in range(int(inst.traj_offsets[-1])):
        k, r = int(inst.sku[t]), int(inst.region[t])
        best = None
        for w in range(inst.N):
            if x[(k, w)] > 0 and c[w] > 0:
                if best is None or inst.cost[0][w, r] < inst.cost[0][best, r]:
                    best = w
        if best is None:
            out.append(-1)
        else:
            out.append(best)
            x[(k, best)] -= 1
            c[best] -= 1
    return np.array(out, np.int32)


def test_hand_worked(oracle):
    from paper_2406_01939_amd.instances import Instance
    # two nodes, cost 1 and 2; node 0 can ship one unit, node 1 five; stock 5 each
    inst = Instance(N=2, K=1, R=1, traj_offsets=np.array([0, 3], np.int64),
                    sku=np.zeros(3, np.int32), region=np.zeros(3, np.int32),
                    qty=np.ones(3, np.int32), x0=np.array([[[5, 5]]], np.int32),
                    cost=np.array([[[1], [2]]], np.int32), rng_seed=0, params=None,
                    name="hand")
    r = oracle.serial_cap(inst, np.array([1, 5], np.int32))
    assert r["actions"].tolist() == [0, 1, 1]
    assert r["final_cap"].tolist() == [0, 3]
    assert r["final_inv"].tolist() == [[4, 3]]
    # no capacity anywhere: every order is lost
    r = oracle.serial_cap(inst, np.array([0, 0], np.int32))
    assert r["actions"].tolist() == [-1, -1, -1]
    # stock binds before capacity at node 0
    inst.x0[0][0, 0] = 1
    r = oracle.serial_cap(inst, np.array([9, 9], np.int32))
    assert r["actions"].tolist() == [0, 1, 1]


@pytest.mark.parametrize("seed", range(40))
def test_serial_brute_force(oracle, seed):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 4, R=1 + seed % 3, T=20,
                       inv_max=4)
    r = oracle.serial_cap(inst, cap0)
    assert np.array_equal(r["actions"], _brute_serial(inst, cap0))
    # library special case: numpy's argmin returns the first minimum (lowest index)
    x = inst.x0[0].astype(np.int64).copy()
    c = cap0.astype(np.int64).copy()
    for t in range(int(inst.traj_offsets[-1])):
        k, reg = inst.sku[t], inst.region[t]
        masked = np.where((x[k] > 0) & (c > 0), inst.cost[0][:, reg].astype(np.float64), np.inf)
        a = -1 if np.isinf(masked.min()) else int(np.argmin(masked))
        assert r["actions"][t] == a
        if a >= 0:
            x[k, a] -= 1
            c[a] -= 1
    # invariants
    assert (r["final_cap"] >= 0).all() and (r["final_inv"] >= 0).all()
    sent = np.bincount(r["actions"][r["actions"] >= 0], minlength=inst.N)
    assert np.array_equal(cap0 - r["final_cap"], sent)
    per = np.zeros((inst.K, inst.N), np.int64)
    np.add.at(per, (inst.sku[r["actions"] >= 0], r["actions"][r["actions"] >= 0]), 1)
    assert np.array_equal(inst.x0[0] - r["final_inv"], per)


@pytest.mark.parametrize("seed", range(20))
def test_reductions_to_no_capacity(oracle, seed):
    inst, _ = _tiny(seed, N=2 + seed % 5, K=1 + seed % 4, R=1 + seed % 3, T=20, inv_max=4)
    T = int(inst.traj_offsets[-1])
    # capacities that never bind
    big = np.full(inst.N, T, np.int32)
    assert np.array_equal(oracle.serial_cap(inst, big)["actions"],
                          oracle.serial(inst, greedy=True)["actions"])
    # one SKU with stock equal to the capacities
    one = _one_sku(inst)
    assert np.array_equal(oracle.serial_cap(one, one.x0[0][0].copy())["actions"],
                          oracle.serial(one, greedy=True)["actions"])
    # unbounded stock: capacity acts as the stock of one shared SKU
    rng = np.random.default_rng(seed)
    cap0 = rng.integers(0, 4, inst.N).astype(np.int32)
    free = _with_x0(inst, np.full((inst.K, inst.N), T, np.int32))
    shared = _one_sku(inst)
    shared.x0[0][0] = cap0
    assert np.array_equal(oracle.serial_cap(free, cap0)["actions"],
                          oracle.serial(shared, greedy=True)["actions"])


def _with_x0(inst, x0):
    import dataclasses
    return dataclasses.replace(inst, x0=x0[None].astype(np.int32).copy())


def _one_sku(inst):
    import dataclasses
    return dataclasses.replace(inst, K=1, sku=np.zeros_like(inst.sku),
                               x0=inst.x0[:, :1, :].copy())


@pytest.mark.parametrize("seed", range(30))
def test_alg1_fixed_point_and_prop21(oracle, seed):
    inst, cap0 = _tiny(seed, N=2 + seed % 4, K=1 + seed % 3, R=1 + seed % 3, T=12,
                       inv_max=3)
    T = int(inst.traj_offsets[-1])
    rng = np.random.default_rng(seed)
    ser = oracle.serial_cap(inst, cap0)["actions"]
    for kind in range(3):
        if kind == 0:
            worker, P = np.arange(T), T
        elif kind == 1:
            P = 1 + seed % 4
            worker = rng.integers(0, P, T)
        else:
            worker, P = inst.sku.astype(np.int64), inst.K
        init = None if seed % 2 == 0 else rng.integers(-1, inst.N, T).astype(np.int32)
        r = oracle.alg1_cap(inst, cap0, worker, P, init_cache=init)
        assert r["converged"]
        assert np.array_equal(r["actions"], ser)
        assert r["passes"] <= T + 1                       # Proposition 2.1
        # the returned pass is the first repeat: k* + 1 exactly
        a0 = np.full(T, -1, np.int32) if init is None else init
        seq = [a0] + list(r["caches"])
        kstar = next(k for k, c in enumerate(seq) if np.array_equal(c, ser))
        assert r["passes"] == kstar + 1


@pytest.mark.parametrize("seed", range(40))
def test_timeblocks_equal_alg1(oracle, seed):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 4, R=1 + seed % 3, T=16,
                       inv_max=3)
    T = int(inst.traj_offsets[-1])
    rng = np.random.default_rng(seed)
    for B in (1, 2, 3, 5, T):
        init = None if (seed + B) % 2 == 0 else rng.integers(-1, inst.N, T).astype(np.int32)
        lit = oracle.alg1_cap(inst, cap0, oracle.time_block_workers(T, B), (T + B - 1) // B,
                              init_cache=init)
        tb = oracle.picard_timeblocks_cap(inst, cap0, B, init_cache=init, record=True)
        assert lit["passes"] == tb["passes"]
        assert np.array_equal(lit["caches"], tb["caches"])
        prev = np.full(T, -1, np.int32) if init is None else init
        for k, c in enumerate(tb["caches"]):
            assert tb["changed"][k] == int((c != prev).sum())
            prev = c
        if B >= T:
            assert tb["passes"] <= 2  # one process: exact in one pass


def _tau(cap0, actions):
    """tau_j = first t (0-based: the state before order t) with c_{t,j} = 0, T + 1 if no
    order meets node j without capacity; Q_T = {j : tau_j <= T - 1}."""
    T = len(actions)
    tau = np.full(len(cap0), T + 1, np.int64)
    c = cap0.astype(np.int64).copy()
    for j in range(len(cap0)):
        if c[j] == 0:
            tau[j] = 0
    for t, a in enumerate(actions):
        if a >= 0:
            c[a] -= 1
            if c[a] == 0:
                tau[a] = t + 1
    return tau


@pytest.mark.parametrize("seed", range(40))
def test_special_case_bound_any_partition(oracle, seed):
    """Stock never binds (x_1 = T), greedy: Lemma 3.2 and k* <= |Q_T| + 1."""
    rng = np.random.default_rng(seed)
    N, K, T = 2 + seed % 5, 1 + seed % 3, 18
    inst = random_tiny(seed, N=N, K=K, R=1 + seed % 4, T=T, qmax=1)
    inst = _with_x0(inst, np.full((K, N), T, np.int32))
    cap0 = rng.integers(0, 6, N).astype(np.int32)
    ser = oracle.serial_cap(inst, cap0)
    tau = _tau(cap0, ser["actions"])
    q_T = int((tau <= T - 1).sum())
    assert q_T <= int((ser["final_cap"] == 0).sum())
    for kind in range(3):
        if kind == 0:
            P = 1 + seed % 5
            worker = rng.integers(0, P, T)
        elif kind == 1:
            B = 1 + seed % 4
            worker, P = np.arange(T) // B, (T + B - 1) // B
        else:
            worker, P = np.arange(T), T
        r = oracle.alg1_cap(inst, cap0, worker, P)
        kstar = _kstar(r["caches"], ser["actions"])
        assert kstar <= q_T + 1
        for c in r["caches"]:
            for t in range(T):
                a = c[t]
                assert a == ser["actions"][t] or (a >= 0 and tau[a] <= t)


@pytest.mark.parametrize("seed", range(40))
def test_theorem31_product_partition(oracle, seed):
    """Product partition, stock and capacity both binding: k* <= |Q_T| + 1."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=2 + seed % 3, R=1 + seed % 3, T=18,
                       inv_max=4)
    ser = oracle.serial_cap(inst, cap0)
    q_T = int((_tau(cap0, ser["actions"]) <= len(ser["actions"]) - 1).sum())
    r = oracle.alg1_cap(inst, cap0, inst.sku.astype(np.int64), inst.K)
    assert _kstar(r["caches"], ser["actions"]) <= q_T + 1


def test_capacity_generator():
    c = capacity(10, 10_000)
    assert c.dtype == np.int32 and c.tolist() == [800] * 10


def test_rejects_multi_unit(oracle):
    inst = random_tiny(3, N=3, K=2, R=2, T=10, qmax=3)
    inst.qty[:] = 2
    with pytest.raises(ValueError):
        oracle.serial_cap(inst, np.ones(3, np.int32))


# ---------------------------------------------------------------- capacity-dependent policy
def _brute_gamma(inst, cap0, gamma):
    """The appendix's capacity-dependent policy from its description, in exact rationals:
    score_w = rank_r(w) + gamma (N-1) (1 - c_w / M), M the largest remaining capacity,
    least score among nodes with stock and capacity, lowest index on ties."""
    from fractions import Fraction
    g = Fraction(*gamma)
    N = inst.N
    x = inst.x0[0].astype(np.int64).copy()
    c = [int(v) for v in cap0]
    out = []
    for t in range(int(inst.traj_offsets[-1])):
        k, r = int(inst.sku[t]), int(inst.region[t])
        order = sorted(range(N), key=lambda w: (int(inst.cost[0][w, r]), w))
        rank = {w: i for i, w in enumerate(order)}
        M = max(c)
        best, bs = -1, None
        for w in range(N):
            if x[k, w] > 0 and c[w] > 0:
                sc = rank[w] + g * (N - 1) * (1 - Fraction(c[w], M))
                if bs is None or sc < bs:
                    best, bs = w, sc
        out.append(best)
        if best >= 0:
            x[k, best] -= 1
            c[best] -= 1
    return np.array(out, np.int32)


@pytest.mark.parametrize("gamma", [(1, 2), (1, 1), (3, 1), (7, 3)])
@pytest.mark.parametrize("seed", range(12))
def test_gamma_policy_brute_force(oracle, seed, gamma):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=24, inv_max=4)
    r = oracle.serial_cap(inst, cap0, gamma=gamma)
    assert np.array_equal(r["actions"], _brute_gamma(inst, cap0, gamma))
    # gamma = 0 (any denominator) is the greedy policy
    assert np.array_equal(oracle.serial_cap(inst, cap0, gamma=(0, 7))["actions"],
                          oracle.serial_cap(inst, cap0)["actions"])


@pytest.mark.parametrize("seed", range(12))
def test_gamma_large_picks_most_capacity(oracle, seed):
    """gamma -> infinity: the feasible node with the most capacity left (the appendix's
    limiting case), ties to the better-ranked node."""
    inst, cap0 = _tiny(seed, N=3 + seed % 4, K=2, R=2, T=20, inv_max=4)
    r = oracle.serial_cap(inst, cap0, gamma=(1000, 1))
    x = inst.x0[0].astype(np.int64).copy()
    c = cap0.astype(np.int64).copy()
    for t in range(int(inst.traj_offsets[-1])):
        k, reg = inst.sku[t], inst.region[t]
        feas = [w for w in range(inst.N) if x[k, w] > 0 and c[w] > 0]
        if not feas:
            assert r["actions"][t] == -1
            continue
        a = min(feas, key=lambda w: (-c[w], int(inst.cost[0][w, reg]), w))
        # the rank term decides only among equal capacities when gamma (N-1) / M exceeds N
        if 1000 * (inst.N - 1) > inst.N * max(c.max(), 1) * 1:
            assert r["actions"][t] == a
        a = r["actions"][t]
        x[k, a] -= 1
        c[a] -= 1


@pytest.mark.parametrize("seed", range(20))
def test_gamma_picard(oracle, seed):
    """Proposition 2.1 for the capacity-dependent policy (the bound of Theorem 3.1 does not
    apply: the policy breaks Assumption 3), and the time-block replay against the brute-force
    Algorithm 1 pass by pass."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=16, inv_max=3)
    T = int(inst.traj_offsets[-1])
    gamma = [(1, 2), (1, 1), (2, 1)][seed % 3]
    ser = oracle.serial_cap(inst, cap0, gamma=gamma)["actions"]
    rng = np.random.default_rng(seed)
    worker = rng.integers(0, 1 + seed % 4, T)
    r = oracle.alg1_cap(inst, cap0, worker, 1 + seed % 4, gamma=gamma)
    assert r["converged"] and np.array_equal(r["actions"], ser) and r["passes"] <= T + 1
    for B in (1, 3, T):
        lit = oracle.alg1_cap(inst, cap0, oracle.time_block_workers(T, B), (T + B - 1) // B,
                              gamma=gamma)
        tb = oracle.picard_timeblocks_cap(inst, cap0, B, record=True, gamma=gamma)
        assert lit["passes"] == tb["passes"]
        assert np.array_equal(lit["caches"], tb["caches"])


@pytest.mark.parametrize("seed", range(40))
def test_gamma_scale_is_the_largest_capacity_of_any_node(oracle, seed):
    """M is the largest remaining capacity over every node, with or without stock of the
    order's SKU (scarce stock, so that the node with the most capacity often has none)."""
    rng = np.random.default_rng(30_000 + seed)
    inst = random_tiny(seed, N=4 + seed % 4, K=3, R=2, T=30, qmax=1, inv_max=1)
    cap0 = rng.integers(1, 12, inst.N).astype(np.int32)
    gamma = [(1, 1), (2, 1), (1, 2), (5, 2)][seed % 4]
    r = oracle.serial_cap(inst, cap0, gamma=gamma)
    assert np.array_equal(r["actions"], _brute_gamma(inst, cap0, gamma))


# ---------------------------------------------------------------- near-exhaustion reading
def _brute_gamma_low(inst, cap0, gamma, low):
    """The second reading of the appendix's capacity-dependent policy, in exact rationals
    from its description: only nodes with less than `low` capacity left pay a shadow price,
    rising linearly to gamma (N-1) as they empty; score_w = rank_r(w) + gamma (N-1)
    max(0, low - c_w) / low, least among nodes with stock and capacity, lowest index on
    ties."""
    from fractions import Fraction
    g = Fraction(*gamma)
    N = inst.N
    x = inst.x0[0].astype(np.int64).copy()
    c = [int(v) for v in cap0]
    out = []
    for t in range(int(inst.traj_offsets[-1])):
        k, r = int(inst.sku[t]), int(inst.region[t])
        order = sorted(range(N), key=lambda w: (int(inst.cost[0][w, r]), w))
        rank = {w: i for i, w in enumerate(order)}
        best, bs = -1, None
        for w in range(N):
            if x[k, w] > 0 and c[w] > 0:
                sc = rank[w] + g * (N - 1) * Fraction(max(0, low - c[w]), low)
                if bs is None or sc < bs:
                    best, bs = w, sc
        out.append(best)
        if best >= 0:
            x[k, best] -= 1
            c[best] -= 1
    return np.array(out, np.int32)


@pytest.mark.parametrize("gamma", [(1, 2), (1, 1), (3, 1), (7, 3)])
@pytest.mark.parametrize("seed", range(12))
def test_gamma_low_brute_force(oracle, seed, gamma):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=24, inv_max=4)
    low = 1 + seed % 4
    r = oracle.serial_cap(inst, cap0, gamma=gamma + (low,))
    assert np.array_equal(r["actions"], _brute_gamma_low(inst, cap0, gamma, low))


@pytest.mark.parametrize("seed", range(12))
def test_gamma_low_without_scarce_nodes_is_greedy(oracle, seed):
    """While no node falls below the threshold no price is charged: with every capacity
    above `low` plus the horizon the policy is the greedy one, whatever gamma."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=24, inv_max=4)
    T = int(inst.traj_offsets[-1])
    big = np.full(inst.N, 3 + T, np.int32)
    g = oracle.serial_cap(inst, big)["actions"]
    for gamma in ((1, 1), (1000, 1)):
        assert np.array_equal(oracle.serial_cap(inst, big, gamma=gamma + (3,))["actions"], g)


def test_gamma_low_hand_worked(oracle):
    """Two nodes, one region, node 0 cheaper; low = 4, gamma = 1 (N - 1 = 1): node 0's
    price is max(0, 4 - c0) / 4.  With c = (2, 9) node 0 scores 0 + 2/4 and node 1 scores
    1: node 0 ships.  After that c0 = 1, score 3/4 < 1: node 0 again.  Then c0 = 0: node 1.
    With gamma = 3: node 0 at c0 = 2 scores 6/4 > 1, so node 1 ships from the first order."""
    inst = random_tiny(1, N=2, K=1, R=1, T=3, qmax=1, inv_max=5)
    inst.x0[:] = 5
    inst.cost[:] = np.array([[1], [2]], np.int32)
    cap0 = np.array([2, 9], np.int32)
    assert oracle.serial_cap(inst, cap0, gamma=(1, 1, 4))["actions"].tolist() == [0, 0, 1]
    assert oracle.serial_cap(inst, cap0, gamma=(3, 1, 4))["actions"].tolist() == [1, 1, 1]
    assert oracle.serial_cap(inst, cap0, gamma=(0, 1, 4))["actions"].tolist() == [0, 0, 1]


@pytest.mark.parametrize("seed", range(20))
def test_gamma_low_picard(oracle, seed):
    """Proposition 2.1 for the near-exhaustion reading, and the time-block replay against
    the brute-force Algorithm 1 pass by pass."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=16, inv_max=3)
    T = int(inst.traj_offsets[-1])
    gamma = [(1, 2, 2), (1, 1, 3), (2, 1, 1)][seed % 3]
    ser = oracle.serial_cap(inst, cap0, gamma=gamma)["actions"]
    rng = np.random.default_rng(seed)
    worker = rng.integers(0, 1 + seed % 4, T)
    r = oracle.alg1_cap(inst, cap0, worker, 1 + seed % 4, gamma=gamma)
    assert r["converged"] and np.array_equal(r["actions"], ser) and r["passes"] <= T + 1
    for B in (1, 3, T):
        lit = oracle.alg1_cap(inst, cap0, oracle.time_block_workers(T, B), (T + B - 1) // B,
                              gamma=gamma)
        tb = oracle.picard_timeblocks_cap(inst, cap0, B, record=True, gamma=gamma)
        assert lit["passes"] == tb["passes"]
        assert np.array_equal(lit["caches"], tb["caches"])


def test_gamma_low_rejects_negative_threshold(oracle):
    inst, cap0 = _tiny(0, N=3, K=2, R=2, T=10, inv_max=3)
    with pytest.raises(ValueError):
        oracle.serial_cap(inst, cap0, gamma=(1, 1, -1))


# ---------------------------------------------------------------- bid-price policy
def _bids(inst, seed, spread=4):
    rng = np.random.default_rng(50_000 + seed)
    bi = rng.integers(-spread, spread + 1, (inst.K, inst.N)).astype(np.int32)
    bc = rng.integers(0, spread + 1, inst.N).astype(np.int32)
    return bi, bc


def _brute_bids(inst, cap0, bi, bc):
    """The dual policy of Section 4.2 with fixed prices, from its definition: the node
    maximising r_j - mu_inv(i, j) - mu_cap(j), with reward r_j = -cost[j][region], among the
    nodes with stock and capacity; lowest index on ties."""
    N = inst.N
    x = inst.x0[0].astype(np.int64).copy()
    c = [int(v) for v in cap0]
    out = []
    for t in range(int(inst.traj_offsets[-1])):
        k, r = int(inst.sku[t]), int(inst.region[t])
        best, bv = -1, None
        for w in range(N):
            if x[k, w] > 0 and c[w] > 0:
                v = -int(inst.cost[0][w, r]) - int(bi[k, w]) - int(bc[w])
                if bv is None or v > bv:
                    best, bv = w, v
        out.append(best)
        if best >= 0:
            x[k, best] -= 1
            c[best] -= 1
    return np.array(out, np.int32)


@pytest.mark.parametrize("seed", range(30))
def test_bid_price_brute_force(oracle, seed):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=24, inv_max=4)
    bi, bc = _bids(inst, seed)
    r = oracle.serial_cap(inst, cap0, bids=(bi, bc))
    assert np.array_equal(r["actions"], _brute_bids(inst, cap0, bi, bc))
    # one of the two price vectors alone
    r1 = oracle.serial_cap(inst, cap0, bids=(None, bc))
    assert np.array_equal(r1["actions"], _brute_bids(inst, cap0, 0 * bi, bc))
    # zero prices are the greedy policy
    z = oracle.serial_cap(inst, cap0, bids=(0 * bi, 0 * bc))
    assert np.array_equal(z["actions"], oracle.serial_cap(inst, cap0)["actions"])


def test_bid_price_hand_worked(oracle):
    """Two nodes, costs 1 and 3 in the one region; a capacity price of 5 on node 0 moves
    orders to node 1 (3 < 1 + 5) until node 1 runs out of capacity (2 units), then node 0."""
    inst = random_tiny(2, N=2, K=1, R=1, T=4, qmax=1, inv_max=5)
    inst.x0[:] = 5
    inst.cost[:] = np.array([[1], [3]], np.int32)
    cap0 = np.array([9, 2], np.int32)
    bc = np.array([5, 0], np.int32)
    assert oracle.serial_cap(inst, cap0, bids=(None, bc))["actions"].tolist() == [1, 1, 0, 0]
    # a stock price of SKU 0 at node 1: 2 leaves node 1 ahead (3 + 2 = 5 < 1 + 5 = 6), 3
    # ties it with node 0 (6 = 6: the lower index wins), 4 puts it behind
    bi = np.array([[0, 2]], np.int32)
    assert oracle.serial_cap(inst, cap0, bids=(bi, bc))["actions"].tolist() == [1, 1, 0, 0]
    for p in (3, 4):
        bi = np.array([[0, p]], np.int32)
        assert oracle.serial_cap(inst, cap0, bids=(bi, bc))["actions"].tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("seed", range(20))
def test_bid_price_theorem_bound(oracle, seed):
    """Fixed bid prices keep Assumptions 1-3 (the paper names bid-price policies as the
    class that meets them), so Theorem 3.1's bound holds: with the product partition,
    k* <= |Q_T| + 1, Q_T the nodes that run out of capacity in the serial rollout."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=2 + seed % 3, R=1 + seed % 3, T=18, inv_max=4)
    bi, bc = _bids(inst, seed)
    ser = oracle.serial_cap(inst, cap0, bids=(bi, bc))
    q_T = int((_tau(cap0, ser["actions"]) <= len(ser["actions"]) - 1).sum())
    r = oracle.alg1_cap(inst, cap0, inst.sku.astype(np.int64), inst.K, bids=(bi, bc))
    assert r["converged"] and np.array_equal(r["actions"], ser["actions"])
    assert _kstar(r["caches"], ser["actions"]) <= q_T + 1


@pytest.mark.parametrize("seed", range(20))
def test_bid_price_picard(oracle, seed):
    """Proposition 2.1 for the bid-price policy, and the time-block replay against the
    brute-force Algorithm 1 pass by pass."""
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=16, inv_max=3)
    T = int(inst.traj_offsets[-1])
    bids = _bids(inst, seed)
    ser = oracle.serial_cap(inst, cap0, bids=bids)["actions"]
    rng = np.random.default_rng(seed)
    worker = rng.integers(0, 1 + seed % 4, T)
    r = oracle.alg1_cap(inst, cap0, worker, 1 + seed % 4, bids=bids)
    assert r["converged"] and np.array_equal(r["actions"], ser) and r["passes"] <= T + 1
    for B in (1, 3, T):
        lit = oracle.alg1_cap(inst, cap0, oracle.time_block_workers(T, B), (T + B - 1) // B,
                              bids=bids)
        tb = oracle.picard_timeblocks_cap(inst, cap0, B, record=True, bids=bids)
        assert lit["passes"] == tb["passes"]
        assert np.array_equal(lit["caches"], tb["caches"])


def test_bid_price_rejects_mixed_policy_and_bad_shapes(oracle):
    inst, cap0 = _tiny(0, N=3, K=2, R=2, T=10, inv_max=3)
    bi, bc = _bids(inst, 0)
    with pytest.raises(ValueError):
        oracle.serial_cap(inst, cap0, gamma=(1, 1), bids=(bi, bc))
    with pytest.raises(ValueError):
        oracle.serial_cap(inst, cap0, bids=(bi[:, :2], bc))
