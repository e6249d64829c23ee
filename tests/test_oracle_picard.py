"""Pins of the oracle's Picard iteration (Algorithm 1) and its run form.

* Proposition 2.1: for ANY partition and ANY initial cache, Algorithm 1 returns the
  serial actions after at most T iterations, i.e. k* <= T with k* the first pass whose
  cache equals the serial trajectory, and the returned pass index is k* + 1.
* Any fixed point equals the serial trajectory.
* Section 3.1 (special case, applied per SKU since SKUs do not interact without
  capacity): with the greedy policy and alpha^0 = lost sale, the cache is correct after
  max_k d_k + 1 passes, d_k = number of warehouses that SKU k empties in the serial run.
* Block partitions: run j of a segment is exact by pass j (Proposition 2.1's induction
  with runs as units), so k* <= max number of runs of a segment; a product partition
  (Section 3) gives k* <= 1.
* The run form equals the brute-force algorithm pass by pass on random tiny instances.
"""
import numpy as np
import pytest

from paper_2406_01939_amd.instances import random_tiny


def _kstar(caches, serial_actions, init=None):
    """First k >= 0 with alpha^k == serial (alpha^0 = init or all lost sales)."""
    a0 = np.full_like(serial_actions, -1) if init is None else init
    if np.array_equal(a0, serial_actions):
        return 0
    for k, c in enumerate(caches, start=1):
        if np.array_equal(c, serial_actions):
            return k
    raise AssertionError("never reached the serial trajectory")


def _depleted(inst, final_inv):
    return ((inst.x0[0] > 0) & (final_inv == 0)).sum(axis=1)


@pytest.mark.parametrize("seed", range(60))
def test_alg1_equals_runs_blocks(oracle, seed):
    mlp = seed % 3 == 2
    inst = random_tiny(seed, N=2 + seed % 4, K=1 + seed % 3, R=1 + seed % 3, T=14,
                       qmax=1 + seed % 2, inv_max=3, mlp=mlp, n_hidden_layers=1 + seed % 2)
    T = inst.total_orders
    for B in (1, 2, 3, 5, T):
        w = oracle.block_workers(inst, B)
        lit = oracle.alg1(inst, w, int(w.max()) + 1)
        run = oracle.picard_runs(inst, w, record=True)
        assert lit["passes"] == run["passes"]
        np.testing.assert_array_equal(lit["caches"], run["caches"])
        ser = oracle.serial(inst)["actions"]
        np.testing.assert_array_equal(lit["actions"], ser)


@pytest.mark.parametrize("seed", range(40))
def test_prop21_any_partition_any_init(oracle, seed):
    rng = np.random.default_rng(1000 + seed)
    mlp = seed % 4 == 3
    inst = random_tiny(seed + 500, N=3, K=2, R=2, T=12, qmax=1 + seed % 3, mlp=mlp)
    T = inst.total_orders
    P = int(rng.integers(1, T + 1))
    worker = rng.integers(0, P, T)  # arbitrary, non-contiguous partition
    init = rng.integers(-1, inst.N, T).astype(np.int32) if seed % 2 else None
    r = oracle.alg1(inst, worker, P, init_cache=init)
    ser = oracle.serial(inst)["actions"]
    assert r["converged"]
    np.testing.assert_array_equal(r["actions"], ser)
    ks = _kstar(r["caches"], ser, init)
    assert ks <= T
    assert r["passes"] == ks + 1


@pytest.mark.parametrize("seed", range(30))
def test_greedy_depletion_bound(oracle, seed):
    inst = random_tiny(seed + 2000, N=5, K=3, R=3, T=40, qmax=1 + seed % 3, inv_max=4)
    ser = oracle.serial(inst)
    bound = int(_depleted(inst, ser["final_inv"]).max()) + 1
    rng = np.random.default_rng(seed)
    T = inst.total_orders
    partitions = [oracle.block_workers(inst, B) for B in (1, 2, 4, 7)]
    partitions.append(rng.integers(0, 6, T))  # random (uniform) partition, Section 4.1
    for w in partitions:
        r = oracle.alg1(inst, w, int(w.max()) + 1)
        assert _kstar(r["caches"], ser["actions"]) <= bound


@pytest.mark.parametrize("seed", range(20))
def test_run_count_bound_and_product_partition(oracle, seed):
    mlp = seed % 2 == 1
    inst = random_tiny(seed + 3000, N=4, K=3, R=2, T=40, qmax=2, inv_max=3, mlp=mlp)
    ser = oracle.serial(inst)["actions"]
    rng = np.random.default_rng(seed)
    init = rng.integers(-1, inst.N, inst.total_orders).astype(np.int32)
    for B in (1, 3, 8):
        w = oracle.block_workers(inst, B)
        r = oracle.picard_runs(inst, w, init_cache=init, record=True)
        runs = oracle.n_runs_per_segment(inst, w).max()
        assert _kstar(r["caches"], ser, init) <= runs
    prod = oracle.product_workers(inst)
    r = oracle.alg1(inst, prod, inst.K)
    assert r["passes"] <= 2
    np.testing.assert_array_equal(r["actions"], ser)


def test_runs_split_process_alternating(oracle):
    """Each process owns two runs of the one SKU: the run form carries the process's own
    fresh-minus-cached consumption from its first run to its second."""
    inst = random_tiny(5, N=3, K=1, R=1, T=6)
    worker = np.array([0, 1, 0, 1, 0, 1])
    lit = oracle.alg1(inst, worker, 2)
    run = oracle.picard_runs(inst, worker, record=True)
    assert lit["passes"] == run["passes"]
    np.testing.assert_array_equal(lit["caches"], run["caches"])
    np.testing.assert_array_equal(run["actions"], oracle.serial(inst)["actions"])


@pytest.mark.parametrize("seed", range(40))
def test_alg1_equals_runs_random_partitions(oracle, seed):
    """Uniform random partitions (Section 4.1): a process owns scattered orders, so it
    has many runs of one SKU.  Every pass's cache equals Algorithm 1's."""
    rng = np.random.default_rng(4000 + seed)
    mlp = seed % 4 == 1
    inst = random_tiny(seed + 4100, N=4, K=1 + seed % 3, R=3, T=30, qmax=1 + seed % 3,
                       inv_max=5, mlp=mlp)
    T = inst.total_orders
    P = int(rng.integers(2, 8))
    worker = rng.integers(0, P, T)
    init = rng.integers(-1, inst.N, T).astype(np.int32) if seed % 2 else None
    lit = oracle.alg1(inst, worker, P, init_cache=init)
    run = oracle.picard_runs(inst, worker, init_cache=init, record=True)
    assert lit["passes"] == run["passes"]
    np.testing.assert_array_equal(lit["caches"], run["caches"])


def test_not_converged_reports_partial(oracle):
    inst = random_tiny(17, N=4, K=1, R=2, T=30, inv_max=3)
    w = oracle.block_workers(inst, 1)
    full = oracle.picard_runs(inst, w, record=True)
    assert full["passes"] >= 3
    part = oracle.picard_runs(inst, w, max_passes=1)
    assert not part["converged"] and part["passes"] == 1
    np.testing.assert_array_equal(part["actions"], full["caches"][0])


def test_fixed_point_is_serial(oracle):
    """Starting from the serial actions, the first pass changes nothing (k* = 0)."""
    for seed in range(10):
        inst = random_tiny(seed + 77, N=4, K=2, R=2, T=25, qmax=2, mlp=seed % 2 == 0)
        ser = oracle.serial(inst)["actions"]
        w = oracle.block_workers(inst, 3)
        r = oracle.picard_runs(inst, w, init_cache=ser)
        assert r["passes"] == 1
        np.testing.assert_array_equal(r["actions"], ser)


@pytest.mark.parametrize("B", [1, 64, 100, 1000])
def test_workload_small_converges_to_serial(oracle, B):
    from paper_2406_01939_amd.instances import make_instance
    inst = make_instance("greedy_n10_k100_t1e4")
    ser = oracle.serial(inst)
    w = oracle.block_workers(inst, B)
    r = oracle.picard_runs(inst, w)
    np.testing.assert_array_equal(r["actions"], ser["actions"])
    bound = int(_depleted(inst, ser["final_inv"]).max()) + 1
    assert r["passes"] - 1 <= bound
