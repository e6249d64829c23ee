"""GPU parity of the path with node capacity against the CPU oracle (bit-exact: integer
work).

Compared element by element: the actions of the serial GPU sweep and of Picard against
the oracle's serial rollout with capacity; final stock and capacities; the pass count,
the changed-order count of every pass and the cache after every pass against the
oracle's Algorithm 1 under the same time blocks.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import (bid_prices, capacity, make_instance, random_tiny,
                                             workload_capacity)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_01939_amd import api as A
    A.lib()
    return A


def _tiny(seed, **kw):
    rng = np.random.default_rng(20_000 + seed)
    inst = random_tiny(seed, qmax=1, **kw)
    T = int(inst.traj_offsets[-1])
    cap0 = rng.integers(0, max(2, T // inst.N + 2), inst.N).astype(np.int32)
    return inst, cap0


def _check_against_oracle(api, oracle, inst, cap0, B, init=None, record=True, gamma=(0, 1),
                          bids=None):
    T = int(inst.traj_offsets[-1])
    prob = api.DeviceProblem.from_instance(inst)
    want = oracle.serial_cap(inst, cap0, gamma=gamma, bids=bids)
    ref = oracle.picard_timeblocks_cap(inst, cap0, B, init_cache=init, record=record,
                                       gamma=gamma, bids=bids)
    init_dev = None if init is None else torch.from_numpy(init).cuda()
    out = api.pk_picard_simulate_capacity(prob, cap0, block_len=B, init_cache=init_dev,
                                          record=record, gamma=gamma, bids=bids)
    np.testing.assert_array_equal(out["actions"].cpu().numpy(), want["actions"])
    np.testing.assert_array_equal(out["final_inv"].cpu().numpy()[0], want["final_inv"])
    np.testing.assert_array_equal(out["final_cap"].cpu().numpy(), want["final_cap"])
    assert out["passes"] == ref["passes"]
    np.testing.assert_array_equal(out["changed"], ref["changed"])
    if record:
        np.testing.assert_array_equal(out["caches"].cpu().numpy(), ref["caches"])
    ser = api.pk_serial_simulate_capacity(prob, cap0, gamma=gamma, bids=bids)
    np.testing.assert_array_equal(ser["actions"].cpu().numpy(), want["actions"])
    np.testing.assert_array_equal(ser["final_inv"].cpu().numpy()[0], want["final_inv"])
    np.testing.assert_array_equal(ser["final_cap"].cpu().numpy(), want["final_cap"])
    return out


@pytest.mark.parametrize("B", [1, 2, 3, 7, 64, 255])
@pytest.mark.parametrize("seed", range(4))
def test_tiny(api, oracle, seed, B):
    inst, cap0 = _tiny(seed, N=2 + seed % 5, K=1 + seed % 4, R=1 + seed % 3, T=40,
                       inv_max=4)
    _say(f"capacity tiny seed={seed} B={B}")
    _check_against_oracle(api, oracle, inst, cap0, B)


@pytest.mark.parametrize("seed", range(3))
def test_tiny_warm_start(api, oracle, seed):
    inst, cap0 = _tiny(seed + 50, N=5, K=3, R=3, T=60, inv_max=5)
    T = int(inst.traj_offsets[-1])
    init = np.random.default_rng(seed).integers(-1, inst.N, T).astype(np.int32)
    _say(f"capacity warm start seed={seed}")
    _check_against_oracle(api, oracle, inst, cap0, 4, init=init)
    # warm start from the answer: one pass confirms it
    want = oracle.serial_cap(inst, cap0)["actions"]
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate_capacity(prob, cap0, block_len=4,
                                          init_cache=torch.from_numpy(want).cuda())
    assert out["passes"] == 1


def test_wide_and_ragged(api, oracle):
    """N = 128 (every lane holds two nodes), T not a multiple of B, several SKU pieces."""
    inst = make_instance("greedy_cap_n10_k100_t1e4", N=128, K=3, R=7, T=5003)
    cap0 = capacity(inst.N, 5003, 0.5)
    _say("capacity wide N=128 T=5003 B=97")
    _check_against_oracle(api, oracle, inst, cap0, 97)


def test_small_workload(api, oracle):
    """N=10, K=100, R=20, T=1e4, 80% capacity, B=100 (every pass against the oracle)."""
    inst = make_instance("greedy_cap_n10_k100_t1e4")
    cap0 = workload_capacity("greedy_cap_n10_k100_t1e4")
    _say("capacity workload n10 k100 t1e4 B=100")
    out = _check_against_oracle(api, oracle, inst, cap0, 100)
    _say(f"  passes {out['passes']}")


def test_edge_cases(api, oracle):
    inst, _ = _tiny(7, N=4, K=3, R=2, T=30, inv_max=3)
    prob = api.DeviceProblem.from_instance(inst)
    T = int(inst.traj_offsets[-1])
    _say("capacity edge cases")
    # no capacity anywhere: every order lost, one pass
    out = api.pk_picard_simulate_capacity(prob, np.zeros(inst.N, np.int32), block_len=5)
    assert (out["actions"].cpu().numpy() == -1).all() and out["passes"] == 1
    # capacity that never binds: the no-capacity greedy rollout
    big = np.full(inst.N, T, np.int32)
    out = api.pk_picard_simulate_capacity(prob, big, block_len=5)
    ref = api.pk_serial_simulate(prob, "greedy")
    np.testing.assert_array_equal(out["actions"].cpu().numpy(), ref["actions"].cpu().numpy())
    # input checks on the device: multi-unit order, bad initial cache
    bad = dataclasses.replace(inst, qty=inst.qty.copy())
    bad.qty[3] = 2
    with pytest.raises(api.PicardError, match="quantity"):
        api.pk_picard_simulate_capacity(api.DeviceProblem.from_instance(bad), big)
    with pytest.raises(api.PicardError, match="initial cache"):
        api.pk_picard_simulate_capacity(prob, big, init_cache=torch.full((T,), inst.N,
                                        dtype=torch.int32, device="cuda"))
    # too few passes
    out = api.pk_picard_simulate_capacity(prob, np.full(inst.N, 3, np.int32), block_len=1,
                                          max_passes=1, raise_not_converged=False)
    assert out["status"] in (api.PK_OK, api.PK_ERR_NOT_CONVERGED)


def test_full_size(api, oracle):
    """N=100, K=1e5, R=200, T=1e6, 60% capacity, default blocks (96 orders): Picard equals
    the serial GPU sweep and the oracle's serial rollout; pass count and changed orders per
    pass equal the oracle's Algorithm 1 under the same blocks."""
    inst = make_instance("greedy_cap_n100_k1e5_t1e6")
    cap0 = workload_capacity("greedy_cap_n100_k1e5_t1e6")
    _say("capacity full size n100 k1e5 t1e6 B=96")
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate_capacity(prob, cap0)
    want = oracle.serial_cap(inst, cap0)
    np.testing.assert_array_equal(out["actions"].cpu().numpy(), want["actions"])
    np.testing.assert_array_equal(out["final_inv"].cpu().numpy()[0], want["final_inv"])
    np.testing.assert_array_equal(out["final_cap"].cpu().numpy(), want["final_cap"])
    ser = api.pk_serial_simulate_capacity(prob, cap0, want_final=False)
    np.testing.assert_array_equal(ser["actions"].cpu().numpy(), want["actions"])
    ref = oracle.picard_timeblocks_cap(inst, cap0, 96)
    _say(f"  passes gpu {out['passes']} oracle {ref['passes']}")
    assert out["passes"] == ref["passes"]
    np.testing.assert_array_equal(out["changed"], ref["changed"])


@pytest.mark.parametrize("gamma", [(1, 2), (1, 1), (1000, 1)])
@pytest.mark.parametrize("B", [1, 5, 64])
@pytest.mark.parametrize("seed", range(3))
def test_gamma_tiny(api, oracle, seed, B, gamma):
    """The capacity-dependent policy (the appendix's ablation), every pass."""
    inst, cap0 = _tiny(seed + 80, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=50,
                       inv_max=3)
    _say(f"capacity gamma={gamma} seed={seed} B={B}")
    _check_against_oracle(api, oracle, inst, cap0, B, gamma=gamma)


@pytest.mark.parametrize("gamma", [(1, 2), (1, 1)])
def test_gamma_workloads(api, oracle, gamma):
    """gamma 0.5 and 1 on the 1e4-order workload (every pass) and on N=128, 5003 orders."""
    inst = make_instance("greedy_cap_n10_k100_t1e4")
    _say(f"capacity gamma={gamma} workload n10 k100 t1e4 B=100")
    out = _check_against_oracle(api, oracle, inst, workload_capacity("greedy_cap_n10_k100_t1e4"),
                                100, gamma=gamma)
    _say(f"  passes {out['passes']}")
    wide = make_instance("greedy_cap_n10_k100_t1e4", N=128, K=3, R=7, T=5003)
    _say(f"capacity gamma={gamma} wide N=128 T=5003 B=97")
    _check_against_oracle(api, oracle, wide, capacity(wide.N, 5003, 0.5), 97, gamma=gamma)


@pytest.mark.parametrize("gamma", [(1, 2, 2), (1, 1, 5), (1000, 1, 3)])
@pytest.mark.parametrize("B", [1, 5, 64])
@pytest.mark.parametrize("seed", range(3))
def test_gamma_low_tiny(api, oracle, seed, B, gamma):
    """The near-exhaustion reading (only nodes with less than `low` capacity left pay a
    shadow price), every pass."""
    inst, cap0 = _tiny(seed + 90, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=50,
                       inv_max=3)
    _say(f"capacity gamma_low={gamma} seed={seed} B={B}")
    _check_against_oracle(api, oracle, inst, cap0, B, gamma=gamma)


@pytest.mark.parametrize("gamma", [(1, 2), (1, 1), (2, 1)])
def test_gamma_low_workloads(api, oracle, gamma):
    """The near-exhaustion reading on the 1e4-order workload (every pass; prices below a
    fifth of each node's capacity) and on N=128, 5003 orders."""
    name = "greedy_cap_n10_k100_t1e4"
    inst = make_instance(name)
    cap0 = workload_capacity(name)
    g = gamma + (max(1, int(cap0.max()) // 5),)
    _say(f"capacity gamma_low={g} workload n10 k100 t1e4 B=100")
    out = _check_against_oracle(api, oracle, inst, cap0, 100, gamma=g)
    _say(f"  passes {out['passes']}")
    wide = make_instance(name, N=128, K=3, R=7, T=5003)
    wc = capacity(wide.N, 5003, 0.5)
    _say(f"capacity gamma_low wide N=128 T=5003 B=97")
    _check_against_oracle(api, oracle, wide, wc, 97, gamma=gamma + (max(1, int(wc.max()) // 5),))


@pytest.mark.parametrize("which", ["both", "inv", "cap"])
@pytest.mark.parametrize("B", [1, 4, 64])
@pytest.mark.parametrize("seed", range(3))
def test_bid_prices_tiny(api, oracle, seed, B, which):
    """The bid-price policy (least cost + price of the unit of stock + price of the unit of
    capacity), with both price vectors or one of them, every pass."""
    inst, cap0 = _tiny(seed + 300, N=2 + seed % 5, K=1 + seed % 3, R=1 + seed % 3, T=50,
                       inv_max=3)
    bi, bc = bid_prices(inst.K, inst.N, seed, spread=60)
    bids = (bi if which != "cap" else None, bc if which != "inv" else None)
    _say(f"capacity bids={which} seed={seed} B={B}")
    _check_against_oracle(api, oracle, inst, cap0, B, bids=bids)


def test_bid_prices_workloads(api, oracle):
    """The bid-price policy on the 1e4-order workload (every pass) and on N=128, 5003
    orders; zero prices are the greedy policy."""
    name = "greedy_cap_n10_k100_t1e4"
    inst = make_instance(name)
    cap0 = workload_capacity(name)
    _say("capacity bids workload n10 k100 t1e4 B=100")
    out = _check_against_oracle(api, oracle, inst, cap0, 100,
                                bids=bid_prices(inst.K, inst.N, 1))
    _say(f"  passes {out['passes']}")
    wide = make_instance(name, N=128, K=3, R=7, T=5003)
    wc = capacity(wide.N, 5003, 0.5)
    _say("capacity bids wide N=128 T=5003 B=97")
    _check_against_oracle(api, oracle, wide, wc, 97, bids=bid_prices(wide.K, wide.N, 2))
    prob = api.DeviceProblem.from_instance(inst)
    z = api.pk_picard_simulate_capacity(prob, cap0, block_len=100,
                                        bids=(np.zeros((inst.K, inst.N), np.int32),
                                              np.zeros(inst.N, np.int32)))
    np.testing.assert_array_equal(z["actions"].cpu().numpy(),
                                  oracle.serial_cap(inst, cap0)["actions"])


def test_bid_prices_rejected(api):
    """Prices outside [0, 2^24) and bid prices with a capacity-dependent gamma are errors."""
    inst, cap0 = _tiny(7, N=3, K=2, R=2, T=20)
    prob = api.DeviceProblem.from_instance(inst)
    bi, bc = bid_prices(inst.K, inst.N, 0)
    for bad in ((bi - 100, None), (None, bc + (1 << 24))):
        _say(f"capacity bids rejected")
        with pytest.raises(api.PicardError, match=r"bits 0x80:"):
            api.pk_picard_simulate_capacity(prob, cap0, block_len=4, bids=bad)
        with pytest.raises(api.PicardError, match=r"bits 0x80:"):
            api.pk_serial_simulate_capacity(prob, cap0, bids=bad)
    with pytest.raises(api.PicardError, match="gamma_num = 0"):
        api.pk_picard_simulate_capacity(prob, cap0, gamma=(1, 2), bids=(bi, bc))


@pytest.mark.parametrize("seed", range(3))
def test_pass_limit(api, oracle, seed):
    """Passes go out in groups: a limit one short of convergence returns PK_ERR_NOT_CONVERGED
    with the oracle's cache after that many passes; a limit at convergence returns the
    fixed point with the oracle's pass count."""
    inst, cap0 = _tiny(seed + 200, N=5, K=3, R=3, T=80, inv_max=4)
    ref = oracle.picard_timeblocks_cap(inst, cap0, 3, record=True)
    k = ref["passes"]
    assert k >= 3, "instance too easy for this test"
    prob = api.DeviceProblem.from_instance(inst)
    _say(f"capacity pass limit seed={seed} passes={k}")
    out = api.pk_picard_simulate_capacity(prob, cap0, block_len=3, max_passes=k)
    assert out["status"] == api.PK_OK and out["passes"] == k
    np.testing.assert_array_equal(out["changed"], ref["changed"])
    for lim in (k - 1, k - 2):
        out = api.pk_picard_simulate_capacity(prob, cap0, block_len=3, max_passes=lim,
                                              raise_not_converged=False)
        assert out["status"] == api.PK_ERR_NOT_CONVERGED and out["passes"] == lim
        np.testing.assert_array_equal(out["actions"].cpu().numpy(), ref["caches"][lim - 1])
