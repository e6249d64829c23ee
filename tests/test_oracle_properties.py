"""Property-based pins of the oracle (hypothesis): random tiny instances, partitions and
initial caches, shrunk to a minimal case on failure.

- Algorithm 1 by brute force and the run form give the same cache after every pass and
  the same pass count, for any partition and initial cache.
- Proposition 2.1: from any initial cache the iteration returns within T + 1 passes
  with the serial rollout's actions.
- The advantages of a rollout: consecutive differences are the step rewards, they sum
  to zero over the trajectory, and the first step's reward-to-go is the total reward.
- With node capacity (either policy): the time-block replay equals the brute-force
  Algorithm 1 pass by pass and reaches the serial rollout within T + 1 passes.
"""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2406_01939_amd.instances import Instance

SETTINGS = settings(max_examples=60, deadline=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def tiny_case(draw, mlp=False):
    N = draw(st.integers(1, 4))
    K = draw(st.integers(1, 3))
    R = draw(st.integers(1, 3))
    T = draw(st.integers(1, 14))
    qmax = draw(st.integers(1, 3))
    ints = lambda lo, hi, n: np.array(draw(st.lists(st.integers(lo, hi), min_size=n,
                                                      max_size=n)), dtype=np.int32)
    sku, region, qty = ints(0, K - 1, T), ints(0, R - 1, T), ints(1, qmax, T)
    x0 = ints(0, 4, K * N).reshape(1, K, N)
    cost = ints(1, 5, N * R).reshape(1, N, R)
    P = draw(st.integers(1, T))
    worker = ints(0, P - 1, T).astype(np.int64)
    init = ints(-1, N - 1, T) if draw(st.booleans()) else None
    params = None
    if mlp:
        from paper_2406_01939_amd.instances import make_params
        params = make_params(R, draw(st.integers(0, 1000)))
    inst = Instance(N=N, K=K, R=R, traj_offsets=np.array([0, T], np.int64), sku=sku,
                    region=region, qty=qty, x0=x0, cost=cost,
                    rng_seed=draw(st.integers(0, 2**63 - 1)), params=params, name="hyp")
    return inst, worker, P, init


@SETTINGS
@given(tiny_case())
def test_alg1_equals_run_form_greedy(oracle, case):
    inst, worker, P, init = case
    lit = oracle.alg1(inst, worker, P, init_cache=init)
    run = oracle.picard_runs(inst, worker, init_cache=init, record=True)
    assert lit["passes"] == run["passes"]
    np.testing.assert_array_equal(lit["caches"], run["caches"])


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_case(mlp=True))
def test_alg1_equals_run_form_learned(oracle, case):
    inst, worker, P, init = case
    lit = oracle.alg1(inst, worker, P, init_cache=init)
    run = oracle.picard_runs(inst, worker, init_cache=init, record=True)
    assert lit["passes"] == run["passes"]
    np.testing.assert_array_equal(lit["caches"], run["caches"])


@SETTINGS
@given(tiny_case())
def test_prop21_converges_to_serial(oracle, case):
    inst, worker, P, init = case
    r = oracle.alg1(inst, worker, P, init_cache=init)
    assert r["converged"] and r["passes"] <= inst.total_orders + 1
    np.testing.assert_array_equal(r["actions"], oracle.serial(inst)["actions"])


@SETTINGS
@given(tiny_case(), st.integers(-3, 12))
def test_advantage_identities(oracle, case, revenue):
    inst = case[0]
    s = oracle.serial(inst)
    out = oracle.advantages(inst, s["actions"], s["shipped"], revenue)
    r, G, A = out["rewards"], out["rtg"], out["advantages"].astype(np.float64)
    assert out["ret"] == int(r.sum()) == int(G[0])
    np.testing.assert_array_equal(G[:-1] - G[1:], r[:-1])
    scale = max(1.0, float(np.abs(A).max()))
    np.testing.assert_allclose(A[:-1] - A[1:], r[:-1].astype(np.float64),
                               atol=4 * scale * 2**-24)
    assert abs(A.sum()) <= r.size * scale * 2**-23


# ---------------------------------------------------------------- node capacity
@st.composite
def tiny_capacity_case(draw):
    N = draw(st.integers(1, 5))
    K = draw(st.integers(1, 3))
    R = draw(st.integers(1, 3))
    T = draw(st.integers(1, 16))
    ints = lambda lo, hi, n: np.array(draw(st.lists(st.integers(lo, hi), min_size=n,
                                                      max_size=n)), dtype=np.int32)
    inst = Instance(N=N, K=K, R=R, traj_offsets=np.array([0, T], np.int64),
                    sku=ints(0, K - 1, T), region=ints(0, R - 1, T),
                    qty=np.ones(T, np.int32), x0=ints(0, 4, K * N).reshape(1, K, N),
                    cost=ints(1, 5, N * R).reshape(1, N, R), rng_seed=0, params=None,
                    name="hypcap")
    cap0 = ints(0, 6, N)
    B = draw(st.integers(1, T))
    init = ints(-1, N - 1, T) if draw(st.booleans()) else None
    gamma = draw(st.sampled_from([(0, 1), (0, 1), (1, 2), (1, 1), (3, 1)]))
    return inst, cap0, B, init, gamma


@SETTINGS
@given(tiny_capacity_case())
def test_capacity_time_blocks_equal_alg1(oracle, case):
    """With node capacity, for either policy: the time-block replay equals the brute-force
    Algorithm 1 under the same blocks pass by pass, and both end at the serial rollout
    within T + 1 passes from any initial cache (Proposition 2.1)."""
    inst, cap0, B, init, gamma = case
    T = int(inst.traj_offsets[-1])
    lit = oracle.alg1_cap(inst, cap0, oracle.time_block_workers(T, B), (T + B - 1) // B,
                          init_cache=init, gamma=gamma)
    tb = oracle.picard_timeblocks_cap(inst, cap0, B, init_cache=init, record=True,
                                      gamma=gamma)
    assert lit["converged"] and tb["converged"]
    assert lit["passes"] == tb["passes"] <= T + 1
    assert np.array_equal(lit["caches"], tb["caches"])
    assert np.array_equal(tb["actions"], oracle.serial_cap(inst, cap0, gamma=gamma)["actions"])
