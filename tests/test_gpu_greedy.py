"""GPU parity of the greedy path against the CPU oracle (bit-exact: integer work).

Compared element by element: actions, units shipped and final inventory against the
serial oracle; passes per trajectory and the cache after every pass against the
oracle's Picard iteration under the same block partition.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import Instance, make_instance, random_tiny

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


def _oracle_batch(oracle, inst, B=None):
    """Serial results per trajectory (+ Picard passes under blocks of B if given)."""
    acts, ships, fins, passes = [], [], [], []
    workers = oracle.block_workers(inst, B) if B else None
    for b in range(inst.n_traj):
        r = oracle.serial(inst, b)
        acts.append(r["actions"]); ships.append(r["shipped"]); fins.append(r["final_inv"])
        if B:
            lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
            pr = oracle.picard_runs(inst, workers[lo:hi], b)
            assert pr["converged"]
            np.testing.assert_array_equal(pr["actions"], r["actions"])
            passes.append(pr["passes"])
    return (np.concatenate(acts) if acts else np.zeros(0, np.int32),
            np.concatenate(ships) if ships else np.zeros(0, np.int32),
            np.stack(fins), np.array(passes))


def _check(out, inst, want_a, want_s, want_f):
    np.testing.assert_array_equal(out["actions"].cpu().numpy(), want_a)
    if out.get("shipped") is not None:
        np.testing.assert_array_equal(out["shipped"].cpu().numpy(), want_s)
    if out.get("final_inv") is not None:
        np.testing.assert_array_equal(out["final_inv"].cpu().numpy(), want_f)


@pytest.mark.parametrize("B", [1, 2, 3, 7, 64, 1000])
@pytest.mark.parametrize("seed", range(4))
def test_tiny_batches(api, oracle, seed, B):
    inst = random_tiny(seed, N=1 + seed * 3, K=4, R=3, T=150, qmax=1 + seed % 3, inv_max=5,
                       n_traj=3)
    _say(f"case tiny seed={seed} B={B} total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=B, validate=True)
    _check(out, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(out["passes"], want_p)


def test_every_pass_matches_oracle_cache(api, oracle):
    inst = make_instance("greedy_n10_k100_t1e4")
    B = 100
    w = oracle.block_workers(inst, B)
    ref = oracle.picard_runs(inst, w, record=True)
    prob = api.DeviceProblem.from_instance(inst)
    _say(f"case small workload passes={ref['passes']}")
    for k in range(1, ref["passes"] + 1):
        out = api.pk_picard_simulate(prob, "greedy", block_len=B, max_passes=k,
                                     raise_not_converged=False)
        np.testing.assert_array_equal(out["actions"].cpu().numpy(), ref["caches"][k - 1])
        if k < ref["passes"]:
            assert out["status"] == api.PK_ERR_NOT_CONVERGED
        else:
            assert out["status"] == api.PK_OK
    assert int(out["passes"][0]) == ref["passes"]


@pytest.mark.parametrize("B", [100, 1, 17, 10_000])
def test_small_workload(api, oracle, B):
    inst = make_instance("greedy_n10_k100_t1e4")
    _say(f"case small workload B={B}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=B)
    _check(out, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(out["passes"], want_p)
    if B >= 10_000:
        assert out["passes"][0] <= 2  # product partition


@pytest.mark.parametrize("N,R,n_traj,qmax", [
    (200, 20, 1, 1),   # stock set in LDS (N > 128), 16-bit keys, one trajectory
    (200, 20, 3, 2),   # the same, batched: key table in global memory
    (300, 30, 1, 1),   # 32-bit keys (N > 256)
    (300, 30, 2, 3),
    (100, 1000, 1, 1), # one trajectory whose key table does not fit in LDS
])
@pytest.mark.parametrize("B", [97, 1000])  # short runs only; runs of several 64-order steps
def test_wide_shapes(api, oracle, N, R, n_traj, qmax, B):
    """Warehouse and region counts past the benchmark's: every layout of the walk (stock
    set in registers or LDS, 16- or 32-bit keys, key table in LDS or global memory)."""
    inst = random_tiny(100 + N + R, N=N, K=6, R=R, T=2500, qmax=qmax, inv_max=2, n_traj=n_traj)
    _say(f"case wide N={N} R={R} n_traj={n_traj} B={B} total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=B, validate=True)
    _check(out, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(out["passes"], want_p)


@pytest.mark.parametrize("N", [255, 256, 257])
@pytest.mark.parametrize("n_traj", [1, 2])
def test_last_warehouse_costliest_and_only_stock(api, oracle, N, n_traj):
    """Key-width boundary: the costliest warehouse of every region is the last one and the
    only one with stock.  Its key is the largest of the table (at N = 256 with 16-bit keys
    it would be 0xffff, the value that stands for "no stock"), so Picard and the serial
    sweep must still ship from it until it runs out."""
    inst = random_tiny(400 + N, N=N, K=3, R=5, T=600, qmax=2, inv_max=0, n_traj=n_traj)
    inst.cost[:] = np.random.default_rng(N).integers(1, 100, inst.cost.shape)
    inst.cost[:, N - 1, :] = 100
    inst.x0[:] = 0
    inst.x0[:, :, N - 1] = 150
    _say(f"case last warehouse only stock N={N} n_traj={n_traj} total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, 64)
    assert (want_a == N - 1).any() and (want_a == -1).any()
    prob = api.DeviceProblem.from_instance(inst)
    for B in (64, 1000):
        out = api.pk_picard_simulate(prob, "greedy", block_len=B, validate=True)
        _check(out, inst, want_a, want_s, want_f)
    out = api.pk_picard_simulate(prob, "greedy", block_len=64, validate=True)
    np.testing.assert_array_equal(out["passes"], want_p)
    ser = api.pk_serial_simulate(prob, "greedy")
    _check(ser, inst, want_a, want_s, want_f)


def test_serial_sweep_matches_oracle(api, oracle):
    inst = random_tiny(11, N=70, K=5, R=4, T=400, qmax=3, inv_max=6, n_traj=5)
    _say("case serial sweep tiny batch")
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_serial_simulate(prob, "greedy")
    _check(out, inst, want_a, want_s, want_f)
    inst = make_instance("greedy_n10_k100_t1e4")
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    out = api.pk_serial_simulate(api.DeviceProblem.from_instance(inst), "greedy")
    _check(out, inst, want_a, want_s, want_f)


@pytest.mark.parametrize("N,K,T,qmax", [(1, 1, 300, 3), (64, 1, 1000, 2), (65, 2, 777, 3),
                                         (128, 3, 1500, 1), (100, 7, 2049, 3), (129, 2, 500, 2),
                                         (70, 2, 1024, 2), (66, 3, 1040, 3), (100, 1, 5, 2),
                                         (3, 2, 16, 1), (90, 4, 64 + 15, 2)])
def test_serial_sweep_prefetch_window(api, oracle, N, K, T, qmax):
    """The serial sweep loads an order's stock row several orders ahead; with one to seven
    SKUs almost every order shares its SKU with one of the orders decided since, so its row
    must come from the most recent of them, not from memory.  Warehouse counts on both sides
    of one and two per lane (64, 65, 128, 129), horizons not a multiple of 16 or 64, and
    enough stock that warehouses run out mid-way; horizons that end a group of 16 orders
    inside a chunk of 64, end a chunk, or stop short of one group."""
    demand = 0.75 * T * (qmax + 1) / 2  # per trajectory, about
    inst = random_tiny(500 + N + K, N=N, K=K, R=5, T=T, qmax=qmax,
                       inv_max=max(1, int(demand / (K * N))), n_traj=3)  # stock ~ half of it
    _say(f"case serial prefetch window N={N} K={K} T={T} total={inst.total_orders}")
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    if T >= 100:
        assert (want_a == -1).any() and (want_a >= 0).any()
    out = api.pk_serial_simulate(api.DeviceProblem.from_instance(inst), "greedy")
    _check(out, inst, want_a, want_s, want_f)


def test_serial_sweep_full_workloads(api, oracle):
    """The serial sweep on the 1e6-order workload and on the 256-trajectory batch
    (1.2e8 orders, quantities 1..3), bit-exact against the oracle's serial rollouts (run
    in threads, one trajectory each)."""
    from concurrent.futures import ThreadPoolExecutor
    for name in ("greedy_n100_k1e5_t1e6", "greedy_batch256_n50_k2e4"):
        inst = make_instance(name)
        _say(f"case serial sweep full {name}: {inst.total_orders} orders")
        prob = api.DeviceProblem.from_instance(inst)
        out = api.pk_serial_simulate(prob, "greedy")
        acts = out["actions"].cpu().numpy()
        ship = out["shipped"].cpu().numpy()
        fin = out["final_inv"].cpu().numpy()
        del out, prob

        def one(b):
            lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
            r = oracle.serial(inst, b)
            return (np.array_equal(r["actions"], acts[lo:hi]) and
                    np.array_equal(r["shipped"], ship[lo:hi]) and
                    np.array_equal(r["final_inv"], fin[b]))

        with ThreadPoolExecutor(max_workers=16) as ex:
            ok = list(ex.map(one, range(inst.n_traj)))
        assert all(ok), [b for b, v in enumerate(ok) if not v][:10]


def test_edge_cases(api, oracle):
    # a batch with empty trajectories in it
    inst = random_tiny(21, N=3, K=2, R=2, T=20, n_traj=3)
    inst.traj_offsets = np.array([0, 0, 10, 10], dtype=np.int64)
    inst.sku, inst.region, inst.qty = inst.sku[:10], inst.region[:10], inst.qty[:10]
    _say("case empty trajectories")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, 4)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=4)
    _check(out, inst, want_a, want_s, want_f)
    assert list(out["passes"]) == [1, want_p[1], 1]
    # no orders at all
    inst0 = random_tiny(22, N=3, K=2, R=2, T=5)
    inst0.traj_offsets = np.array([0, 0], dtype=np.int64)
    inst0.sku = inst0.sku[:0]; inst0.region = inst0.region[:0]; inst0.qty = inst0.qty[:0]
    _say("case no orders")
    out = api.pk_picard_simulate(api.DeviceProblem.from_instance(inst0), "greedy", block_len=4)
    np.testing.assert_array_equal(out["final_inv"].cpu().numpy(), inst0.x0)
    # no stock anywhere: every order is lost, the first pass already equals alpha^0
    inst1 = random_tiny(23, N=4, K=3, R=2, T=50)
    inst1.x0[:] = 0
    _say("case no stock")
    out = api.pk_picard_simulate(api.DeviceProblem.from_instance(inst1), "greedy", block_len=5)
    assert (out["actions"].cpu().numpy() == -1).all() and out["passes"][0] == 1
    # one warehouse, one order
    inst2 = random_tiny(24, N=1, K=1, R=1, T=1, inv_max=1)
    _say("case single order")
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst2)
    out = api.pk_picard_simulate(api.DeviceProblem.from_instance(inst2), "greedy", block_len=1)
    _check(out, inst2, want_a, want_s, want_f)


def test_partial_ship_then_same_warehouse(api, oracle):
    """Regression: in one step a warehouse's only order asks for more than its stock and
    ships partially (no order is cut); the warehouse must leave the stock set, so an
    order in the next step that prefers it goes elsewhere.  Two warehouses, region 0
    prefers w0 and region 1 prefers w1."""
    from paper_2406_01939_amd.instances import Instance
    T = 66
    region = np.ones(T, np.int32)
    region[0] = 0
    region[T - 1] = 0
    qty = np.ones(T, np.int32)
    qty[0] = 3
    inst = Instance(N=2, K=1, R=2, traj_offsets=np.array([0, T], np.int64),
                    sku=np.zeros(T, np.int32), region=region, qty=qty,
                    x0=np.array([[[2, 1000]]], np.int32),
                    cost=np.array([[[1, 9], [9, 1]]], np.int32), rng_seed=0)
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    assert want_s[0] == 2 and want_a[T - 1] == 1 and want_f.ravel()[0] == 0
    _say("case partial ship then the same warehouse")
    for B in (T, 70, 1):
        out = api.pk_picard_simulate(api.DeviceProblem.from_instance(inst), "greedy", block_len=B)
        _check(out, inst, want_a, want_s, want_f)


def test_warm_start(api, oracle):
    inst = random_tiny(31, N=6, K=3, R=3, T=300, qmax=2, inv_max=8, n_traj=2)
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    prob = api.DeviceProblem.from_instance(inst)
    _say("case warm start from the serial actions")
    init = torch.from_numpy(want_a).cuda()
    out = api.pk_picard_simulate(prob, "greedy", block_len=16, init_cache=init, validate=True)
    _check(out, inst, want_a, want_s, want_f)
    assert list(out["passes"]) == [1, 1]
    _say("case warm start from a random cache")
    rnd = np.random.default_rng(0).integers(-1, inst.N, inst.total_orders).astype(np.int32)
    out = api.pk_picard_simulate(prob, "greedy", block_len=16,
                                 init_cache=torch.from_numpy(rnd).cuda(), validate=True)
    _check(out, inst, want_a, want_s, want_f)
    w = oracle.block_workers(inst, 16)
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        pr = oracle.picard_runs(inst, w[lo:hi], b, init_cache=rnd[lo:hi])
        assert out["passes"][b] == pr["passes"]


def test_errors(api):
    inst = random_tiny(41, N=4, K=3, R=2, T=40)
    prob = api.DeviceProblem.from_instance(inst)
    _say("case errors")
    bad = api.DeviceProblem.from_instance(inst)
    bad.sku = bad.sku.clone()
    bad.sku[3] = 99
    with pytest.raises(api.PicardError) as e:
        api.pk_picard_simulate(bad, "greedy", block_len=4, validate=True)
    assert e.value.status == api.PK_ERR_INVALID_ARG
    bad = api.DeviceProblem.from_instance(inst)
    bad.init_inv = bad.init_inv.clone()
    bad.init_inv[0, 0, 0] = -3
    with pytest.raises(api.PicardError) as e:
        api.pk_picard_simulate(bad, "greedy", block_len=4, validate=True)
    assert e.value.status == api.PK_ERR_INVALID_ARG
    # workspace too small
    import ctypes as C
    p, po = prob.c_problem(), prob.c_policy("greedy")
    o = api.pk_picard_opts(4, 0, 1, 0, None, 0)
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    act = torch.empty(prob.total, dtype=torch.int32, device="cuda")
    st = api.lib().pk_picard_simulate(C.byref(p), C.byref(po), C.byref(o), ws.data_ptr(), 64,
                                      act.data_ptr(), None, None, None, None)
    assert st == api.PK_ERR_WORKSPACE
    # not converged: max_passes = 1 returns the first cache
    out = api.pk_picard_simulate(prob, "greedy", block_len=1, max_passes=1,
                                 raise_not_converged=False)
    assert out["status"] == api.PK_ERR_NOT_CONVERGED


def test_at_scale_1m_orders(api, oracle):
    """The benchmark workload (N=100, K=1e5, R=200, T=1e6) at full size, bit-exact."""
    inst = make_instance("greedy_n100_k1e5_t1e6")
    B = 1024
    _say(f"case 1M orders B={B}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=B)
    _check(out, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(out["passes"], want_p)
    _say(f"passes={out['passes']} stats={out['stats']}")


def test_batched_uneven_horizons(api, oracle):
    """Batched trajectories of uneven horizon (N=50, K=2e4, R=100, q in 1..3), reduced to
    16 trajectories with horizons in [1e4, 1e5]."""
    inst = make_instance("greedy_batch256_n50_k2e4", n_traj=16, T=(10_000, 100_000))
    B = 256
    _say(f"case batch16 total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    for lm in (0, 200):  # automatic (too little work: no lane walk), and lanes up to 200
        out = api.pk_picard_simulate(prob, "greedy", block_len=B, lane_max=lm)
        _check(out, inst, want_a, want_s, want_f)
        np.testing.assert_array_equal(out["passes"], want_p)


def test_no_frontier_gives_same_passes(api, oracle):
    """Re-walking every run every pass (no restart frontier) reproduces the same caches
    and pass counts; the frontier only skips work."""
    inst = make_instance("greedy_n10_k100_t1e4")
    _say("case no frontier")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, 100)
    prob = api.DeviceProblem.from_instance(inst)
    a = api.pk_picard_simulate(prob, "greedy", block_len=100, use_frontier=False)
    _check(a, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(a["passes"], want_p)
    b = api.pk_picard_simulate(prob, "greedy", block_len=100, use_frontier=True)
    assert b["stats"]["orders_walked"] < a["stats"]["orders_walked"]
    assert a["stats"]["orders_walked"] == inst.total_orders * int(want_p[0])


def test_autotune_picks_a_valid_block(api, oracle):
    inst = make_instance("greedy_n10_k100_t1e4")
    _say("case autotune")
    prob = api.DeviceProblem.from_instance(inst)
    B = api.pk_autotune(prob, "greedy")
    assert B in (64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 65536)
    assert api.pk_autotune(prob, "greedy") == B  # cached
    want_a, want_s, want_f, _ = _oracle_batch(oracle, inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=0)
    _check(out, inst, want_a, want_s, want_f)
    assert out["stats"]["block_len"] == B


def test_captured_graph_replays(api, oracle):
    """The pass loop captured as a HIP graph (U passes per replay) gives the no-graph result
    on every replay, with eager work and synchronisations between the replays."""
    inst = make_instance("greedy_batch256_n50_k2e4", n_traj=8, T=(10_000, 50_000))
    prob = api.DeviceProblem.from_instance(inst)
    _say("case graph replays")
    ref = api.pk_picard_simulate(prob, "greedy", block_len=128, graph_unroll=1)
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, 128)
    _check(ref, inst, want_a, want_s, want_f)
    out = None
    for rep in range(4):
        out = api.pk_picard_simulate(prob, "greedy", block_len=128, graph_unroll=3, out=out)
        junk = torch.randn(1 << 20, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out["actions"], ref["actions"]), rep
        assert torch.equal(out["shipped"], ref["shipped"]), rep
        assert torch.equal(out["final_inv"], ref["final_inv"]), rep
        np.testing.assert_array_equal(out["passes"], want_p)
        del junk
    # timing inside the graph (event record nodes around every walk): same results, one
    # duration per walk launch of every replay
    _say("case graph replays with walk timing")
    for rep in range(3):
        out = api.pk_picard_simulate(prob, "greedy", block_len=128, graph_unroll=3, out=out,
                                     timing=True)
        torch.cuda.synchronize()
        assert torch.equal(out["actions"], ref["actions"]), rep
        st = out["stats"]
        assert st["walk_launches"] % 3 == 0 and st["walk_launches"] >= int(want_p.max())
        assert st["walk_ms"] > 0.0


def test_batched_256_trajectories_full_size(api, oracle):
    """Batched greedy workload at full size: 256 trajectories, horizons uniform in
    [1e4, 1e6] (about 1.3e8 orders), N=50, K=2e4, R=100, quantities 1..3.  Actions, units
    shipped and final inventory bit-exact against the serial oracle for every trajectory;
    passes checked against the oracle's Picard iteration on a sample of trajectories."""
    inst = make_instance("greedy_batch256_n50_k2e4")
    prob = api.DeviceProblem.from_instance(inst)
    _say(f"case batch256 full total={inst.total_orders}")
    out = api.pk_picard_simulate(prob, "greedy", block_len=0)
    B = out["stats"]["block_len"]
    acts = out["actions"].cpu().numpy()
    ship = out["shipped"].cpu().numpy()
    fin = out["final_inv"].cpu().numpy()
    w = oracle.block_workers(inst, B)
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        r = oracle.serial(inst, b)
        np.testing.assert_array_equal(acts[lo:hi], r["actions"])
        np.testing.assert_array_equal(ship[lo:hi], r["shipped"])
        np.testing.assert_array_equal(fin[b], r["final_inv"])
        if b % 32 == 0:
            pr = oracle.picard_runs(inst, w[lo:hi], b)
            assert out["passes"][b] == pr["passes"], b
    _say(f"B={B} passes max={out['passes'].max()} mean={out['passes'].mean():.2f}")


@pytest.mark.parametrize("N", [16, 17, 48, 64, 65, 128])
@pytest.mark.parametrize("warm", [False, True])
def test_first_pass_lane_walk(api, oracle, N, warm):
    """The first pass walks runs of up to lane_max orders one per lane and longer runs a wave
    per run.  Run lengths on both sides of the limit (one SKU takes about half the orders,
    in blocks of 700), every preference-row layout (16 to 64 candidates loaded ahead, or two
    chunks of a longer row read further on demand), with and without an initial cache; the
    same results without the lane walk."""
    rng = np.random.default_rng(600 + N)
    inst = random_tiny(600 + N + int(warm), N=N, K=40, R=7, T=4000, qmax=3, inv_max=3,
                       n_traj=2)
    inst.sku[rng.random(inst.total_orders) < 0.5] = 0
    inst.x0[:, 0, :] = rng.integers(0, 40, (inst.n_traj, N))
    B = 700
    _say(f"case lane walk N={N} warm={warm} total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    init = None
    if warm:
        init = rng.integers(-1, N, inst.total_orders).astype(np.int32)
    init_d = None if init is None else torch.from_numpy(init).cuda()
    out = api.pk_picard_simulate(prob, "greedy", block_len=B, validate=True, init_cache=init_d,
                                 lane_max=510)
    _check(out, inst, want_a, want_s, want_f)
    off = api.pk_picard_simulate(prob, "greedy", block_len=B, init_cache=init_d, lane_max=-1)
    assert torch.equal(off["actions"], out["actions"])
    assert torch.equal(off["final_inv"], out["final_inv"])
    np.testing.assert_array_equal(off["passes"], out["passes"])
    w = oracle.block_workers(inst, B)
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        pr = oracle.picard_runs(inst, w[lo:hi], b,
                                init_cache=None if init is None else init[lo:hi])
        assert out["passes"][b] == pr["passes"], b
    assert out["stats"]["orders_walked"] >= inst.total_orders
    # the first pass alone: the cache after one pass, against the oracle's
    out1 = api.pk_picard_simulate(prob, "greedy", block_len=B, max_passes=1,
                                  raise_not_converged=False, init_cache=init_d, lane_max=100)
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        pr = oracle.picard_runs(inst, w[lo:hi], b, max_passes=1, record=True,
                                init_cache=None if init is None else init[lo:hi])
        np.testing.assert_array_equal(out1["actions"].cpu().numpy()[lo:hi], pr["caches"][0])


@pytest.mark.parametrize("K,R,qmax", [
    (70_000, 200, 3),      # 17 SKU bits: two sort passes, region and quantity packed above
    (1 << 21, 2048, 2),    # 21 + 11 bits: region and quantity read through the permutation
    (5_000, 300, 5_000),   # quantities too large for the key word's top bits
])
def test_setup_key_packing(api, oracle, K, R, qmax):
    """The per-call setup sorts each trajectory's orders by SKU with region and quantity
    carried in the key word when they fit: multi-pass sorts whose last digit stops below
    the packed fields, key words with no room for them, and quantities past their field."""
    inst = random_tiny(700 + K % 97 + R, N=5, K=K, R=R, T=6000, qmax=qmax, inv_max=4,
                       n_traj=3)
    inst.qty[::7] = np.minimum(inst.qty[::7], 2)
    B = 64
    _say(f"case key packing K={K} R={R} qmax={qmax} total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, B)
    prob = api.DeviceProblem.from_instance(inst)
    for lm in (0, 64):
        out = api.pk_picard_simulate(prob, "greedy", block_len=B, validate=True, lane_max=lm)
        _check(out, inst, want_a, want_s, want_f)
        np.testing.assert_array_equal(out["passes"], want_p)


def test_results_back_to_time_order_tile_edges(api, oracle):
    """Actions and units shipped return to time order through a sort by destination tile
    of 4096 orders and an in-LDS placement: trajectories empty, of one order, and just
    below, at and above tile multiples."""
    lens = [0, 1, 4095, 4096, 4097, 8197, 0, 3, 12288]
    rng = np.random.default_rng(808)
    base = random_tiny(808, N=7, K=30, R=5, T=sum(lens), qmax=3, inv_max=40)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    nt = len(lens)
    inst = Instance(N=7, K=30, R=5, traj_offsets=offs, sku=base.sku, region=base.region,
                    qty=base.qty, x0=rng.integers(0, 40, (nt, 30, 7)).astype(np.int32),
                    cost=rng.integers(1, 6, (nt, 7, 5)).astype(np.int32), rng_seed=1)
    _say(f"case unpermute tile edges total={inst.total_orders}")
    want_a, want_s, want_f, want_p = _oracle_batch(oracle, inst, 100)
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "greedy", block_len=100, validate=True)
    _check(out, inst, want_a, want_s, want_f)
    np.testing.assert_array_equal(out["passes"], want_p)
