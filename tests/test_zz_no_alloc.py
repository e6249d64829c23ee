"""pk_picard_simulate_noalloc (static device scratch, no workspace) against
pk_picard_simulate on the same inputs: actions, units shipped, final inventory and passes
identical, on two calls in a row with the second on a smaller problem (the static buffer
keeps the first call's contents), for the greedy and the learned policy; the host-side
rejections (a problem too large for the buffer, timing) come back as errors."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import make_instance, random_tiny

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


def _same(api, prob, policy, block_len, partition=None):
    ref = api.pk_picard_simulate(prob, policy, block_len=block_len, partition=partition,
                                 graph_unroll=1)
    got = api.pk_picard_simulate_noalloc(prob, policy, block_len=block_len,
                                         partition=partition)
    assert torch.equal(got["actions"], ref["actions"])
    assert torch.equal(got["shipped"], ref["shipped"])
    assert torch.equal(got["final_inv"], ref["final_inv"])
    np.testing.assert_array_equal(got["passes"], ref["passes"])
    assert got["stats"]["changed_total"] == ref["stats"]["changed_total"]
    assert got["stats"]["orders_walked"] == ref["stats"]["orders_walked"]
    return got


def test_greedy_large_then_small(api):
    big = make_instance("greedy_n100_k1e5_t1e6", T=200_000, K=20_000)
    small = make_instance("greedy_n10_k100_t1e4")
    for name, inst, B in (("greedy 2e5 orders N=100", big, 1024),
                          ("greedy 1e4 orders N=10", small, 100)):
        _say(f"case noalloc {name} B={B}")
        prob = api.DeviceProblem.from_instance(inst)
        out = _same(api, prob, "greedy", B)
        _say(f"  passes {int(out['passes'].max())}")


def test_batch_and_partition_then_smaller(api):
    inst = make_instance("greedy_batch256_n50_k2e4", n_traj=6, T=(2_000, 30_000), K=3000)
    prob = api.DeviceProblem.from_instance(inst)
    _say("case noalloc batch of 6, multi-unit, B=512")
    _same(api, prob, "greedy", 512)
    tiny = random_tiny(41, N=7, K=3, R=4, T=300, qmax=3, inv_max=8, n_traj=2)
    tprob = api.DeviceProblem.from_instance(tiny)
    part = torch.from_numpy(
        np.random.default_rng(3).integers(0, 9, tiny.total_orders).astype(np.int32)).cuda()
    _say("case noalloc tiny, random partition over 9 processes")
    _same(api, tprob, "greedy", 0, partition=part)


def test_learned_then_smaller(api):
    a = random_tiny(52, N=40, K=4, R=6, T=900, qmax=2, inv_max=30, n_traj=3, mlp=True)
    b = random_tiny(53, N=9, K=2, R=3, T=100, qmax=1, inv_max=6, n_traj=1, mlp=True)
    for inst, B in ((a, 16), (b, 4)):
        _say(f"case noalloc learned N={inst.N} T={inst.total_orders} B={B}")
        _same(api, api.DeviceProblem.from_instance(inst), "mlp", B)


def test_rejections(api):
    """A problem whose scratch exceeds the static buffer, and timing, are refused on the
    host (nothing is launched)."""
    T = 4_000_000
    z = torch.zeros(T, dtype=torch.int32, device="cuda")
    one = torch.ones(T, dtype=torch.int32, device="cuda")
    x0 = torch.ones((1, 4, 8), dtype=torch.int32, device="cuda")
    cost = torch.ones((1, 8, 2), dtype=torch.int32, device="cuda")
    offs = np.array([0, T], dtype=np.int64)
    p = api.pk_problem(8, 4, 2, 1, offs.ctypes.data, z.data_ptr(), z.data_ptr(), one.data_ptr(),
                       x0.data_ptr(), cost.data_ptr(), 0)
    po = api.pk_policy(api.PK_POLICY_GREEDY, 0, 0, 0, None)
    o = api.pk_picard_opts(1024, 0, 1, 0, None, 0, None)
    acts = torch.empty(T, dtype=torch.int32, device="cuda")
    _say("case noalloc rejects a problem larger than the static scratch")
    st = api.lib().pk_picard_simulate_noalloc(C.byref(p), C.byref(po), C.byref(o),
                                              acts.data_ptr(), None, None, None, None)
    assert st == api.PK_ERR_WORKSPACE
    assert b"static buffer" in api.lib().pk_last_error()
    small = np.array([0, 10], dtype=np.int64)
    p.traj_offsets = small.ctypes.data
    stats = api.pk_stats()
    stats.timing = 1
    st = api.lib().pk_picard_simulate_noalloc(C.byref(p), C.byref(po), C.byref(o),
                                              acts.data_ptr(), None, None, C.byref(stats), None)
    assert st == api.PK_ERR_UNSUPPORTED
    torch.cuda.synchronize()
