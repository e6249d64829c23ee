"""GPU parity of the policy-gradient pieces (Section 4.2) against the CPU oracle.

Advantages: bit-exact (the sums are exact int64 and the one rounding is the same double
expression on both sides) on the oracle's own rollouts, over batches whose trajectories
straddle the kernel's 2048-order tiles, with an empty trajectory, partial shipments
(q > 1) and learned-policy rollouts; host-forced errors for an out-of-range action and
for rewards past the exact-sum bound.  Adam: against the oracle's float64 step within
float32 rounding.  The training loop: the warm-started Picard, cold Picard and serial
rollouts give the same parameters bit for bit after several iterations (every rollout
equals the serial one, Proposition 2.1); at unchanged parameters a warm start returns
after one pass; one iteration equals the oracle's iteration within the gradient's
tolerance.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import make_instance, random_tiny

pytestmark = pytest.mark.gpu
REV = 200


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


def _oracle_batch(oracle, inst, revenue, greedy):
    acts, ship, adv, ret = [], [], [], []
    for b in range(inst.n_traj):
        s = oracle.serial(inst, b, greedy=greedy)
        o = oracle.advantages(inst, s["actions"], s["shipped"], revenue, b)
        acts.append(s["actions"])
        ship.append(s["shipped"])
        adv.append(o["advantages"])
        ret.append(o["ret"])
    return (np.concatenate(acts), np.concatenate(ship), np.concatenate(adv),
            np.array(ret, np.int64))


def _with_empty_trajectory(inst):
    """The same batch with an empty trajectory inserted after the first one."""
    offs = inst.traj_offsets
    new_offs = np.concatenate([offs[:2], offs[1:]]).astype(np.int64)
    pick = np.concatenate([[0, 0], np.arange(1, inst.n_traj)])
    return dataclasses.replace(inst, traj_offsets=new_offs, x0=inst.x0[pick],
                               cost=inst.cost[pick])


def _check_adv(api, oracle, inst, revenue=REV, greedy=True):
    acts, ship, want_adv, want_ret = _oracle_batch(oracle, inst, revenue, greedy)
    prob = api.DeviceProblem.from_instance(inst)
    got = api.pk_reinforce_advantages(prob, torch.from_numpy(acts).cuda(),
                                      torch.from_numpy(ship).cuda(), revenue)
    np.testing.assert_array_equal(got["advantages"].cpu().numpy(), want_adv)
    np.testing.assert_array_equal(got["returns"].cpu().numpy(), want_ret)


@pytest.mark.parametrize("seed", range(3))
def test_advantages_tiny(api, oracle, seed):
    inst = random_tiny(700 + seed, N=5, K=3, R=4, T=90, qmax=3, inv_max=6, n_traj=3)
    _say(f"case advantages tiny seed={seed}")
    _check_adv(api, oracle, inst, revenue=4)  # negative margins too (cost in 1..5)


def test_advantages_tiles_and_empty_trajectory(api, oracle):
    inst = make_instance("greedy_batch256_n50_k2e4", T=(1500, 5000), n_traj=5, K=500)
    _say("case advantages batch of 5 across tiles")
    _check_adv(api, oracle, inst)
    _say("case advantages with an empty trajectory")
    _check_adv(api, oracle, _with_empty_trajectory(inst))


def test_advantages_learned_rollout(api, oracle):
    inst = random_tiny(710, N=9, K=3, R=4, T=400, qmax=2, inv_max=9, n_traj=2, mlp=True)
    _say("case advantages of a learned-policy rollout")
    _check_adv(api, oracle, inst, greedy=False)


def test_advantages_full_horizon(api, oracle):
    inst = make_instance("greedy_n100_k1e5_t1e6")
    _say("case advantages N=100 K=1e5 T=1e6")
    _check_adv(api, oracle, inst)


def test_advantages_errors(api, oracle):
    inst = random_tiny(720, N=4, K=3, R=3, T=100_000, qmax=1, inv_max=3)
    acts, ship, _, _ = _oracle_batch(oracle, inst, REV, True)
    assert (ship > 0).any()
    prob = api.DeviceProblem.from_instance(inst)
    a, s = torch.from_numpy(acts).cuda(), torch.from_numpy(ship).cuda()
    _say("case advantages: reward beyond the exact-sum bound")
    # T = 1e5 bounds |r| by 2^62 / (T (T + 1) / 2), about 9.2e8; a 2e9 margin exceeds it
    with pytest.raises(api.PicardError) as e:
        api.pk_reinforce_advantages(prob, a, s, 2_000_000_000)
    assert e.value.status == api.PK_ERR_INVALID_ARG and "exceeds" in str(e.value)
    _say("case advantages: action out of range")
    bad = a.clone()
    bad[7] = inst.N
    with pytest.raises(api.PicardError) as e:
        api.pk_reinforce_advantages(prob, bad, s, REV)
    assert e.value.status == api.PK_ERR_INVALID_ARG
    _say("case advantages: valid call after the errors")
    api.pk_reinforce_advantages(prob, a, s, REV)


@pytest.mark.parametrize("ascend", [True, False])
def test_adam_matches_oracle(api, oracle, ascend):
    rng = np.random.default_rng(11)
    n, lr, steps = 5441 + 16 * 200, 3e-3, 4
    theta = rng.standard_normal(n).astype(np.float32)
    grads = [(rng.standard_normal(n) * 10.0 ** rng.integers(-3, 2, n)).astype(np.float32)
             for _ in range(steps)]
    grads[1][:100] = 0.0
    p = torch.from_numpy(theta.copy()).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    th, mo, vo = theta.astype(np.float64), np.zeros(n), np.zeros(n)
    sm = np.zeros(n)  # size of the terms of m: the same recursion on |g|
    _say(f"case adam ascend={ascend}")
    for k, g in enumerate(grads, start=1):
        api.pk_adam_step(p, torch.from_numpy(g).cuda(), m, v, k, lr, ascend=ascend)
        th, mo, vo = oracle.adam_step(th, g.astype(np.float64), mo, vo, k, lr, ascend=ascend)
        sm = 0.9 * sm + 0.1 * np.abs(g.astype(np.float64))
        # float32 rounding: a few ulps of the move (size <= lr) per step, plus the
        # rounding of theta itself at every step
        tol = k * (1e-6 * lr + 2.0**-23 * np.abs(th))
        err = np.abs(p.cpu().numpy().astype(np.float64) - th)
        assert (err <= tol).all(), (k, float((err - tol).max()))
        # m: terms of both signs may cancel, so its error is a few ulps of their size;
        # v: all terms are >= 0, a few ulps of v itself
        em = np.abs(m.cpu().numpy().astype(np.float64) - mo)
        assert (em <= k * 2.0**-21 * sm).all(), (k, float((em / np.maximum(sm, 1e-300)).max()))
        np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=1e-6 * k, atol=1e-30)


def test_training_loop_rollout_modes_agree(api):
    from paper_2406_01939_amd.train import PolicyGradient
    inst = make_instance("mlp_batch64_n100_k5e4_t2e5", n_traj=3, T=4000, K=800)
    runs = {}
    for mode, warm in (("picard", True), ("picard", False), ("serial", False)):
        prob = api.DeviceProblem.from_instance(inst)
        pg = PolicyGradient(prob, lr=3e-3, revenue=REV, rollout=mode, warm_start=warm,
                            block_len=256)
        _say(f"case training loop rollout={mode} warm={warm}")
        hist = pg.run(4)
        runs[(mode, warm)] = (prob.params.clone(), pg.out["actions"].clone(), hist)
        _say("  passes per iteration", [h.passes_max for h in hist])
    ref_p, ref_a, _ = runs[("serial", False)]
    for key in (("picard", True), ("picard", False)):
        p, a, hist = runs[key]
        assert torch.equal(p, ref_p), key
        assert torch.equal(a, ref_a), key
    warm_hist = runs[("picard", True)][2]
    cold_hist = runs[("picard", False)][2]
    assert warm_hist[0].passes_max == cold_hist[0].passes_max  # both start cold
    assert not torch.equal(ref_p, api.DeviceProblem.from_instance(inst).params)


def test_warm_start_at_unchanged_parameters_takes_one_pass(api):
    """With lr = 0 the policy does not change, so the previous iterate's actions are the
    fixed point and the warm-started rollout returns after its first pass."""
    from paper_2406_01939_amd.train import PolicyGradient
    inst = make_instance("mlp_batch64_n100_k5e4_t2e5", n_traj=2, T=3000, K=600)
    prob = api.DeviceProblem.from_instance(inst)
    pg = PolicyGradient(prob, lr=0.0, revenue=REV, rollout="picard", block_len=128)
    _say("case warm start at unchanged parameters")
    h1 = pg.step()
    a1 = pg.out["actions"].clone()
    h2 = pg.step()
    assert h1.passes_max > 1 and h2.passes_max == 1
    assert torch.equal(pg.out["actions"], a1)


def test_training_iteration_matches_oracle(api, oracle):
    """One iteration on the GPU equals the oracle's: serial rollout, advantages, FP64
    gradient, FP64 Adam step.  Both sides roll out the same policy; the GPU's FP32 scores
    may only flip near-ties, which this instance does not have."""
    from paper_2406_01939_amd.train import PolicyGradient
    inst = random_tiny(730, N=8, K=3, R=4, T=300, qmax=2, inv_max=8, n_traj=2, mlp=True)
    acts, ship, adv, _ = _oracle_batch(oracle, inst, REV, greedy=False)
    g64 = np.zeros(inst.params.size)
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        g64 += oracle.reinforce(inst, acts[lo:hi], adv[lo:hi].astype(np.float64), b)["grad"]
    lr = 3e-3
    th1, _, _ = oracle.adam_step(inst.params.astype(np.float64), g64, np.zeros_like(g64),
                                 np.zeros_like(g64), 1, lr)
    prob = api.DeviceProblem.from_instance(inst)
    pg = PolicyGradient(prob, lr=lr, revenue=REV, rollout="picard", block_len=16)
    _say("case one training iteration against the oracle")
    pg.step()
    np.testing.assert_array_equal(pg.out["actions"].cpu().numpy(), acts)
    got = prob.params.cpu().numpy().astype(np.float64)
    # the first Adam move is lr * g / (|g| + eps): within lr of the start wherever the
    # gradient is tiny, and lr * sign(g) to within the gradient's relative error elsewhere
    big = np.abs(g64) > 1e-2 * np.abs(g64).max()
    np.testing.assert_allclose(got[big], th1[big], rtol=0, atol=1e-6 + 2.0**-22 * np.abs(th1[big]).max())
    assert (np.abs(got - inst.params) <= lr * (1 + 1e-5) + 2.0**-22 * np.abs(inst.params)).all()
