"""Learned-policy and gradient parity at the full sizes of the two learned workloads.

The GPU scores in FP32 and the oracle in FP64, so an action may differ from the FP64
policy only where the top two perturbed scores are within 1e-5 relative (a near-tie).

* 64 trajectories x 2e5 orders, N = 100, K = 5e4 (the whole batch): Picard equals the GPU
  serial sweep bit for bit on every trajectory; on two whole trajectories the FP64 policy
  at every state the GPU actions induce picks the GPU's action except at near-ties; the
  final inventory of every trajectory is x0 less the units the actions ship.
* The REINFORCE gradient over one whole 2e5-order trajectory at fixed actions (the
  oracle's greedy rollout, so no input comes from the GPU) and the oracle's advantages:
  within 1e-4 per parameter tensor of the FP64 oracle.
* 16 trajectories x 1e7 orders, N = 500, K = 1e6 (the whole horizon): Picard equals the
  GPU serial sweep bit for bit on the first 3e5 orders of every trajectory; on 1e5 steps
  sampled uniformly from all 1.6e8 the FP64 policy at the GPU-induced state picks the
  GPU's action except at near-ties; units shipped and the final inventory of sampled SKUs
  agree with the actions.
"""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import make_instance

pytestmark = pytest.mark.gpu
TIE = 1e-5
TOL = 1e-4
REV = 200
THREADS = max(1, min(16, os.cpu_count() or 1))


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


def _near(z1, z2):
    with np.errstate(invalid="ignore"):
        rel = (z1 - z2) / np.maximum(np.abs(z1), np.abs(z2))
    return np.isfinite(z2) & (rel <= TIE)


def _final_from_actions(x0_rows, keys, w, q, N):
    """max(0, x0 - units sent per warehouse) for the SKU rows x0_rows (the clamp composes
    the per-order shipments min(q, x))."""
    sent = np.zeros(x0_rows.shape, np.int64)
    np.add.at(sent, (keys, w), q)
    return np.maximum(0, x0_rows.astype(np.int64) - sent)


def test_learned_batch64_full(api, oracle):
    inst = make_instance("mlp_batch64_n100_k5e4_t2e5")
    prob = api.DeviceProblem.from_instance(inst)
    _say(f"case mlp full 64 x 2e5, N={inst.N}, K={inst.K}")
    out = api.pk_picard_simulate(prob, "mlp", block_len=256)
    ser = api.pk_serial_simulate(prob, "mlp")
    for k in ("actions", "shipped", "final_inv"):
        assert torch.equal(out[k], ser[k]), k
    acts = out["actions"].cpu().numpy()
    ship = out["shipped"].cpu().numpy()
    fin = out["final_inv"].cpu().numpy()
    _say(f"  passes max {int(out['passes'].max())}, GPU near-ties (all passes) "
         f"{out['stats']['near_ties']}")
    # shipped = min(q, stock) > 0 for a warehouse choice, 0 for a lost sale
    assert ((ship >= 0) & (ship <= inst.qty)).all()
    assert ((ship > 0) == (acts >= 0)).all()
    for b in range(inst.n_traj):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        a, s = acts[lo:hi], inst.sku[lo:hi]
        m = a >= 0
        want = _final_from_actions(inst.x0[b], s[m], a[m], inst.qty[lo:hi][m], inst.N)
        np.testing.assert_array_equal(fin[b], want)
    total_mism = total_ties = 0
    for b in (0, inst.n_traj - 1):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        ev = oracle.eval_at(inst, acts[lo:hi], b, threads=THREADS)
        near = _near(ev["z1"], ev["z2"])
        mism = ev["choice"] != acts[lo:hi]
        bad = mism & ~near
        _say(f"  trajectory {b}: {hi - lo} steps, FP64 near-ties {int(near.sum())}, "
             f"mismatches {int(mism.sum())} (all at near-ties: {not bad.any()})")
        assert not bad.any(), f"traj {b}: {int(bad.sum())} mismatches away from near-ties"
        total_mism += int(mism.sum())
        total_ties += int(near.sum())
    assert total_mism <= total_ties


def test_gradient_full_trajectory(api, oracle):
    inst = make_instance("mlp_batch64_n100_k5e4_t2e5").trajectory(0)
    _say(f"case grad full trajectory T={inst.total_orders}")
    g = oracle.serial(inst, 0, greedy=True)  # feasible fixed actions, from the oracle
    adv = oracle.advantages(inst, g["actions"], g["shipped"], REV)["advantages"]
    prob = api.DeviceProblem.from_instance(inst)
    res = api.pk_policy_grad(prob, torch.from_numpy(g["actions"]).cuda(),
                             torch.from_numpy(adv).cuda())
    ref = oracle.reinforce(inst, g["actions"], adv.astype(np.float64), 0, threads=THREADS)
    got = res["grad"].cpu().numpy().astype(np.float64)
    want = ref["grad"]
    H, R = 64, inst.R
    o = 0
    scale = np.abs(want).max()
    for name, n in (("E", R * 16), ("W1", H * 18), ("b1", H), ("W2", H * H), ("b2", H),
                    ("w3", H), ("b3", 1)):
        gp, wp = got[o:o + n], want[o:o + n]
        o += n
        if name == "b3":
            assert abs(gp[0] - wp[0]) <= TOL * scale, (gp, wp)
            continue
        err = np.linalg.norm(gp - wp) / max(np.linalg.norm(wp), 1e-30)
        _say(f"  {name}: relative error {err:.2e}")
        assert err <= TOL, (name, err)
    assert o == got.size
    lp = res["logp"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(lp, ref["logp"], rtol=1e-4, atol=1e-4)
    assert abs(res["objective"] - ref["objective"]) <= 1e-4 * (1 + abs(ref["objective"]))


def _states_at(acts_b, sku_b, qty_b, x0_b, ts, ks, N):
    """Inventory rows of SKUs ks just before time ts (time indices within the trajectory;
    ts = T gives the final inventory), from the actions alone: x0 less the quantities of
    the SKU's earlier orders sent to each warehouse, clamped at zero (min(q, x) shipments
    compose to that clamp).  Plain torch on the GPU: orders with a warehouse action sorted
    by (SKU, warehouse, time), prefix sums of their quantities, two binary searches per
    (state, warehouse)."""
    dev = acts_b.device
    m = acts_b >= 0
    t_all = torch.arange(acts_b.numel(), device=dev, dtype=torch.int64)
    key = (sku_b[m].long() * N + acts_b[m].long()) * (1 << 24) + t_all[m]
    key, order = torch.sort(key)
    cq = torch.zeros(key.numel() + 1, dtype=torch.int64, device=dev)
    cq[1:] = torch.cumsum(qty_b[m].long()[order], 0)
    ts = torch.as_tensor(ts, device=dev, dtype=torch.int64)
    k = torch.as_tensor(ks, device=dev, dtype=torch.int64)
    w = torch.arange(N, device=dev, dtype=torch.int64)
    base = (k[:, None] * N + w[None, :]) * (1 << 24)
    lo = torch.searchsorted(key, base)
    hi = torch.searchsorted(key, base + ts[:, None])
    sent = cq[hi] - cq[lo]
    x = torch.clamp(x0_b[k].long() - sent, min=0)
    return x.to(torch.int32)


def test_learned_large_full_horizon(api, oracle):
    inst = make_instance("mlp_batch16_n500_k1e6_t1e7")
    N = inst.N
    _say(f"case mlp full horizon 16 x 1e7, N={N}, K={inst.K}: {inst.total_orders} orders")
    prob = api.DeviceProblem.from_instance(inst)
    out = api.pk_picard_simulate(prob, "mlp", block_len=256)
    torch.cuda.synchronize()
    _say(f"  Picard: passes max {int(out['passes'].max())}, mean "
         f"{float(out['passes'].mean()):.1f}; GPU near-ties (all passes) "
         f"{out['stats']['near_ties']}")
    acts_d, ship_d = out["actions"], out["shipped"]
    # the serial sweep on the first 3e5 orders of every trajectory (its rollout is the
    # prefix of the whole rollout)
    M = 300_000
    offs = inst.traj_offsets
    idx = np.concatenate([np.arange(offs[b], offs[b] + M) for b in range(inst.n_traj)])
    new = np.arange(inst.n_traj + 1, dtype=np.int64) * M
    it = torch.from_numpy(idx).cuda()
    sub = api.DeviceProblem(N=prob.N, K=prob.K, R=prob.R, traj_offsets=new,
                            sku=prob.sku[it].contiguous(), region=prob.region[it].contiguous(),
                            qty=prob.qty[it].contiguous(), init_inv=prob.init_inv,
                            cost=prob.cost, rng_seed=prob.rng_seed, params=prob.params,
                            n_hidden_layers=prob.n_hidden_layers, hidden=prob.hidden)
    ser = api.pk_serial_simulate(sub, "mlp", want_final=False)
    assert torch.equal(ser["actions"], acts_d[it])
    assert torch.equal(ser["shipped"], ship_d[it])
    _say(f"  serial sweep equal on the first {M} orders of each trajectory")
    del ser, sub, it
    # shipped = min(q, stock) > 0 for a warehouse choice, 0 for a lost sale
    q_d = prob.qty
    assert bool(((ship_d >= 0) & (ship_d <= q_d)).all())
    assert bool(((ship_d > 0) == (acts_d >= 0)).all())
    # 1e5 steps sampled uniformly from the whole batch
    rng = np.random.default_rng(2024)
    samples = np.sort(rng.choice(inst.total_orders, 100_000, replace=False))
    traj_of = np.searchsorted(offs, samples, side="right") - 1
    mism = ties = checked_rows = 0
    for b in range(inst.n_traj):
        lo, hi = int(offs[b]), int(offs[b + 1])
        ts = samples[traj_of == b] - lo
        if ts.size == 0:
            continue
        x = _states_at(acts_d[lo:hi], prob.sku[lo:hi], q_d[lo:hi], prob.init_inv[b],
                       ts, inst.sku[lo + ts], N).cpu().numpy()
        checked_rows += int((x > 0).sum())
        ev = oracle.policy_at(inst, b, ts, x, threads=THREADS)
        gpu = acts_d[lo:hi][torch.from_numpy(ts).cuda()].cpu().numpy()
        near = _near(ev["z1"], ev["z2"])
        miss = ev["choice"] != gpu
        bad = miss & ~near
        assert not bad.any(), (b, ts[bad][:5], gpu[bad][:5], ev["choice"][bad][:5])
        mism += int(miss.sum())
        ties += int(near.sum())
        # the final inventory of the sampled SKUs follows from the actions too
        if b in (0, inst.n_traj - 1):
            ks = np.unique(inst.sku[lo + ts[:200]])
            fin = out["final_inv"][b][torch.from_numpy(ks).cuda()].cpu().numpy()
            ends = _states_at(acts_d[lo:hi], prob.sku[lo:hi], q_d[lo:hi], prob.init_inv[b],
                              np.full(ks.size, hi - lo), ks, N).cpu().numpy()
            np.testing.assert_array_equal(fin, ends)
    _say(f"  {samples.size} sampled steps ({checked_rows} scored rows): FP64 near-ties "
         f"{ties}, mismatches {mism} (all at near-ties)")
    assert mism <= ties
