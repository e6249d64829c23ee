"""Pins of the oracle's learned policy, its noise and its REINFORCE gradient.

* Scores: a PyTorch float64 forward of the same two-layer ReLU MLP (library cross-check).
* Serial learned rollout: an independent numpy float64 rollout.
* Gumbel-max: argmax_w (s_w + G_w) is distributed as softmax(s) over the feasible set;
  checked with a chi-square test of the oracle's noise.
* Philox4x32-10 (SC'11): bitwise equal to rocRAND's host-callable engine.
* REINFORCE: central finite differences of the oracle's own FP64 objective, torch
  float64 autograd of the same surrogate, and closed forms (softmax shift invariance
  makes dL/db3 = 0; a step with one feasible warehouse contributes nothing).
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import random_tiny, make_params, EMB_DIM


def _unpack(params, R, H=64, L=2):
    p = params.astype(np.float64)
    o = 0
    E = p[o:o + R * EMB_DIM].reshape(R, EMB_DIM); o += R * EMB_DIM
    W1 = p[o:o + H * 18].reshape(H, 18); o += H * 18
    b1 = p[o:o + H]; o += H
    W2 = b2 = None
    if L == 2:
        W2 = p[o:o + H * H].reshape(H, H); o += H * H
        b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return E, W1, b1, W2, b2, w3, b3


def _torch_scores(params, R, cost_col, x_row, r, L=2):
    E, W1, b1, W2, b2, w3, b3 = [None if a is None else torch.as_tensor(a)
                                 for a in _unpack(params, R, L=L)]
    N = x_row.size
    f = torch.cat([torch.as_tensor(cost_col, dtype=torch.float64)[:, None],
                   torch.log1p(torch.as_tensor(x_row, dtype=torch.float64))[:, None],
                   E[r][None, :].expand(N, EMB_DIM)], dim=1)
    h = torch.relu(torch.nn.functional.linear(f, W1, b1))
    if L == 2:
        h = torch.relu(torch.nn.functional.linear(h, W2, b2))
    return (h @ w3 + b3).numpy()


@pytest.mark.parametrize("L", [1, 2])
def test_scores_match_torch(oracle, L):
    inst = random_tiny(4, N=9, K=2, R=5, mlp=True, n_hidden_layers=L)
    rng = np.random.default_rng(0)
    for r in range(inst.R):
        x = rng.integers(0, 50, inst.N).astype(np.int32)
        got = oracle.mlp_scores(inst, r, x)
        want = _torch_scores(inst.params, inst.R, inst.cost[0, :, r], x, r, L=L)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def _numpy_learned_serial(oracle, inst):
    E, W1, b1, W2, b2, w3, b3 = _unpack(inst.params, inst.R, L=inst.n_hidden_layers)
    x = inst.x0[0].astype(np.int64).copy()
    acts, z1s, z2s = [], [], []
    for t in range(inst.total_orders):
        k, r, q = inst.sku[t], inst.region[t], inst.qty[t]
        feas = np.nonzero(x[k] > 0)[0]
        if feas.size == 0:
            acts.append(-1); z1s.append(-np.inf); z2s.append(-np.inf); continue
        f = np.stack([inst.cost[0, feas, r].astype(np.float64), np.log1p(x[k, feas]),
                      *[np.full(feas.size, E[r, i]) for i in range(EMB_DIM)]], axis=1)
        h = np.maximum(f @ W1.T + b1, 0.0)
        if W2 is not None:
            h = np.maximum(h @ W2.T + b2, 0.0)
        s = h @ w3 + b3
        g = np.array([oracle.gumbel(inst.rng_seed, 0, t, int(w)) for w in feas])
        z = s + g
        i = int(np.argmax(z))  # first maximum: lowest index on exact ties
        a = int(feas[i])
        acts.append(a); z1s.append(z[i])
        z2s.append(np.sort(z)[-2] if z.size > 1 else -np.inf)
        x[k, a] -= min(q, x[k, a])
    return np.array(acts), np.array(z1s), np.array(z2s)


@pytest.mark.parametrize("seed", range(6))
def test_learned_serial_matches_numpy(oracle, seed):
    inst = random_tiny(seed + 40, N=6, K=3, R=4, T=80, qmax=2, inv_max=5, mlp=True,
                       n_hidden_layers=1 + seed % 2)
    r = oracle.serial(inst)
    a, z1, z2 = _numpy_learned_serial(oracle, inst)
    np.testing.assert_array_equal(r["actions"], a)
    m = a >= 0
    np.testing.assert_allclose(r["z1"][m], z1[m], rtol=1e-12, atol=1e-12)
    # the runner-up score (the near-tie margin z1 - z2 is what parity tests key on)
    np.testing.assert_array_equal(np.isinf(r["z2"]), np.isinf(z2))
    f = np.isfinite(z2)
    np.testing.assert_allclose(r["z2"][f], z2[f], rtol=1e-12, atol=1e-12)


def test_uniform_is_binary32_exact_and_uniform(oracle):
    us = np.array([oracle.uniform(12345, 3, t, w) for t in range(2000) for w in range(4)])
    assert ((us > 0) & (us < 1)).all()
    np.testing.assert_array_equal(us, us.astype(np.float32).astype(np.float64))
    # each value is the centre of one of 2^23 equal bins, so U and 1 - U are equally
    # likely and neither 0 nor 1 can occur
    np.testing.assert_array_equal(np.modf(us * 2.0**23)[0], 0.5)
    from scipy import stats
    assert stats.kstest(us, "uniform").pvalue > 1e-3


def test_gumbel_max_is_softmax(oracle):
    """argmax(s + G) ~ softmax(s): chi-square over 40000 independent counters."""
    from scipy import stats
    s = np.array([0.3, -1.0, 1.2, 0.0, 0.8])
    M = 40000
    counts = np.zeros(s.size)
    for t in range(M):
        z = [s[w] + oracle.gumbel(99, 1, t, w) for w in range(s.size)]
        counts[int(np.argmax(z))] += 1
    p = np.exp(s - s.max()); p /= p.sum()
    chi2 = ((counts - M * p) ** 2 / (M * p)).sum()
    assert stats.chi2.sf(chi2, df=s.size - 1) > 1e-4


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned int c[4], k[2];
  while (scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
    unsigned long long offset = 4ull * (((unsigned long long)c[1] << 32) | c[0]);
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    uint4 v = e.next4();
    printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(oracle):
    """External cross-check: rocRAND's Philox4x32-10 engine, host side.  Its seed gives
    the key, the subsequence the high counter words and offset/4 the low ones."""
    rng = np.random.default_rng(5)
    # offset = 4 * (c1:c0) must fit 64 bits, so the second counter word stays < 2^30
    cases = [np.concatenate([rng.integers(0, 2**32, 1), rng.integers(0, 2**30, 1),
                             rng.integers(0, 2**32, 2), rng.integers(0, 2**32, 2)])
             for _ in range(64)]
    cases += [np.array([0, 0, 0, 0, 0, 0]),
              np.array([2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1])]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.check_call(["hipcc", "-O1", "-I/opt/rocm/include", src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                             check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        want = np.array([int(v) for v in line.split()], dtype=np.uint32)
        got = oracle.philox4x32_10(c[:4], c[4:])
        np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------- REINFORCE gradient
def _rollout_with_adv(oracle, inst, seed=0):
    ser = oracle.serial(inst)
    adv = np.random.default_rng(seed).standard_normal(inst.total_orders)
    return ser["actions"], adv


def _objective(oracle, inst, params, actions, adv):
    old = inst.params
    inst.params = params.astype(np.float32)
    try:
        return oracle.reinforce(inst, actions, adv, want_grad=False)["objective"]
    finally:
        inst.params = old


@pytest.mark.parametrize("L", [1, 2])
def test_reinforce_finite_differences(oracle, L):
    """Directional central differences with Richardson extrapolation (steps h and 2h,
    h = 2^-16).  The parameters are float32 on input, so each stencil point is rounded
    to float32 and the directional derivative is compared along the direction actually
    taken.  Directions whose stencil crosses a ReLU kink (the two step sizes disagree)
    are skipped."""
    inst = random_tiny(61, N=5, K=2, R=3, T=40, qmax=2, inv_max=6, mlp=True,
                       n_hidden_layers=L)
    actions, adv = _rollout_with_adv(oracle, inst)
    g = oracle.reinforce(inst, actions, adv)["grad"]
    p0 = inst.params.astype(np.float64)
    rng = np.random.default_rng(1)
    h = 2.0 ** -16
    checked = 0
    for trial in range(40):
        if trial < 20:
            v = np.zeros_like(p0)
            v[rng.integers(0, p0.size)] = 1.0
        else:
            v = np.sign(rng.standard_normal(p0.size))
        pts = {c: (p0 + c * h * v).astype(np.float32).astype(np.float64) for c in (-2, -1, 1, 2)}
        f = {c: _objective(oracle, inst, pts[c], actions, adv) for c in pts}
        d1 = (f[1] - f[-1]) / (2 * h)
        d2 = (f[2] - f[-2]) / (4 * h)
        if abs(d1 - d2) > 1e-6 * (abs(d1) + 1e-3):
            continue  # kink inside the stencil
        rich = (4 * d1 - d2) / 3
        v1 = (pts[1] - pts[-1]) / (2 * h)
        v2 = (pts[2] - pts[-2]) / (4 * h)
        want = float(g @ ((4 * v1 - v2) / 3))
        assert abs(rich - want) <= 1e-6 * (1 + abs(want)), (trial, rich, want)
        checked += 1
    assert checked >= 25


def test_reinforce_matches_torch_autograd(oracle):
    inst = random_tiny(62, N=6, K=3, R=4, T=50, qmax=3, inv_max=5, mlp=True)
    actions, adv = _rollout_with_adv(oracle, inst, 3)
    res = oracle.reinforce(inst, actions, adv)
    p = torch.tensor(inst.params.astype(np.float64), requires_grad=True)
    R, H = inst.R, 64
    o = 0
    E = p[o:o + R * 16].view(R, 16); o += R * 16
    W1 = p[o:o + H * 18].view(H, 18); o += H * 18
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].view(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    x = inst.x0[0].astype(np.int64).copy()
    total = torch.zeros((), dtype=torch.float64)
    for t in range(inst.total_orders):
        k, r, q, a = inst.sku[t], inst.region[t], inst.qty[t], actions[t]
        feas = np.nonzero(x[k] > 0)[0]
        if feas.size:
            f = torch.cat([torch.tensor(inst.cost[0, feas, r], dtype=torch.float64)[:, None],
                           torch.log1p(torch.tensor(x[k, feas], dtype=torch.float64))[:, None],
                           E[r][None, :].expand(feas.size, 16)], dim=1)
            h = torch.relu(f @ W1.T + b1)
            h = torch.relu(h @ W2.T + b2)
            s = h @ w3 + b3
            lp = s[int(np.nonzero(feas == a)[0][0])] - torch.logsumexp(s, 0)
            total = total + float(adv[t]) * lp
        if a >= 0:
            x[k, a] -= min(q, x[k, a])
    total.backward()
    assert abs(total.item() - res["objective"]) < 1e-10 * (1 + abs(total.item()))
    np.testing.assert_allclose(res["grad"], p.grad.numpy(), rtol=1e-9, atol=1e-10)


def test_reinforce_closed_forms(oracle):
    inst = random_tiny(63, N=5, K=2, R=3, T=60, qmax=2, inv_max=4, mlp=True)
    actions, adv = _rollout_with_adv(oracle, inst, 4)
    res = oracle.reinforce(inst, actions, adv)
    g = res["grad"]
    assert abs(g[-1]) < 1e-10 * (1 + np.abs(g).max())  # dL/db3 = 0 (shift invariance)
    ev = oracle.eval_at(inst, actions)
    single = ev["n_feasible"] <= 1
    assert single.any()
    np.testing.assert_array_equal(res["logp"][single], 0.0)
    # Zeroing the advantage of every step with <= 1 feasible warehouse changes nothing.
    adv2 = adv.copy()
    adv2[single] = 0.0
    np.testing.assert_array_equal(oracle.reinforce(inst, actions, adv2)["grad"], g)
    assert (res["logp"] <= 0).all()


def test_reinforce_rejects_infeasible_action(oracle):
    inst = random_tiny(64, N=4, K=1, R=2, T=10, inv_max=2, mlp=True)
    actions, adv = _rollout_with_adv(oracle, inst)
    bad = actions.copy()
    ev = oracle.eval_at(inst, actions)
    t = int(np.nonzero(ev["n_feasible"] > 0)[0][0])
    bad[t] = -1
    with pytest.raises(ValueError):
        oracle.reinforce(inst, bad, adv)


# ---------------------------------------------------------------- windows and given states
def test_windows_equal_whole_horizon(oracle):
    """eval_at and reinforce over disjoint windows of steps (run in threads; each window
    replays the given actions up to its start) equal one pass over the whole horizon:
    the same choices and scores bit for bit, and the gradient and objective to FP64
    rounding of the regrouped sum."""
    inst = random_tiny(65, N=7, K=3, R=4, T=400, qmax=3, inv_max=9, mlp=True)
    actions, adv = _rollout_with_adv(oracle, inst, 5)
    whole = oracle.eval_at(inst, actions)
    win = oracle.eval_at(inst, actions, threads=3)
    for k in whole:
        np.testing.assert_array_equal(win[k], whole[k])
    r1 = oracle.reinforce(inst, actions, adv)
    r2 = oracle.reinforce(inst, actions, adv, threads=3)
    np.testing.assert_array_equal(r2["logp"], r1["logp"])
    np.testing.assert_allclose(r2["grad"], r1["grad"], rtol=1e-12,
                               atol=1e-12 * np.abs(r1["grad"]).max())
    assert abs(r2["objective"] - r1["objective"]) <= 1e-12 * (1 + abs(r1["objective"]))


def test_policy_at_states_of_a_replay(oracle):
    """The policy at given states (the order's SKU row before each step, from a plain
    Python replay of the serial actions) gives eval_at's choice and top two scores at
    every step, and the serial rollout's action."""
    inst = random_tiny(66, N=6, K=3, R=4, T=150, qmax=2, inv_max=6, mlp=True)
    ser = oracle.serial(inst)
    x = inst.x0[0].astype(np.int64).copy()
    rows = np.empty((inst.total_orders, inst.N), np.int32)
    for t in range(inst.total_orders):
        k, a = inst.sku[t], ser["actions"][t]
        rows[t] = x[k]
        if a >= 0:
            x[k, a] -= min(inst.qty[t], x[k, a])
    ts = np.arange(inst.total_orders)
    perm = np.random.default_rng(2).permutation(ts.size)  # any order of the states
    got = oracle.policy_at(inst, 0, ts[perm], rows[perm], threads=2)
    ev = oracle.eval_at(inst, ser["actions"])
    np.testing.assert_array_equal(got["choice"], ev["choice"][perm])
    np.testing.assert_array_equal(got["choice"], ser["actions"][perm])
    np.testing.assert_array_equal(got["z1"], ev["z1"][perm])
    np.testing.assert_array_equal(got["z2"], ev["z2"][perm])
