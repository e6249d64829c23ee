"""The autotuner: block length for both policies (and the learned walk's waves per
workgroup), cached in the process and written to the results file named by
$PICARD_AUTOTUNE_CACHE; a simulation that asks for the tuned choice (block_len 0) uses it,
and every candidate gives the same actions."""
import json
import os
import sys
import time

import numpy as np
import pytest
import torch

from paper_2406_01939_amd.instances import make_instance

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


@pytest.mark.parametrize("policy", ["greedy", "mlp"])
def test_autotune_cached_and_used(api, tmp_path, monkeypatch, policy):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PICARD_AUTOTUNE_CACHE", str(path))  # results written here
    # shapes of their own (no recorded result): 3 trajectories of 30000 orders
    if policy == "greedy":
        inst = make_instance("greedy_batch256_n50_k2e4", n_traj=3, T=(29_000, 31_000), K=1237)
    else:
        inst = make_instance("mlp_batch64_n100_k5e4_t2e5", n_traj=3, T=30_000, K=1237)
    prob = api.DeviceProblem.from_instance(inst)
    _say(f"case autotune {policy}: {inst.total_orders} orders")
    t0 = time.perf_counter()
    B = api.pk_autotune(prob, policy)
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    B2 = api.pk_autotune(prob, policy)
    t_again = time.perf_counter() - t0
    _say(f"  tuned block_len {B} in {t_first:.2f} s; cached lookup {t_again * 1e3:.2f} ms")
    assert B2 == B and B >= 64
    assert t_again < 0.05 and t_again < t_first / 10
    rec = json.load(open(path))
    (key, val), = [(k, v) for k, v in rec.items()
                   if k.startswith(policy + "/") and "/K1237/" in k]
    assert val["block_len"] == B and val["waves"] in (4, 8)
    _say(f"  recorded {key}: {val}")
    out = api.pk_picard_simulate(prob, policy)  # block_len 0: the tuned choice
    assert out["stats"]["block_len"] == B
    ser = api.pk_serial_simulate(prob, policy)
    assert torch.equal(out["actions"], ser["actions"])
    for b2, w2 in ((B // 2 if B >= 128 else B * 2, 4), (B, 8)):
        alt = api.pk_picard_simulate(prob, policy, block_len=b2, walk_waves=w2)
        assert torch.equal(alt["actions"], ser["actions"]), (b2, w2)


def test_walk_waves_rejected(api):
    inst = make_instance("mlp_batch64_n100_k5e4_t2e5", n_traj=1, T=500, K=50)
    prob = api.DeviceProblem.from_instance(inst)
    with pytest.raises(api.PicardError) as e:
        api.pk_picard_simulate(prob, "mlp", block_len=64, walk_waves=6)
    assert e.value.status == api.PK_ERR_INVALID_ARG
