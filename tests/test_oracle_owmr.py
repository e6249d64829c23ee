"""Pins of the OWMR inventory oracle (the appendix's inventory-control extension).

* Serial rollout: hand-worked cases (tests/golden/owmr_handworked.txt), an independent
  pure-Python rollout written from the model, and invariants (retailer stock within
  capacity, central stock never negative, R counts the resets, a ledger of the central
  stock: its initial stock plus what every reset added minus what the retailers received).
* Algorithm 1 (brute force, any assignment of steps to processes): the fixed point is the
  serial rollout from any initial cache (Proposition 2.1) within T + 1 passes.
* The per-process form (processes own whole retailers, two scans of the cache per pass)
  equals the brute force pass by pass.
* The appendix's theorem: when s >= every retailer capacity, processes by retailer and
  the first pass from an empty cache (no orders, no resets), the cache is the serial
  rollout after at most 2R + 1 passes (R resets; the one before the 2R is the pass that
  makes every retailer order exact, reading the theorem's count as starting there), so
  Algorithm 1 returns after at most 2R + 2.  With a central stock that never binds and
  never resets, retailers decouple and two passes suffice.
"""
import os

import numpy as np
import pytest

from paper_2406_01939_amd.instances import OwmrInstance, make_owmr_instance, random_owmr

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def owmr():
    from oracle import owmr as O
    O.build(force=False)
    return O


def _golden():
    cases, cur = [], None
    for line in open(os.path.join(HERE, "golden", "owmr_handworked.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        head, *rest = line.split()
        if head == "case":
            cur = {"name": rest[0]}
            cases.append(cur)
        elif "N" not in cur:
            cur["N"], cur["s0"], cur["S0"], cur["x0_init"] = map(int, [head] + rest)
        else:
            cur[head] = [int(v) for v in rest]
    return cases


def _inst(c):
    i32 = lambda k: np.array(c[k], dtype=np.int32)
    return OwmrInstance(N=c["N"], retailer=i32("retailer"), demand=i32("demand"),
                        s_ret=i32("s_ret"), S_ret=i32("S_ret"), cap=i32("cap"),
                        x_init=i32("x_init"), s0=c["s0"], S0=c["S0"], x0_init=c["x0_init"])


def _python_serial(inst):
    """The model written out in plain Python."""
    x = [int(v) for v in inst.x_init]
    x0 = int(inst.x0_init)
    qs, rs = [], []
    for n, d in zip(inst.retailer.tolist(), inst.demand.tolist()):
        p = max(0, x[n] - d)
        level = min(int(inst.S_ret[n]), int(inst.cap[n]))
        q = level - p if (p <= inst.s_ret[n] and level > p) else 0
        reset = int(x0 - q <= inst.s0)
        x[n] = p + min(q, x0)
        x0 = int(inst.S0) if reset else max(0, x0 - q)
        qs.append(q)
        rs.append(reset)
    return np.array(qs), np.array(rs), x0, np.array(x)


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_handworked(owmr, case):
    r = owmr.serial(_inst(case))
    np.testing.assert_array_equal(r["q"], case["q"])
    np.testing.assert_array_equal(r["reset"], case["reset"])
    assert r["final_x0"] == case["final_x0"][0]
    np.testing.assert_array_equal(r["final_x"], case["final_x"])
    assert r["R"] == sum(case["reset"])


@pytest.mark.parametrize("seed", range(40))
def test_serial_matches_python_and_invariants(owmr, seed):
    inst = random_owmr(seed, N=1 + seed % 5, T=30 + 7 * seed, dmax=1 + seed % 4)
    r = owmr.serial(inst)
    q, rs, x0, x = _python_serial(inst)
    np.testing.assert_array_equal(r["q"], q)
    np.testing.assert_array_equal(r["reset"], rs)
    assert r["final_x0"] == x0
    np.testing.assert_array_equal(r["final_x"], x)
    assert r["R"] == int(rs.sum())
    # replay with a ledger: stocks stay in range, and the central stock is its start plus
    # what the resets added minus what the retailers received
    xs = inst.x_init.astype(np.int64).copy()
    c0, added, received = int(inst.x0_init), 0, 0
    for t in range(inst.T):
        n, d = int(inst.retailer[t]), int(inst.demand[t])
        got = min(int(r["q"][t]), c0)
        xs[n] = max(0, xs[n] - d) + got
        received += got
        after = max(0, c0 - int(r["q"][t]))
        if r["reset"][t]:
            added += int(inst.S0) - after
            c0 = int(inst.S0)
        else:
            c0 = after
        assert 0 <= xs[n] <= inst.cap[n] and c0 >= 0
        assert (r["q"][t] >= 0) and (r["q"][t] == 0 or max(0, xs[n] - got) <= inst.s_ret[n])
    # what leaves the central stock at a step is what the retailer receives, min(q, x_0)
    assert c0 == int(inst.x0_init) + added - received


@pytest.mark.parametrize("seed", range(30))
def test_alg1_fixed_point_is_serial(owmr, seed):
    """Proposition 2.1: any partition, any initial cache."""
    inst = random_owmr(100 + seed, N=1 + seed % 4, T=20 + 3 * seed, dmax=3)
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 6))
    worker = rng.integers(0, P, inst.T)
    init = (rng.integers(0, 7, inst.T), rng.integers(0, 2, inst.T)) if seed % 2 else None
    a = owmr.alg1(inst, worker, P, init=init)
    s = owmr.serial(inst)
    assert a["converged"] and a["passes"] <= inst.T + 1
    np.testing.assert_array_equal(a["q"], s["q"])
    np.testing.assert_array_equal(a["reset"], s["reset"])


@pytest.mark.parametrize("seed", range(30))
def test_runs_equal_alg1_pass_by_pass(owmr, seed):
    inst = random_owmr(200 + seed, N=2 + seed % 5, T=25 + 4 * seed, dmax=2 + seed % 3)
    rng = np.random.default_rng(seed)
    G = int(rng.integers(1, inst.N + 1))
    group = rng.integers(0, G, inst.N)
    init = (rng.integers(0, 5, inst.T), rng.integers(0, 2, inst.T)) if seed % 3 == 0 else None
    a = owmr.alg1(inst, group[inst.retailer], G, init=init, record=True)
    b = owmr.runs(inst, group, G, init=init, record=True)
    assert a["passes"] == b["passes"] and a["converged"] and b["converged"]
    np.testing.assert_array_equal(a["caches_q"], b["caches_q"])
    np.testing.assert_array_equal(a["caches_r"], b["caches_r"])


@pytest.mark.parametrize("seed", range(60))
def test_theorem_2r_bound(owmr, seed):
    """s >= every retailer capacity, one process per retailer, empty initial cache."""
    base = random_owmr(300 + seed, N=2 + seed % 6, T=40 + 5 * seed, dmax=1 + seed % 3)
    cap = int(base.cap.max())
    S0 = cap + int(np.random.default_rng(seed).integers(1, 4 * cap + 3))
    inst = random_owmr(300 + seed, N=base.N, T=base.T, dmax=1 + seed % 3, s0=cap, S0=S0)
    R = owmr.serial(inst)["R"]
    b = owmr.runs(inst, np.arange(inst.N), inst.N, record=True)
    s = owmr.serial(inst)
    caches = [(np.zeros(inst.T, np.int32), np.zeros(inst.T, np.int32))] + list(
        zip(b["caches_q"], b["caches_r"]))  # alpha^0, alpha^1, ...
    k_star = next(k for k, (cq, cr) in enumerate(caches)
                  if np.array_equal(cq, s["q"]) and np.array_equal(cr, s["reset"]))
    assert k_star <= 2 * R + 1, (R, k_star)
    assert b["passes"] == k_star + 1


def test_no_binding_central_takes_two_passes(owmr):
    for seed in range(10):
        inst = random_owmr(400 + seed, N=5, T=200, dmax=3, s0=-1, S0=10 ** 9)
        inst.x0_init = 10 ** 9
        b = owmr.runs(inst, np.arange(inst.N), inst.N)
        assert b["passes"] <= 2
        assert owmr.serial(inst)["R"] == 0


def test_base_case_shape(owmr):
    """The appendix's base case: about one reset a week over a year."""
    inst = make_owmr_instance("owmr_n4000_t3650000")
    r = owmr.serial(inst)
    assert 40 <= r["R"] <= 60
    assert int(r["final_x"].max()) <= 20
