"""ctypes wrapper of the CPU oracle (picard_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's
CPU-baseline leg, never by the GPU path.  Every function takes an `Instance` from
paper_2406_01939_amd.instances (numpy arrays) and a trajectory index.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "picard_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LOST = -1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics kept)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-variable", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("R", C.c_int32), ("T", C.c_int64),
                ("sku", C.c_void_p), ("region", C.c_void_p), ("qty", C.c_void_p),
                ("x0", C.c_void_p), ("cost", C.c_void_p), ("params", C.c_void_p),
                ("hidden", C.c_int32), ("n_hidden_layers", C.c_int32),
                ("rng_seed", C.c_uint64), ("traj", C.c_int32)]


_lib = None


def lib():
    """The oracle library.  PICARD_ORACLE_LIB names another build of the same source
    (the mutation tests point it at deliberately broken copies)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PICARD_ORACLE_LIB")
        if not path:
            if not os.path.exists(LIB):
                build(force=False)
            path = LIB
        _lib = load(path)
    return _lib


def load(path: str):
    """Load a build of picard_oracle.c and declare its entry points."""
    L = C.CDLL(path)
    P = C.POINTER(_Problem)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.orc_serial.argtypes = [P, vp, vp, vp, vp, vp]
    L.orc_eval_at.argtypes = [P, vp, vp, vp, vp, vp]
    L.orc_eval_at_range.argtypes = [P, vp, i64, i64, vp, vp, vp, vp]
    L.orc_reinforce_range.argtypes = [P, vp, vp, i64, i64, vp, vp, vp]
    L.orc_policy_at.argtypes = [P, i64, vp, vp, vp, vp, vp]
    L.orc_alg1.argtypes = [P, vp, i64, vp, i32, vp, vp, vp]
    L.orc_picard_runs.argtypes = [P, vp, vp, i32, vp, vp, vp, vp]
    L.orc_reinforce.argtypes = [P, vp, vp, vp, vp, vp]
    Pol = C.POINTER(_CapPolicy)
    L.orc_serial_cap.argtypes = [P, vp, Pol, vp, vp, vp]
    L.orc_alg1_cap.argtypes = [P, vp, Pol, vp, i64, vp, i32, vp, vp, vp]
    L.orc_picard_timeblocks_cap.argtypes = [P, vp, Pol, i64, vp, i32, vp, vp, vp, vp]
    L.orc_mlp_scores.argtypes = [P, i32, vp, vp]
    L.orc_philox4x32_10.argtypes = [vp, vp, vp]
    L.orc_philox4x32_10.restype = None
    L.orc_uniform.argtypes = [C.c_uint64, i32, i64, i32]
    L.orc_uniform.restype = C.c_double
    L.orc_gumbel.argtypes = [C.c_uint64, i32, i64, i32]
    L.orc_gumbel.restype = C.c_double
    L.orc_param_count.argtypes = [i32, i32, i32]
    L.orc_param_count.restype = C.c_int64
    return L


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Bound:
    """Keeps the numpy arrays behind a _Problem alive while it is in use."""

    def __init__(self, inst, b: int):
        lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
        self.sku = np.ascontiguousarray(inst.sku[lo:hi], dtype=np.int32)
        self.region = np.ascontiguousarray(inst.region[lo:hi], dtype=np.int32)
        self.qty = np.ascontiguousarray(inst.qty[lo:hi], dtype=np.int32)
        # the per-state policy (policy_at) reads no initial inventory: workloads whose x0
        # is only a generator bind none
        self.x0 = (None if inst.x0 is None
                   else np.ascontiguousarray(inst.x0[b], dtype=np.int32))
        self.cost = np.ascontiguousarray(inst.cost[b], dtype=np.int32)
        self.params = (None if inst.params is None
                       else np.ascontiguousarray(inst.params, dtype=np.float32))
        self.T = hi - lo
        self.p = _Problem(inst.N, inst.K, inst.R, self.T, _ptr(self.sku), _ptr(self.region),
                          _ptr(self.qty), _ptr(self.x0), _ptr(self.cost), _ptr(self.params),
                          inst.hidden, inst.n_hidden_layers, inst.rng_seed & (2**64 - 1), b)


def _check(rc: int, what: str):
    if rc < 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def serial(inst, b: int = 0, greedy: bool = False) -> dict:
    """Serial rollout of trajectory b (greedy=True forces the greedy policy)."""
    if inst.x0 is None:
        raise ValueError("serial rollout needs the initial inventory (x0 is a generator here)")
    B = _Bound(inst, b)
    if greedy:
        B.p.params = None
    T = B.T
    act = np.empty(T, np.int32)
    sh = np.empty(T, np.int32)
    fin = np.empty((inst.K, inst.N), np.int32)
    z1 = np.empty(T, np.float64)
    z2 = np.empty(T, np.float64)
    _check(lib().orc_serial(C.byref(B.p), _ptr(act), _ptr(sh), _ptr(fin), _ptr(z1), _ptr(z2)),
           "serial")
    return dict(actions=act, shipped=sh, final_inv=fin, z1=z1, z2=z2)


def _windows(T: int, n: int):
    """[0, T) cut into at most n consecutive windows."""
    n = max(1, min(int(n), max(T, 1)))
    cuts = [T * i // n for i in range(n + 1)]
    return [(cuts[i], cuts[i + 1]) for i in range(n)]


def _in_threads(fn, jobs, threads: int):
    """Run fn over jobs in a thread pool (the oracle's C calls release the GIL) and
    return the results in job order."""
    if threads <= 1 or len(jobs) <= 1:
        return [fn(j) for j in jobs]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, jobs))


def eval_at(inst, actions: np.ndarray, b: int = 0, threads: int = 1) -> dict:
    """Policy choice and top-two perturbed scores at the states a given sequence induces.
    threads > 1 evaluates disjoint windows of steps at once (each window replays the
    given actions up to its start)."""
    B = _Bound(inst, b)
    T = B.T
    actions = np.ascontiguousarray(actions, dtype=np.int32)
    ch = np.empty(T, np.int32)
    z1 = np.empty(T, np.float64)
    z2 = np.empty(T, np.float64)
    nf = np.empty(T, np.int32)
    if threads <= 1:
        rcs = [lib().orc_eval_at(C.byref(B.p), _ptr(actions), _ptr(ch), _ptr(z1), _ptr(z2),
                                 _ptr(nf))]
    else:
        rcs = _in_threads(lambda w: lib().orc_eval_at_range(
            C.byref(B.p), _ptr(actions), w[0], w[1], _ptr(ch), _ptr(z1), _ptr(z2), _ptr(nf)),
            _windows(T, 4 * threads), threads)
    for rc in rcs:
        _check(rc, "eval_at")
    if any(rc == -2 for rc in rcs):
        raise ValueError("action sequence is infeasible")
    return dict(choice=ch, z1=z1, z2=z2, n_feasible=nf)


def policy_at(inst, b: int, ts: np.ndarray, x_rows: np.ndarray, threads: int = 1) -> dict:
    """The policy at given states: order ts[i] of trajectory b (time index within the
    trajectory) with its SKU's inventory row x_rows[i] ([n, N]).  Returns the choice and
    the top two perturbed scores per state."""
    B = _Bound(inst, b)
    ts = np.ascontiguousarray(ts, dtype=np.int64)
    x_rows = np.ascontiguousarray(x_rows, dtype=np.int32).reshape(ts.size, inst.N)
    n = ts.size
    ch = np.empty(n, np.int32)
    z1 = np.empty(n, np.float64)
    z2 = np.empty(n, np.float64)
    rcs = _in_threads(lambda w: lib().orc_policy_at(
        C.byref(B.p), w[1] - w[0], _ptr(ts[w[0]:]), _ptr(x_rows[w[0]:]), _ptr(ch[w[0]:]),
        _ptr(z1[w[0]:]), _ptr(z2[w[0]:])), _windows(n, 4 * max(threads, 1)), threads)
    for rc in rcs:
        _check(rc, "policy_at")
    return dict(choice=ch, z1=z1, z2=z2)


def alg1(inst, worker: np.ndarray, n_workers: int, b: int = 0, init_cache=None,
         max_passes: Optional[int] = None, record: bool = True) -> dict:
    """Algorithm 1 by brute force: every process views the whole horizon (tiny instances only)."""
    B = _Bound(inst, b)
    T = B.T
    if max_passes is None:
        max_passes = T + 1
    worker = np.ascontiguousarray(worker, dtype=np.int64)
    init = None if init_cache is None else np.ascontiguousarray(init_cache, dtype=np.int32)
    fin = np.empty(T, np.int32)
    passes = np.zeros(1, np.int32)
    caches = np.empty((max_passes, T), np.int32) if record else None
    rc = lib().orc_alg1(C.byref(B.p), _ptr(worker), n_workers, _ptr(init), max_passes,
                        _ptr(fin), _ptr(passes), _ptr(caches))
    _check(rc, "alg1")
    k = int(passes[0])
    return dict(actions=fin, passes=k, converged=rc == 0,
                caches=None if caches is None else caches[:k])


def picard_runs(inst, worker: np.ndarray, b: int = 0, init_cache=None,
                max_passes: Optional[int] = None, record: bool = False) -> dict:
    """Run-form Picard: the same passes as Algorithm 1, for any partition."""
    B = _Bound(inst, b)
    T = B.T
    if max_passes is None:
        max_passes = T + 1
    worker = np.ascontiguousarray(worker, dtype=np.int64)
    init = None if init_cache is None else np.ascontiguousarray(init_cache, dtype=np.int32)
    fin = np.empty(T, np.int32)
    passes = np.zeros(1, np.int32)
    changed = np.zeros(max_passes, np.int64)
    caches = np.empty((max_passes, T), np.int32) if record else None
    rc = lib().orc_picard_runs(C.byref(B.p), _ptr(worker), _ptr(init), max_passes, _ptr(fin),
                               _ptr(passes), _ptr(changed), _ptr(caches))
    _check(rc, "picard_runs")
    k = int(passes[0])
    return dict(actions=fin, passes=k, converged=rc == 0, changed=changed[:k],
                caches=None if caches is None else caches[:k])


def _cap_array(inst, cap0) -> np.ndarray:
    cap0 = np.ascontiguousarray(cap0, dtype=np.int32)
    if cap0.shape != (inst.N,):
        raise ValueError("capacity must have one entry per warehouse")
    return cap0


class _CapPolicy(C.Structure):
    _fields_ = [("gnum", C.c_int32), ("gden", C.c_int32), ("glow", C.c_int32),
                ("bid_inv", C.c_void_p), ("bid_cap", C.c_void_p)]


def _policy(inst, gamma, bids):
    """The C policy struct and the arrays it points into (kept alive by the caller).
    gamma = (num, den) or (num, den, low); bids = None or (bid_inv [K][N] or None,
    bid_cap [N] or None), int32."""
    keep = []
    bi = bc = None
    if bids is not None:
        if bids[0] is not None:
            bi = np.ascontiguousarray(bids[0], dtype=np.int32)
            if bi.shape != (inst.K, inst.N):
                raise ValueError("bid_inv must be [K][N]")
            keep.append(bi)
        if bids[1] is not None:
            bc = np.ascontiguousarray(bids[1], dtype=np.int32)
            if bc.shape != (inst.N,):
                raise ValueError("bid_cap must be [N]")
            keep.append(bc)
    pol = _CapPolicy(int(gamma[0]), int(gamma[1]), int(gamma[2]) if len(gamma) > 2 else 0,
                     _ptr(bi), _ptr(bc))
    return pol, keep


def serial_cap(inst, cap0, b: int = 0, gamma=(0, 1), bids=None) -> dict:
    """Serial rollout of trajectory b with node capacities cap0 (unit demand); gamma =
    (num, den) or (num, den, low): num 0 for the greedy policy, else the capacity-dependent
    policy, its shadow price on every node relative to the most capacity left (low 0) or
    only on nodes with less than low capacity left; bids = (bid_inv, bid_cap): the
    bid-price policy (with num 0)."""
    B = _Bound(inst, b)
    B.p.params = None
    cap0 = _cap_array(inst, cap0)
    act = np.empty(B.T, np.int32)
    fin = np.empty((inst.K, inst.N), np.int32)
    fcap = np.empty(inst.N, np.int32)
    pol, keep = _policy(inst, gamma, bids)
    _check(lib().orc_serial_cap(C.byref(B.p), _ptr(cap0), C.byref(pol), _ptr(act), _ptr(fin),
                                _ptr(fcap)), "serial_cap")
    return dict(actions=act, final_inv=fin, final_cap=fcap)


def alg1_cap(inst, cap0, worker: np.ndarray, n_workers: int, b: int = 0, init_cache=None,
             max_passes: Optional[int] = None, record: bool = True, gamma=(0, 1),
             bids=None) -> dict:
    """Algorithm 1 with node capacities by brute force (tiny instances only)."""
    B = _Bound(inst, b)
    B.p.params = None
    cap0 = _cap_array(inst, cap0)
    T = B.T
    if max_passes is None:
        max_passes = T + 1
    worker = np.ascontiguousarray(worker, dtype=np.int64)
    init = None if init_cache is None else np.ascontiguousarray(init_cache, dtype=np.int32)
    fin = np.empty(T, np.int32)
    passes = np.zeros(1, np.int32)
    caches = np.empty((max_passes, T), np.int32) if record else None
    pol, keep = _policy(inst, gamma, bids)
    rc = lib().orc_alg1_cap(C.byref(B.p), _ptr(cap0), C.byref(pol), _ptr(worker), n_workers,
                            _ptr(init), max_passes, _ptr(fin),
                            _ptr(passes), _ptr(caches))
    _check(rc, "alg1_cap")
    k = int(passes[0])
    return dict(actions=fin, passes=k, converged=rc == 0,
                caches=None if caches is None else caches[:k])


def picard_timeblocks_cap(inst, cap0, block_len: int, b: int = 0, init_cache=None,
                          max_passes: Optional[int] = None, record: bool = False,
                          gamma=(0, 1), bids=None) -> dict:
    """Algorithm 1's passes with node capacities for the partition into time blocks of
    block_len consecutive orders (one replay per pass)."""
    B = _Bound(inst, b)
    B.p.params = None
    cap0 = _cap_array(inst, cap0)
    T = B.T
    if max_passes is None:
        max_passes = T + 1
    init = None if init_cache is None else np.ascontiguousarray(init_cache, dtype=np.int32)
    fin = np.empty(T, np.int32)
    passes = np.zeros(1, np.int32)
    changed = np.zeros(max_passes, np.int64)
    caches = np.empty((max_passes, T), np.int32) if record else None
    pol, keep = _policy(inst, gamma, bids)
    rc = lib().orc_picard_timeblocks_cap(C.byref(B.p), _ptr(cap0), C.byref(pol), block_len,
                                         _ptr(init), max_passes,
                                         _ptr(fin), _ptr(passes), _ptr(changed), _ptr(caches))
    _check(rc, "picard_timeblocks_cap")
    k = int(passes[0])
    return dict(actions=fin, passes=k, converged=rc == 0, changed=changed[:k],
                caches=None if caches is None else caches[:k])


def time_block_workers(T: int, block_len: int) -> np.ndarray:
    """Process of each order when processes own blocks of consecutive orders."""
    return (np.arange(T, dtype=np.int64) // block_len).astype(np.int64)


def reinforce(inst, actions: np.ndarray, adv: np.ndarray, b: int = 0,
              want_grad: bool = True, threads: int = 1) -> dict:
    """FP64 surrogate L = sum_t A_t log pi(a_t|s_t), per-step log pi and dL/dtheta.
    threads > 1 sums the terms of disjoint windows of steps computed at once (in window
    order)."""
    B = _Bound(inst, b)
    T = B.T
    actions = np.ascontiguousarray(actions, dtype=np.int32)
    adv = np.ascontiguousarray(adv, dtype=np.float64)
    n = int(lib().orc_param_count(inst.R, inst.hidden, inst.n_hidden_layers))
    logp = np.empty(T, np.float64)
    if threads <= 1:
        grad = np.empty(n, np.float64) if want_grad else None
        L = np.zeros(1, np.float64)
        rc = lib().orc_reinforce(C.byref(B.p), _ptr(actions), _ptr(adv), _ptr(logp),
                                 _ptr(grad), _ptr(L))
        parts = [(rc, grad, L)]
    else:
        def one(w):
            g = np.empty(n, np.float64) if want_grad else None
            L = np.zeros(1, np.float64)
            rc = lib().orc_reinforce_range(C.byref(B.p), _ptr(actions), _ptr(adv), w[0], w[1],
                                           _ptr(logp), _ptr(g), _ptr(L))
            return rc, g, L
        parts = _in_threads(one, _windows(T, 4 * threads), threads)
    for rc, _, _ in parts:
        if rc == -2:
            raise ValueError("an action is outside the feasible set of its state")
        _check(rc, "reinforce")
    grad = None
    if want_grad:
        grad = parts[0][1].copy()
        for _, g, _ in parts[1:]:
            grad += g
    return dict(objective=float(sum(float(L[0]) for _, _, L in parts)), logp=logp, grad=grad)


def mlp_scores(inst, r: int, x_row: np.ndarray, b: int = 0) -> np.ndarray:
    B = _Bound(inst, b)
    x_row = np.ascontiguousarray(x_row, dtype=np.int32)
    s = np.empty(inst.N, np.float64)
    _check(lib().orc_mlp_scores(C.byref(B.p), r, _ptr(x_row), _ptr(s)), "mlp_scores")
    return s


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, traj: int, t: int, w: int) -> float:
    return float(lib().orc_uniform(seed & (2**64 - 1), traj, t, w))


def gumbel(seed: int, traj: int, t: int, w: int) -> float:
    return float(lib().orc_gumbel(seed & (2**64 - 1), traj, t, w))


def param_count(R: int, hidden: int = 64, n_hidden_layers: int = 2) -> int:
    return int(lib().orc_param_count(R, hidden, n_hidden_layers))


# --------------------------------------------------------------------------------------
# Partitions (Section 2: each process m owns a disjoint set of steps T_m).
# --------------------------------------------------------------------------------------
def sorted_positions(inst) -> np.ndarray:
    """Position of every order in the batch's (trajectory, SKU)-sorted list, ties kept in
    time order."""
    traj = np.repeat(np.arange(inst.n_traj, dtype=np.int64), np.diff(inst.traj_offsets))
    key = traj * inst.K + inst.sku.astype(np.int64)
    order = np.argsort(key, kind="stable")
    pos = np.empty_like(order)
    pos[order] = np.arange(order.size, dtype=np.int64)
    return pos


def block_workers(inst, block_len: int) -> np.ndarray:
    """Process of every order when blocks of `block_len` consecutive positions of the
    (trajectory, SKU)-sorted list form the processes.  block_len=1 gives every step its
    own process; a block at least as long as every segment gives a product partition."""
    return sorted_positions(inst) // int(block_len)


def product_workers(inst, b: int = 0) -> np.ndarray:
    """Product partition of Section 3: all orders of one SKU go to one process."""
    lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
    return inst.sku[lo:hi].astype(np.int64)


def n_runs_per_segment(inst, worker: np.ndarray, b: int = 0) -> np.ndarray:
    """Number of runs (maximal same-process stretches) of each SKU segment."""
    lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
    sku = inst.sku[lo:hi]
    w = worker[lo:hi] if worker.size == inst.total_orders else worker
    order = np.argsort(sku, kind="stable")
    s, ww = sku[order], w[order]
    new = np.ones(s.size, bool)
    new[1:] = (s[1:] != s[:-1]) | (ww[1:] != ww[:-1])
    return np.bincount(s[new], minlength=inst.K)


# --------------------------------------------------------------------------------------
# Policy-gradient loop (Section 4.2): REINFORCE advantages of a rollout, Adam update.
# --------------------------------------------------------------------------------------
def margin_rewards(inst, actions: np.ndarray, shipped: np.ndarray, revenue: int,
                   b: int = 0) -> np.ndarray:
    """Reward of every step of trajectory b: the chosen warehouse's margin on the units
    it ships, (revenue - cost[a][region]) * shipped, and 0 for a lost sale (Section 3: an
    order earns the reward of the node that serves it, nothing when unserved).  int64."""
    lo, hi = int(inst.traj_offsets[b]), int(inst.traj_offsets[b + 1])
    a = np.asarray(actions[lo:hi] if len(actions) == inst.total_orders else actions, np.int64)
    s = np.asarray(shipped[lo:hi] if len(shipped) == inst.total_orders else shipped, np.int64)
    reg = inst.region[lo:hi].astype(np.int64)
    served = a >= 0
    c = inst.cost[b][np.where(served, a, 0), reg].astype(np.int64)
    return np.where(served, (int(revenue) - c) * s, 0).astype(np.int64)


def advantages(inst, actions: np.ndarray, shipped: np.ndarray, revenue: int,
               b: int = 0) -> dict:
    """REINFORCE advantages of trajectory b: reward-to-go G_t = sum of r_u over u >= t,
    minus its mean over the trajectory.  G and its sum are exact integers; the result is
    rounded once, float32(double(G_t) - double(sum G) / T)."""
    r = margin_rewards(inst, actions, shipped, revenue, b)
    T = r.size
    if T == 0:
        return dict(rewards=r, rtg=r.copy(), advantages=np.zeros(0, np.float32), ret=0)
    G = np.cumsum(r[::-1])[::-1].astype(np.int64)
    S = int(G.sum())
    A = (G.astype(np.float64) - np.float64(S) / np.float64(T)).astype(np.float32)
    return dict(rewards=r, rtg=G, advantages=A, ret=int(G[0]))


def adam_step(theta, g, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, ascend: bool = True):
    """One Adam step (Kingma and Ba, Algorithm 1) in float64: biased moment estimates,
    their bias corrections by 1 - beta^step, and a move of lr * mhat / (sqrt(vhat) + eps)
    up the gradient when ascending (the REINFORCE surrogate is maximised), down
    otherwise.  Returns new (theta, m, v)."""
    theta, g, m, v = (np.asarray(x, np.float64) for x in (theta, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    move = lr * mhat / (np.sqrt(vhat) + eps)
    return (theta + move if ascend else theta - move), m, v
