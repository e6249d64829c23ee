"""Thin Python binding of libpicard's C ABI (include/picard.h).

Argument marshalling only: every step of the simulation runs in the HIP library.  The
entry points keep the C names (pk_picard_simulate, pk_serial_simulate, pk_policy_grad,
pk_workspace_size, pk_autotune); PyTorch supplies device memory and the stream.
Loading fails loudly if the built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpicard.so")

PK_OK = 0
PK_ERR_INVALID_ARG = -1
PK_ERR_SHAPE = -2
PK_ERR_HIP = -3
PK_ERR_NOT_CONVERGED = -4
PK_ERR_WORKSPACE = -5
PK_ERR_UNSUPPORTED = -6
PK_ERR_INTERNAL = -7
PK_LOST = -1
PK_POLICY_GREEDY = 0
PK_POLICY_MLP = 1

STATUS_NAMES = {0: "PK_OK", -1: "PK_ERR_INVALID_ARG", -2: "PK_ERR_SHAPE", -3: "PK_ERR_HIP",
                -4: "PK_ERR_NOT_CONVERGED", -5: "PK_ERR_WORKSPACE", -6: "PK_ERR_UNSUPPORTED",
                -7: "PK_ERR_INTERNAL"}


class PicardError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pk_problem(C.Structure):
    _fields_ = [("n_warehouses", C.c_int32), ("n_skus", C.c_int32), ("n_regions", C.c_int32),
                ("n_traj", C.c_int32), ("traj_offsets", C.c_void_p), ("sku", C.c_void_p),
                ("region", C.c_void_p), ("qty", C.c_void_p), ("init_inv", C.c_void_p),
                ("cost", C.c_void_p), ("rng_seed", C.c_uint64)]


class pk_policy(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_hidden_layers", C.c_int32), ("hidden", C.c_int32),
                ("emb_dim", C.c_int32), ("params", C.c_void_p)]


class pk_picard_opts(C.Structure):
    _fields_ = [("block_len", C.c_int32), ("max_passes", C.c_int32),
                ("use_frontier", C.c_int32), ("graph_unroll", C.c_int32),
                ("init_cache", C.c_void_p), ("validate", C.c_int32), ("partition", C.c_void_p),
                ("walk_waves", C.c_int32), ("lane_max", C.c_int32)]


class pk_cap_policy(C.Structure):
    _fields_ = [("gamma_num", C.c_int32), ("gamma_den", C.c_int32), ("gamma_low", C.c_int32),
                ("reserved", C.c_int32), ("bid_inv", C.c_void_p), ("bid_cap", C.c_void_p)]


class pk_stats(C.Structure):
    _fields_ = [("passes", C.c_void_p), ("passes_max", C.c_int32), ("block_len", C.c_int32),
                ("changed_total", C.c_int64), ("runs_walked", C.c_int64),
                ("orders_walked", C.c_int64), ("near_ties", C.c_int64), ("walk_ms", C.c_double),
                ("walk_launches", C.c_int64), ("walk_bytes", C.c_int64), ("walk_flops", C.c_int64),
                ("timing", C.c_int32), ("scan_ms", C.c_double), ("scan_launches", C.c_int64),
                ("scan_bytes", C.c_int64), ("walk_waves", C.c_int32)]


_lib = None


def lib():
    """The loaded libpicard.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2406_01939_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
        P, Po, O, S = (C.POINTER(pk_problem), C.POINTER(pk_policy), C.POINTER(pk_picard_opts),
                       C.POINTER(pk_stats))
        L.pk_workspace_size.argtypes = [P, Po, O, C.POINTER(sz)]
        L.pk_serial_simulate.argtypes = [P, Po, vp, sz, vp, vp, vp, i32, vp]
        L.pk_picard_simulate.argtypes = [P, Po, O, vp, sz, vp, vp, vp, S, vp]
        L.pk_picard_simulate_noalloc.argtypes = [P, Po, O, vp, vp, vp, S, vp]
        L.pk_policy_grad.argtypes = [P, Po, vp, vp, vp, vp, C.POINTER(C.c_double), vp, sz, i32, vp]
        L.pk_autotune.argtypes = [P, Po, vp, sz, C.POINTER(i32), vp]
        L.pk_policy_scores.argtypes = [P, Po, i32, i32, vp, vp, vp, sz, vp]
        L.pk_advantages_workspace_size.argtypes = [P, C.POINTER(sz)]
        L.pk_reinforce_advantages.argtypes = [P, vp, vp, i32, vp, vp, vp, sz, vp]
        f64 = C.c_double
        L.pk_adam_step.argtypes = [vp, vp, vp, vp, C.c_int64, i32, f64, f64, f64, f64, i32, vp]
        L.pk_capacity_workspace_size.argtypes = [P, vp, i32, C.POINTER(sz)]
        CP = C.POINTER(pk_cap_policy)
        L.pk_serial_simulate_capacity.argtypes = [P, vp, CP, vp, sz, vp, vp, vp, vp]
        L.pk_picard_simulate_capacity.argtypes = [P, vp, CP, i32, i32, vp, vp, sz, vp, vp, vp,
                                                  C.POINTER(i32), vp, vp, vp]
        for f in ("pk_workspace_size", "pk_serial_simulate", "pk_picard_simulate",
                  "pk_picard_simulate_noalloc",
                  "pk_policy_grad", "pk_autotune", "pk_policy_scores",
                  "pk_advantages_workspace_size", "pk_reinforce_advantages", "pk_adam_step",
                  "pk_capacity_workspace_size", "pk_serial_simulate_capacity",
                  "pk_picard_simulate_capacity"):
            getattr(L, f).restype = C.c_int
        L.pk_last_error.restype = C.c_char_p
        L.pk_last_error.argtypes = []
        L.pk_version.restype = C.c_char_p
        L.pk_version.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != PK_OK:
        raise PicardError(status, lib().pk_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class DeviceProblem:
    """A problem resident on the GPU: device tensors plus the host trajectory offsets."""
    N: int
    K: int
    R: int
    traj_offsets: np.ndarray  # host int64
    sku: torch.Tensor
    region: torch.Tensor
    qty: torch.Tensor
    init_inv: torch.Tensor
    cost: torch.Tensor
    rng_seed: int
    params: Optional[torch.Tensor] = None
    n_hidden_layers: int = 2
    hidden: int = 64

    @property
    def n_traj(self) -> int:
        return int(self.traj_offsets.size - 1)

    @property
    def total(self) -> int:
        return int(self.traj_offsets[-1])

    @classmethod
    def from_instance(cls, inst, device="cuda") -> "DeviceProblem":
        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        if inst.x0 is not None:
            x0 = up(inst.x0, torch.int32)
        else:  # drawn on the device by the instance's counter-based generators
            x0 = torch.empty((inst.n_traj, inst.K, inst.N), dtype=torch.int32, device=device)
            for b in range(inst.n_traj):
                inst.x0_gen[b].device(b, inst.N, x0[b])
        return cls(N=inst.N, K=inst.K, R=inst.R,
                   traj_offsets=np.ascontiguousarray(inst.traj_offsets, dtype=np.int64),
                   sku=up(inst.sku, torch.int32), region=up(inst.region, torch.int32),
                   qty=up(inst.qty, torch.int32), init_inv=x0,
                   cost=up(inst.cost, torch.int32), rng_seed=int(inst.rng_seed) & (2**64 - 1),
                   params=None if inst.params is None else up(inst.params, torch.float32),
                   n_hidden_layers=inst.n_hidden_layers, hidden=inst.hidden)

    def c_problem(self) -> pk_problem:
        self._offs = np.ascontiguousarray(self.traj_offsets, dtype=np.int64)
        return pk_problem(self.N, self.K, self.R, self.n_traj, self._offs.ctypes.data,
                          _ptr(self.sku), _ptr(self.region), _ptr(self.qty),
                          _ptr(self.init_inv), _ptr(self.cost), self.rng_seed)

    def c_policy(self, kind: str) -> pk_policy:
        if kind == "greedy":
            return pk_policy(PK_POLICY_GREEDY, 0, 0, 0, None)
        if kind == "mlp":
            if self.params is None:
                raise ValueError("problem has no MLP parameters")
            return pk_policy(PK_POLICY_MLP, self.n_hidden_layers, self.hidden, 16,
                             _ptr(self.params))
        raise ValueError(kind)


_ws_cache = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached uint8 device buffer of at least nbytes (grown on demand)."""
    key = torch.device(device)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        _ws_cache.pop(key, None)
        t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    return t


def pk_workspace_size(prob: DeviceProblem, policy: str = "greedy", block_len: int = 0) -> int:
    p, po = prob.c_problem(), prob.c_policy(policy)
    o = pk_picard_opts(block_len, 0, 1, 0, None, 0, None)
    n = C.c_size_t(0)
    _check(lib().pk_workspace_size(C.byref(p), C.byref(po), C.byref(o), C.byref(n)))
    return int(n.value)


def pk_serial_simulate(prob: DeviceProblem, policy: str = "greedy", want_shipped=True,
                       want_final=True, validate=False, stream=None) -> dict:
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy(policy)
    ws = workspace(pk_workspace_size(prob, policy), dev)
    actions = torch.empty(prob.total, dtype=torch.int32, device=dev)
    shipped = torch.empty_like(actions) if want_shipped else None
    final = torch.empty_like(prob.init_inv) if want_final else None
    _check(lib().pk_serial_simulate(C.byref(p), C.byref(po), _ptr(ws), ws.numel(),
                                    _ptr(actions), _ptr(shipped), _ptr(final), int(validate),
                                    _stream(stream)))
    return dict(actions=actions, shipped=shipped, final_inv=final)


def pk_picard_simulate(prob: DeviceProblem, policy: str = "greedy", block_len: int = 0,
                       max_passes: int = 0, use_frontier: bool = True, graph_unroll: int = 0,
                       init_cache: Optional[torch.Tensor] = None, validate: bool = False,
                       partition: Optional[torch.Tensor] = None,
                       want_shipped=True, want_final=True, timing=False, stream=None,
                       raise_not_converged=True, out: Optional[dict] = None,
                       walk_waves: int = 0, lane_max: int = 0) -> dict:
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy(policy)
    o = pk_picard_opts(block_len, max_passes, int(use_frontier), graph_unroll,
                       _ptr(init_cache), int(validate), _ptr(partition), walk_waves, lane_max)
    n = C.c_size_t(0)
    _check(lib().pk_workspace_size(C.byref(p), C.byref(po), C.byref(o), C.byref(n)))
    ws = workspace(int(n.value), dev)
    if out is None:
        out = dict(actions=torch.empty(prob.total, dtype=torch.int32, device=dev))
        out["shipped"] = torch.empty_like(out["actions"]) if want_shipped else None
        out["final_inv"] = torch.empty_like(prob.init_inv) if want_final else None
    passes = np.zeros(prob.n_traj, dtype=np.int32)
    st = pk_stats()
    st.passes = passes.ctypes.data
    st.timing = int(timing)
    status = lib().pk_picard_simulate(C.byref(p), C.byref(po), C.byref(o), _ptr(ws), ws.numel(),
                                      _ptr(out["actions"]), _ptr(out["shipped"]),
                                      _ptr(out["final_inv"]), C.byref(st), _stream(stream))
    if status != PK_OK and not (status == PK_ERR_NOT_CONVERGED and not raise_not_converged):
        _check(status)
    out["status"] = status
    out["passes"] = passes
    out["stats"] = {f: getattr(st, f) for f, _ in pk_stats._fields_ if f not in ("passes",)}
    return out


def pk_picard_simulate_noalloc(prob: DeviceProblem, policy: str = "greedy",
                               block_len: int = 0, max_passes: int = 0,
                               init_cache: Optional[torch.Tensor] = None, validate: bool = False,
                               partition: Optional[torch.Tensor] = None, out: Optional[dict] = None,
                               stream=None, raise_not_converged=True) -> dict:
    """pk_picard_simulate_noalloc: the library's static scratch instead of a workspace;
    the caller's output tensors (`out`, else allocated here) as for pk_picard_simulate."""
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy(policy)
    o = pk_picard_opts(block_len, max_passes, 1, 0, _ptr(init_cache), int(validate),
                       _ptr(partition))
    if out is None:
        out = dict(actions=torch.empty(prob.total, dtype=torch.int32, device=dev),
                   shipped=torch.empty(prob.total, dtype=torch.int32, device=dev),
                   final_inv=torch.empty_like(prob.init_inv))
    passes = np.zeros(prob.n_traj, dtype=np.int32)
    st = pk_stats()
    st.passes = passes.ctypes.data
    status = lib().pk_picard_simulate_noalloc(C.byref(p), C.byref(po), C.byref(o),
                                              _ptr(out["actions"]), _ptr(out.get("shipped")),
                                              _ptr(out.get("final_inv")), C.byref(st),
                                              _stream(stream))
    if status != PK_OK and not (status == PK_ERR_NOT_CONVERGED and not raise_not_converged):
        _check(status)
    out["status"] = status
    out["passes"] = passes
    out["stats"] = {f: getattr(st, f) for f, _ in pk_stats._fields_ if f not in ("passes",)}
    return out


def pk_policy_grad(prob: DeviceProblem, actions: torch.Tensor, advantages: torch.Tensor,
                   want_logp=True, want_grad=True, validate=False, stream=None) -> dict:
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy("mlp")
    ws = workspace(pk_workspace_size(prob, "mlp"), dev)
    logp = torch.empty(prob.total, dtype=torch.float32, device=dev) if want_logp else None
    grad = torch.empty_like(prob.params) if want_grad else None
    obj = C.c_double(0.0)
    _check(lib().pk_policy_grad(C.byref(p), C.byref(po), _ptr(actions), _ptr(advantages),
                                _ptr(logp), _ptr(grad), C.byref(obj), _ptr(ws), ws.numel(),
                                int(validate), _stream(stream)))
    return dict(logp=logp, grad=grad, objective=obj.value)


def pk_autotune(prob: DeviceProblem, policy: str = "greedy", stream=None) -> int:
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy(policy)
    ws = workspace(pk_workspace_size(prob, policy), dev)
    best = C.c_int32(0)
    _check(lib().pk_autotune(C.byref(p), C.byref(po), _ptr(ws), ws.numel(), C.byref(best),
                             _stream(stream)))
    return int(best.value)


def pk_policy_scores(prob: DeviceProblem, traj: int, region: int, inv_row: torch.Tensor,
                     stream=None) -> torch.Tensor:
    """Noise-free MLP scores of every warehouse (diagnostic)."""
    dev = prob.sku.device
    p, po = prob.c_problem(), prob.c_policy("mlp")
    ws = workspace(pk_workspace_size(prob, "mlp"), dev)
    inv_row = inv_row.to(device=dev, dtype=torch.int32).contiguous()
    out = torch.empty(prob.N, dtype=torch.float32, device=dev)
    _check(lib().pk_policy_scores(C.byref(p), C.byref(po), traj, region, _ptr(inv_row),
                                  _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def pk_reinforce_advantages(prob: DeviceProblem, actions: torch.Tensor, shipped: torch.Tensor,
                            revenue: int, want_returns=True, stream=None) -> dict:
    """REINFORCE advantages of a rollout (reward-to-go minus its trajectory mean) and each
    trajectory's total reward, from the margin reward (revenue - cost) * shipped."""
    dev = prob.sku.device
    p = prob.c_problem()
    n = C.c_size_t(0)
    _check(lib().pk_advantages_workspace_size(C.byref(p), C.byref(n)))
    ws = workspace(int(n.value), dev)
    adv = torch.empty(prob.total, dtype=torch.float32, device=dev)
    ret = torch.empty(prob.n_traj, dtype=torch.int64, device=dev) if want_returns else None
    _check(lib().pk_reinforce_advantages(C.byref(p), _ptr(actions), _ptr(shipped), int(revenue),
                                         _ptr(adv), _ptr(ret), _ptr(ws), ws.numel(),
                                         _stream(stream)))
    return dict(advantages=adv, returns=ret)


def pk_adam_step(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                 step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, ascend: bool = True, stream=None) -> None:
    """One in-place Adam step on float32 device tensors of equal length."""
    for t in (params, grad, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != params.numel():
            raise ValueError("params, grad, m and v must be contiguous float32 of equal length")
    _check(lib().pk_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(),
                              int(step), float(lr), float(beta1), float(beta2), float(eps),
                              int(ascend), _stream(stream)))


def pk_capacity_workspace_size(prob: DeviceProblem, capacity: torch.Tensor,
                               block_len: int = 0) -> int:
    p = prob.c_problem()
    n = C.c_size_t(0)
    _check(lib().pk_capacity_workspace_size(C.byref(p), _ptr(capacity), int(block_len),
                                            C.byref(n)))
    return int(n.value)


def _cap_tensor(prob: DeviceProblem, capacity) -> torch.Tensor:
    c = torch.as_tensor(capacity).to(device=prob.sku.device, dtype=torch.int32).contiguous()
    if c.numel() != prob.N:
        raise ValueError("capacity must have one entry per warehouse")
    return c


def _cap_policy(prob: DeviceProblem, gamma, bids):
    """pk_cap_policy from gamma = (num, den) or (num, den, low) and bids = None or
    (bid_inv [K][N] or None, bid_cap [N] or None); returns it with the device arrays it
    points at (kept alive by the caller)."""
    dev = prob.sku.device
    keep = []
    ptrs = [None, None]
    if bids is not None:
        for i, (b, shape) in enumerate(zip(bids, ((prob.K, prob.N), (prob.N,)))):
            if b is None:
                continue
            t = torch.as_tensor(b).to(device=dev, dtype=torch.int32).contiguous()
            if tuple(t.shape) != shape:
                raise ValueError(f"bid prices must have shape {shape}, got {tuple(t.shape)}")
            keep.append(t)
            ptrs[i] = t.data_ptr()
    pol = pk_cap_policy(int(gamma[0]), int(gamma[1]), int(gamma[2]) if len(gamma) > 2 else 0, 0,
                        ptrs[0], ptrs[1])
    return pol, keep


def pk_serial_simulate_capacity(prob: DeviceProblem, capacity, want_final=True,
                                gamma=(0, 1), bids=None, stream=None) -> dict:
    """Serial sweep with node capacities (one order at a time on the GPU); gamma = (num,
    den) or (num, den, low): num 0 for the greedy policy, else the capacity-dependent
    policy, priced relative to the most capacity left (low 0) or only below low;
    bids = (bid_inv [K][N] or None, bid_cap [N] or None): the bid-price policy (num 0)."""
    dev = prob.sku.device
    cap = _cap_tensor(prob, capacity)
    pol, keep = _cap_policy(prob, gamma, bids)
    p = prob.c_problem()
    ws = workspace(pk_capacity_workspace_size(prob, cap), dev)
    actions = torch.empty(prob.total, dtype=torch.int32, device=dev)
    final = torch.empty_like(prob.init_inv) if want_final else None
    fcap = torch.empty(prob.N, dtype=torch.int32, device=dev) if want_final else None
    _check(lib().pk_serial_simulate_capacity(C.byref(p), _ptr(cap), C.byref(pol), _ptr(ws),
                                             ws.numel(), _ptr(actions), _ptr(final), _ptr(fcap),
                                             _stream(stream)))
    del keep
    return dict(actions=actions, final_inv=final, final_cap=fcap)


def pk_picard_simulate_capacity(prob: DeviceProblem, capacity, block_len: int = 0,
                                max_passes: int = 0,
                                init_cache: Optional[torch.Tensor] = None,
                                want_final=True, record=False, gamma=(0, 1), bids=None,
                                stream=None, raise_not_converged=True) -> dict:
    """Algorithm 1 with node capacities; processes are blocks of consecutive orders;
    gamma and bids as for pk_serial_simulate_capacity."""
    dev = prob.sku.device
    cap = _cap_tensor(prob, capacity)
    pol, keep = _cap_policy(prob, gamma, bids)
    p = prob.c_problem()
    T = prob.total
    mp = max_passes if max_passes > 0 else T + 1
    ws = workspace(pk_capacity_workspace_size(prob, cap, block_len), dev)
    actions = torch.empty(T, dtype=torch.int32, device=dev)
    final = torch.empty_like(prob.init_inv) if want_final else None
    fcap = torch.empty(prob.N, dtype=torch.int32, device=dev) if want_final else None
    caches = torch.empty((mp, T), dtype=torch.int32, device=dev) if record else None
    changed = np.zeros(mp, dtype=np.int64)
    passes = C.c_int32(0)
    status = lib().pk_picard_simulate_capacity(
        C.byref(p), _ptr(cap), C.byref(pol), int(block_len), int(max_passes),
        _ptr(init_cache), _ptr(ws), ws.numel(), _ptr(actions), _ptr(final), _ptr(fcap),
        C.byref(passes), changed.ctypes.data, _ptr(caches), _stream(stream))
    del keep
    if status != PK_OK and not (status == PK_ERR_NOT_CONVERGED and not raise_not_converged):
        _check(status)
    k = int(passes.value)
    return dict(actions=actions, final_inv=final, final_cap=fcap, passes=k, status=status,
                changed=changed[:k], caches=None if caches is None else caches[:k])


# C names are the primary API; the short names are aliases.
picard_simulate = pk_picard_simulate
serial_simulate = pk_serial_simulate
policy_grad = pk_policy_grad
