"""Thin Python binding of libpicard's OWMR inventory-control entry points
(pk_owmr_workspace_size, pk_owmr_serial_simulate, pk_owmr_picard_simulate in
include/picard.h).  Argument marshalling only; the library does every step."""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import api

OW_SHIFT = 40


class pk_owmr_problem(C.Structure):
    _fields_ = [("n_retailers", C.c_int32), ("reserved", C.c_int32), ("n_orders", C.c_int64),
                ("retailer", C.c_void_p), ("demand", C.c_void_p), ("s_ret", C.c_void_p),
                ("S_ret", C.c_void_p), ("cap", C.c_void_p), ("x_init", C.c_void_p),
                ("s0", C.c_int64), ("S0", C.c_int64), ("x0_init", C.c_int64)]


_bound = False


def lib():
    global _bound
    L = api.lib()
    if not _bound:
        P, vp, sz = C.POINTER(pk_owmr_problem), C.c_void_p, C.c_size_t
        i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.pk_owmr_workspace_size.argtypes = [P, C.POINTER(sz)]
        L.pk_owmr_serial_simulate.argtypes = [P, vp, sz, vp, vp, vp, i64p, i64p, vp]
        L.pk_owmr_picard_simulate.argtypes = [P, C.c_int32, vp, vp, vp, sz, vp, vp, vp, i64p,
                                              i32p, vp, vp, vp]
        for f in ("pk_owmr_workspace_size", "pk_owmr_serial_simulate", "pk_owmr_picard_simulate"):
            getattr(L, f).restype = C.c_int
        _bound = True
    return L


@dataclasses.dataclass
class DeviceOwmr:
    """An OWMR problem resident on the GPU."""
    N: int
    retailer: torch.Tensor
    demand: torch.Tensor
    s_ret: torch.Tensor
    S_ret: torch.Tensor
    cap: torch.Tensor
    x_init: torch.Tensor
    s0: int
    S0: int
    x0_init: int

    @property
    def T(self) -> int:
        return int(self.retailer.numel())

    @classmethod
    def from_instance(cls, inst, device="cuda") -> "DeviceOwmr":
        up = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
        return cls(N=inst.N, retailer=up(inst.retailer), demand=up(inst.demand),
                   s_ret=up(inst.s_ret), S_ret=up(inst.S_ret), cap=up(inst.cap),
                   x_init=up(inst.x_init), s0=int(inst.s0), S0=int(inst.S0),
                   x0_init=int(inst.x0_init))

    def c_problem(self) -> pk_owmr_problem:
        p = lambda t: t.data_ptr() if t.numel() else None
        return pk_owmr_problem(self.N, 0, self.T, p(self.retailer), p(self.demand),
                               self.s_ret.data_ptr(), self.S_ret.data_ptr(), self.cap.data_ptr(),
                               self.x_init.data_ptr(), self.s0, self.S0, self.x0_init)


def workspace_size(prob: DeviceOwmr) -> int:
    p = prob.c_problem()
    n = C.c_size_t(0)
    api._check(lib().pk_owmr_workspace_size(C.byref(p), C.byref(n)))
    return int(n.value)


def serial_simulate(prob: DeviceOwmr, stream=None) -> dict:
    dev = prob.retailer.device
    p = prob.c_problem()
    ws = api.workspace(workspace_size(prob), dev)
    q = torch.empty(prob.T, dtype=torch.int32, device=dev)
    r = torch.empty_like(q)
    fx = torch.empty(prob.N, dtype=torch.int32, device=dev)
    x0 = C.c_int64(0)
    R = C.c_int64(0)
    api._check(lib().pk_owmr_serial_simulate(C.byref(p), api._ptr(ws), ws.numel(), api._ptr(q),
                                             api._ptr(r), api._ptr(fx), C.byref(x0), C.byref(R),
                                             api._stream(stream)))
    return dict(q=q, reset=r, final_x=fx, final_x0=int(x0.value), R=int(R.value))


def picard_simulate(prob: DeviceOwmr, max_passes: int = 0, init=None, record: bool = False,
                    stream=None, raise_not_converged=True) -> dict:
    dev = prob.retailer.device
    p = prob.c_problem()
    ws = api.workspace(workspace_size(prob), dev)
    q = torch.empty(prob.T, dtype=torch.int32, device=dev)
    r = torch.empty_like(q)
    fx = torch.empty(prob.N, dtype=torch.int32, device=dev)
    x0 = C.c_int64(0)
    passes = C.c_int32(0)
    changed = np.zeros(max(max_passes, 1), np.int64) if record else None
    caches = (torch.empty((max_passes, prob.T), dtype=torch.int64, device=dev)
              if record else None)
    iq = ir = None
    if init is not None:
        iq = init[0].to(device=dev, dtype=torch.int32).contiguous()
        ir = init[1].to(device=dev, dtype=torch.int32).contiguous()
    st = lib().pk_owmr_picard_simulate(C.byref(p), int(max_passes), api._ptr(iq), api._ptr(ir),
                                       api._ptr(ws), ws.numel(), api._ptr(q), api._ptr(r),
                                       api._ptr(fx), C.byref(x0), C.byref(passes),
                                       None if changed is None else changed.ctypes.data,
                                       api._ptr(caches), api._stream(stream))
    if st != api.PK_OK and not (st == api.PK_ERR_NOT_CONVERGED and not raise_not_converged):
        api._check(st)
    out = dict(q=q, reset=r, final_x=fx, final_x0=int(x0.value), passes=int(passes.value),
               status=st)
    if record:
        k = out["passes"]
        out["changed"] = changed[:k]
        c = caches[:k]
        out["caches_q"] = (c & ((1 << OW_SHIFT) - 1)).to(torch.int32)
        out["caches_r"] = (c >> OW_SHIFT).to(torch.int32)
    return out
