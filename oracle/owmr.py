"""ctypes wrapper of the OWMR inventory oracle (owmr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's
CPU-baseline leg, never by the GPU path.  Every function takes an `OwmrInstance` from
paper_2406_01939_amd.instances (numpy arrays).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "owmr_oracle.c")
LIB = os.path.join(HERE, "libowmr_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", SRC, "-o",
                               tmp])
        os.replace(tmp, LIB)
    return LIB


class _Owmr(C.Structure):
    _fields_ = [("N", C.c_int32), ("T", C.c_int64), ("retailer", C.c_void_p),
                ("demand", C.c_void_p), ("s_ret", C.c_void_p), ("S_ret", C.c_void_p),
                ("cap", C.c_void_p), ("x_init", C.c_void_p), ("s0", C.c_int64),
                ("S0", C.c_int64), ("x0_init", C.c_int64)]


_lib = None


def lib():
    """The oracle library.  PICARD_OWMR_ORACLE_LIB names another build of the same source
    (the mutation tests point it at deliberately broken copies)."""
    global _lib
    if _lib is None:
        path = os.environ.get("PICARD_OWMR_ORACLE_LIB")
        if not path:
            build(force=False)
            path = LIB
        L = C.CDLL(path)
        P = C.POINTER(_Owmr)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.orc_owmr_serial.argtypes = [P, vp, vp, vp, vp]
        L.orc_owmr_serial.restype = C.c_int64
        for f in (L.orc_owmr_alg1, L.orc_owmr_runs):
            f.argtypes = [P, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp]
            f.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Bound:
    def __init__(self, inst):
        c = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self.retailer, self.demand = c(inst.retailer), c(inst.demand)
        self.s_ret, self.S_ret, self.cap, self.x_init = (c(inst.s_ret), c(inst.S_ret),
                                                         c(inst.cap), c(inst.x_init))
        self.p = _Owmr(inst.N, self.retailer.size, _ptr(self.retailer), _ptr(self.demand),
                       _ptr(self.s_ret), _ptr(self.S_ret), _ptr(self.cap), _ptr(self.x_init),
                       int(inst.s0), int(inst.S0), int(inst.x0_init))


def serial(inst) -> dict:
    """The serial rollout: orders q, resets, final stocks and R (the number of resets)."""
    B = _Bound(inst)
    T = B.retailer.size
    q = np.empty(T, np.int32)
    r = np.empty(T, np.int32)
    fx0 = np.zeros(1, np.int64)
    fx = np.empty(inst.N, np.int64)
    R = lib().orc_owmr_serial(C.byref(B.p), _ptr(q), _ptr(r), _ptr(fx0), _ptr(fx))
    if R < 0:
        raise ValueError("invalid OWMR instance")
    return dict(q=q, reset=r, final_x0=int(fx0[0]), final_x=fx, R=int(R))


def _passes(fn, inst, assign: np.ndarray, n: int, init=None, max_passes=None, record=False):
    B = _Bound(inst)
    T = B.retailer.size
    mp = int(max_passes) if max_passes else T + 1
    assign = np.ascontiguousarray(assign, dtype=np.int64)
    iq = ir = None
    if init is not None:
        iq = np.ascontiguousarray(init[0], dtype=np.int32)
        ir = np.ascontiguousarray(init[1], dtype=np.int32)
    oq = np.empty(T, np.int32)
    orr = np.empty(T, np.int32)
    passes = np.zeros(1, np.int32)
    cq = np.empty((mp, T), np.int32) if record else None
    cr = np.empty((mp, T), np.int32) if record else None
    rc = fn(C.byref(B.p), _ptr(assign), n, _ptr(iq), _ptr(ir), mp, _ptr(oq), _ptr(orr),
            _ptr(passes), _ptr(cq), _ptr(cr))
    if rc < 0:
        raise ValueError("invalid OWMR instance or assignment")
    k = int(passes[0])
    out = dict(q=oq, reset=orr, passes=k, converged=rc == 0)
    if record:
        out["caches_q"], out["caches_r"] = cq[:k], cr[:k]
    return out


def alg1(inst, worker: np.ndarray, n_workers: int, init=None, max_passes=None, record=False):
    """Algorithm 1 by brute force for any assignment worker[t] of steps to processes."""
    return _passes(lib().orc_owmr_alg1, inst, worker, n_workers, init, max_passes, record)


def runs(inst, group: np.ndarray, n_groups: int, init=None, max_passes=None, record=False):
    """Algorithm 1's passes when process group[n] owns all of retailer n's steps, from two
    scans of the cache per pass."""
    return _passes(lib().orc_owmr_runs, inst, group, n_groups, init, max_passes, record)
