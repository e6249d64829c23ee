"""The C-ABI library loads and exports every entry point include/picard.h declares; the
Python binding's structs match the header's sizes.  No compute calls (CPU only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "picard.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pk_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("pk_picard_simulate", "pk_serial_simulate", "pk_policy_grad",
                 "pk_workspace_size", "pk_autotune", "pk_last_error", "pk_version"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2406_01939_amd import api
    L = api.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.pk_version().decode().startswith("libpicard")
    assert L.pk_last_error() is not None


def test_struct_layouts():
    from paper_2406_01939_amd import api
    assert C.sizeof(api.pk_problem) == 4 * 4 + 6 * 8 + 8
    assert C.sizeof(api.pk_policy) == 4 * 4 + 8
    assert C.sizeof(api.pk_picard_opts) == 4 * 4 + 8 + 8 + 8 + 8
    assert C.sizeof(api.pk_stats) == 8 + 4 + 4 + 4 * 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(api.pk_cap_policy) == 4 * 4 + 8 + 8


def test_host_validation_without_gpu():
    """Shape errors are caught on the host before any device work."""
    import numpy as np
    from paper_2406_01939_amd import api
    offs = np.array([0, 5], dtype=np.int64)
    p = api.pk_problem(0, 1, 1, 1, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    po = api.pk_policy(0, 0, 0, 0, None)
    n = C.c_size_t(0)
    st = api.lib().pk_workspace_size(C.byref(p), C.byref(po), None, C.byref(n))
    assert st == api.PK_ERR_SHAPE
    assert b"dimensions" in api.lib().pk_last_error()
    p = api.pk_problem(2000, 1, 1, 1, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert api.lib().pk_workspace_size(C.byref(p), C.byref(po), None, C.byref(n)) == api.PK_ERR_SHAPE
    bad = np.array([0, 5, 3], dtype=np.int64)
    p = api.pk_problem(2, 1, 1, 2, bad.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert api.lib().pk_workspace_size(C.byref(p), C.byref(po), None, C.byref(n)) == api.PK_ERR_SHAPE
    p = api.pk_problem(2, 1, 1, 1, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert api.lib().pk_workspace_size(C.byref(p), C.byref(po), None, C.byref(n)) == api.PK_OK
    assert n.value > 0
    po = api.pk_policy(7, 0, 0, 0, None)
    assert api.lib().pk_workspace_size(C.byref(p), C.byref(po), None, C.byref(n)) == api.PK_ERR_INVALID_ARG


def test_training_entry_points_validate_on_host():
    """The policy-gradient entry points reject bad arguments before any device work."""
    import numpy as np
    from paper_2406_01939_amd import api
    L = api.lib()
    # Adam: step, betas, lr and eps are checked before the launch
    assert L.pk_adam_step(None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == api.PK_OK
    assert L.pk_adam_step(None, None, None, None, 4, 1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == api.PK_ERR_INVALID_ARG
    assert L.pk_adam_step(None, None, None, None, -1, 1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == api.PK_ERR_INVALID_ARG
    assert L.pk_adam_step(None, None, None, None, 0, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None) == api.PK_ERR_INVALID_ARG
    assert L.pk_adam_step(None, None, None, None, 0, 1, 1e-3, 1.0, 0.999, 1e-8, 1, None) == api.PK_ERR_INVALID_ARG
    assert L.pk_adam_step(None, None, None, None, 0, 1, -1.0, 0.9, 0.999, 1e-8, 1, None) == api.PK_ERR_INVALID_ARG
    assert L.pk_adam_step(None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 0.0, 1, None) == api.PK_ERR_INVALID_ARG
    assert b"eps" in L.pk_last_error()
    # advantages: workspace size grows with the orders; NULL outputs and a small
    # workspace are rejected
    offs = np.array([0, 5, 5, 12], dtype=np.int64)
    p = api.pk_problem(2, 1, 1, 3, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    n = C.c_size_t(0)
    assert L.pk_advantages_workspace_size(C.byref(p), C.byref(n)) == api.PK_OK
    assert n.value >= 12 * 8 + 4 * 8
    assert L.pk_reinforce_advantages(C.byref(p), None, None, 10, None, None, None, 0,
                                     None) == api.PK_ERR_INVALID_ARG
    assert L.pk_reinforce_advantages(C.byref(p), 1, 1, 10, 1, None, 1, 8,
                                     None) == api.PK_ERR_WORKSPACE


def test_capacity_entry_points_validate_on_host():
    """The capacity entry points reject unsupported shapes before any device work."""
    import numpy as np
    from paper_2406_01939_amd import api
    L = api.lib()
    n = C.c_size_t(0)
    offs = np.array([0, 5], dtype=np.int64)
    p = api.pk_problem(4, 2, 3, 1, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert L.pk_capacity_workspace_size(C.byref(p), 1, 0, C.byref(n)) == api.PK_OK
    assert n.value > 5 * 128  # stock rows of up to one (block, SKU) per order
    assert L.pk_capacity_workspace_size(C.byref(p), None, 0, C.byref(n)) == api.PK_ERR_INVALID_ARG
    assert L.pk_capacity_workspace_size(C.byref(p), 1, 256, C.byref(n)) == api.PK_ERR_INVALID_ARG
    wide = api.pk_problem(129, 2, 3, 1, offs.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert L.pk_capacity_workspace_size(C.byref(wide), 1, 0, C.byref(n)) == api.PK_ERR_UNSUPPORTED
    two = np.array([0, 5, 9], dtype=np.int64)
    p2 = api.pk_problem(4, 2, 3, 2, two.ctypes.data, 1, 1, 1, 1, 1, 0)
    assert L.pk_capacity_workspace_size(C.byref(p2), 1, 0, C.byref(n)) == api.PK_ERR_UNSUPPORTED
    passes = C.c_int32(0)
    CP = api.pk_cap_policy
    greedy = CP(0, 1, 0, 0, None, None)
    assert L.pk_picard_simulate_capacity(C.byref(p), 1, C.byref(greedy), 0, 0, None, None, 0, 1,
                                         None, None, C.byref(passes), None, None,
                                         None) == api.PK_ERR_WORKSPACE
    assert L.pk_serial_simulate_capacity(C.byref(p), 1, None, None, 0, 1, None, None,
                                         None) == api.PK_ERR_WORKSPACE
    # policies outside their ranges (checked before the workspace)
    bad = [(CP(1, 0, 0, 0, None, None), b"gamma"), (CP(1001, 1, 0, 0, None, None), b"gamma"),
           (CP(1, 1, -1, 0, None, None), b"gamma_low"), (CP(0, 1, 0, 7, None, None), b"reserved"),
           (CP(1, 1, 0, 0, 1, None), b"bid prices"), (CP(2, 3, 0, 0, None, 1), b"bid prices")]
    for pol, msg in bad:
        assert L.pk_serial_simulate_capacity(C.byref(p), 1, C.byref(pol), None, 0, 1, None, None,
                                             None) == api.PK_ERR_INVALID_ARG
        assert msg in L.pk_last_error()
        assert L.pk_picard_simulate_capacity(C.byref(p), 1, C.byref(pol), 0, 0, None, None, 0, 1,
                                             None, None, C.byref(passes), None, None,
                                             None) == api.PK_ERR_INVALID_ARG
        assert msg in L.pk_last_error()
