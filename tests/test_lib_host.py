"""CPU checks of the HIP library: it loads, exports every entry point of
include/rtm1.h, validates its arguments on the host, and its host-side
tables (group attributes, HLL eigenvalues) match the oracle's independent
computations."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import physics
from paper_1304_7126_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "rtm1.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = capi.lib()
    names = header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(capi.EXPORTED)


def test_group_attributes_match_oracle():
    from paper_1304_7126_amd.runtime import group_attributes
    for edges in [(13.6, 24.59, 54.42, np.inf), (13.6, np.inf), (13.6, 24.59, np.inf)]:
        a = group_attributes(1e5, edges)
        b = physics.group_attributes(1e5, edges)
        for x, y in zip(a, b):
            assert np.allclose(x, y, rtol=1e-11, atol=0), (edges, x, y)


def test_hll_table_matches_oracle():
    from paper_1304_7126_amd.runtime import hll_table
    a = hll_table()
    b = oracle.hll_table()
    assert a.shape == b.shape == (101, 101, 2)
    assert np.max(np.abs(a - b)) < 1e-12


def _init(**over):
    L = capi.lib()
    g = capi.RtGrid()
    g.nx, g.ny, g.nz, g.dx = 8, 8, 8, 1e20
    for i in range(6):
        g.bc[i] = 0
    gr = capi.RtGroups()
    gr.M, gr.c_r = 1, 3e8
    p = capi.RtParams()
    p.flux, p.otsa, p.isothermal, p.prec = 0, 1, 0, 0
    p.X, p.Y, p.gamma, p.a_exp, p.x_min, p.N_floor, p.max_attempts = 0.76, 0.24, 5 / 3, 1.0, 1e-6, 0.0, 100
    for k, v in over.items():
        for obj in (g, gr, p):
            if hasattr(obj, k):
                setattr(obj, k, v)
    h = ctypes.c_void_p()
    rc = L.rt_init(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(p), ctypes.byref(h))
    return rc, h, L.rt_last_error(None).decode()


@pytest.mark.parametrize("over,code", [
    (dict(nx=0), capi.RT_EINVAL), (dict(dx=-1.0), capi.RT_EINVAL), (dict(M=4), capi.RT_EINVAL),
    (dict(M=0), capi.RT_EINVAL), (dict(c_r=0.0), capi.RT_EINVAL), (dict(flux=2), capi.RT_EINVAL),
    (dict(otsa=2), capi.RT_EINVAL), (dict(prec=3), capi.RT_EINVAL), (dict(X=0.0), capi.RT_EINVAL),
    (dict(gamma=1.0), capi.RT_EINVAL), (dict(x_min=0.0), capi.RT_EINVAL), (dict(max_attempts=0), capi.RT_EINVAL),
    (dict(smooth=2), capi.RT_EINVAL), (dict(otsa=0, brec=(ctypes.c_int * 3)(0, 1, 0)), capi.RT_EINVAL),
    (dict(otsa=0, brec=(ctypes.c_int * 3)(-2, 0, 0)), capi.RT_EINVAL),
])
def test_init_rejects_invalid_arguments(over, code):
    rc, h, msg = _init(**over)
    assert rc == code and not h.value and msg


def test_init_rejects_one_sided_periodic():
    L = capi.lib()
    g = capi.RtGrid()
    g.nx = g.ny = g.nz = 4
    g.dx = 1.0
    for i, b in enumerate((0, 1, 0, 0, 0, 0)):
        g.bc[i] = b
    gr = capi.RtGroups()
    gr.M, gr.c_r = 1, 1.0
    p = capi.RtParams()
    p.otsa, p.X, p.gamma, p.x_min, p.max_attempts, p.a_exp = 1, 1.0, 5 / 3, 1e-6, 10, 1.0
    h = ctypes.c_void_p()
    assert L.rt_init(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(p), ctypes.byref(h)) == capi.RT_EINVAL
    assert b"periodic" in L.rt_last_error(None)


def test_group_attributes_rejects_bad_edges():
    L = capi.lib()
    e = np.array([24.59, 13.6])
    out = [np.zeros(9), np.zeros(9), np.zeros(3), np.zeros(3)]
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.rt_group_attributes(1e5, 1, dp(e), *[dp(o) for o in out]) == capi.RT_EINVAL


def test_null_context_calls_fail_cleanly():
    L = capi.lib()
    assert L.rt_step(None, 1.0, 1) == capi.RT_EINVAL
    assert L.rt_transport(None, 1.0) == capi.RT_EINVAL
    assert L.rt_current(None) == -1
    L.rt_free(None)
