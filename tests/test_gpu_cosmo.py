"""GPU parity of super-comoving RT variables (Sec. 5.4; rt_set_expansion)
through the C ABI against the oracle, which converts to physical variables
and steps cells of width a dx.

  - one and several steps of random states with sources at a = 0.3 and
    a = 0.05 (GLF and HLL, plain and smoothed, FP64 and FP32 transport);
  - a run that changes a between steps matches the oracle run doing the
    same; setting a back to 1 gives the static step bit for bit;
  - the Courant step scales with a, and the photon budget closes in
    comoving photon counts;
  - the adjoint refuses a != 1, and a must be positive.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri
from gpu_util import assert_close, rel_err
from test_gpu_parity import BCS, chem_compare, gas, make_pair, random_rad

pytestmark = pytest.mark.gpu


def loaded(n, bc, M, flux, seed, a, fp32=False, smooth=False):
    rng = np.random.default_rng(seed)
    ctx, o = make_pair(n, bc, M, flux, fp32=fp32, smooth=smooth, N_floor=1e-12 if smooth else 0.0)
    N, F = random_rad(n, M, rng)
    gs = gas(n, rng)
    # super-comoving state: a^3 N, a^4 F, a^3 n_H
    st = {"N": N * a ** 3, "F": F * a ** 4, **gs}
    st["nH"] = gs["nH"] * a ** 3
    if fp32:
        st["N"] = st["N"].astype(np.float32).astype(np.float64)
        st["F"] = st["F"].astype(np.float32).astype(np.float64)
    ctx.load_state(st)
    ctx.set_expansion(a)
    ijk = np.array([[1, 2, 3], [n[0] - 1, 0, n[2] // 2]], np.int32)
    nd = 10 ** rng.uniform(47, 49, len(ijk))
    ctx.set_sources(ijk, ctx.source_rates(nd))
    return ctx, o, st, ijk, nd


@pytest.mark.parametrize("a", [0.3, 0.05])
@pytest.mark.parametrize("flux,smooth", [(0, False), (1, False), (1, True)])
def test_one_step_matches_oracle(a, flux, smooth):
    n = (25, 12, 9)
    ctx, o, st, ijk, nd = loaded(n, BCS[1], 3, flux, seed=300 + flux, a=a, smooth=smooth)
    dt = ctx.courant_dt()
    assert dt == pytest.approx(o.courant_dt(0.8, a), rel=1e-15)
    ctx.step(dt, 1)
    fl, nacc, natt = o.step(st, dt, ijk, o.source_rates(nd), want_counts=True, smooth=smooth, a=a)
    st["nacc"], st["natt"] = nacc, natt
    g = ctx.state_numpy()
    chem_compare(g, st)
    same = (g["nacc"] == nacc) & (g["natt"] == natt)
    for gi in range(3):
        assert_close(g["F"][gi], st["F"][gi], 1e-10, 1e-13, f"F[{gi}]", mask=same)


def test_changing_expansion_matches_oracle():
    n = (21, 10, 8)
    a0 = 0.2
    ctx, o, st, ijk, nd = loaded(n, BCS[0], 2, 0, seed=310, a=a0)
    ondot = o.source_rates(nd)
    a = a0
    for k in range(6):
        dt = ctx.courant_dt()
        ctx.step(dt, 1)
        o.step(st, dt, ijk, ondot, a=a)
        a *= 1.15
        ctx.set_expansion(a)
    g = ctx.state_numpy()
    for key in ("xHII", "xHeII", "xHeIII", "T"):
        assert rel_err(g[key], st[key]) < 1e-9, (key, rel_err(g[key], st[key]))
    for gi in range(2):
        assert rel_err(g["N"][gi], st["N"][gi]) < 1e-9
        assert rel_err(g["F"][gi], st["F"][gi]) < 1e-9


def test_fp32_transport_against_fp64_oracle():
    n = (23, 11, 9)
    a = 0.25
    ctx, o, st, ijk, nd = loaded(n, BCS[2], 3, 1, seed=320, a=a, fp32=True)
    dt = ctx.courant_dt()
    ctx.step(dt, 1)
    o.step(st, dt, ijk, o.source_rates(nd), a=a)
    g = ctx.state_numpy()
    for gi in range(3):
        assert rel_err(g["N"][gi], st["N"][gi]) < 1e-5
    assert rel_err(g["xHII"], st["xHII"]) < 1e-4


def test_back_to_one_is_the_static_step():
    n = (17, 9, 7)
    runs = []
    for detour in (False, True):
        rng = np.random.default_rng(330)
        ctx, o = make_pair(n, BCS[0], 2, 1)
        N, F = random_rad(n, 2, rng)
        ctx.load_state({"N": N, "F": F, **gas(n, rng)})
        if detour:
            ctx.set_expansion(0.3)
            ctx.set_expansion(1.0)
        ctx.step(ctx.courant_dt(), 3)
        runs.append(ctx.state_numpy())
    for k in ("N", "F", "xHII", "T", "nacc", "natt"):
        assert np.array_equal(runs[0][k], runs[1][k]), k


@pytest.mark.parametrize("fp32", [False, True])
def test_budget_closes(fp32):
    ctx, o, st, ijk, nd = loaded((19, 17, 13), BCS[1], 3, 1, seed=340, a=0.4, fp32=fp32)
    ctx.set_accounting(True)
    ctx.reset_stats()
    p0 = np.array(ctx.stats()["photons"])
    dt = ctx.courant_dt()
    ctx.step(dt, 12)
    s = ctx.stats()
    p1 = np.array(s["photons"])
    inj, ab, out = (np.array(s[k]) for k in ("injected", "absorbed", "outflow"))
    resid = p1 - (p0 + inj - ab - out)
    tol = 1e-5 if fp32 else 1e-12
    assert np.all(np.abs(resid) <= tol * (p0 + inj)), resid / (p0 + inj)
    assert np.all(out != 0)


def test_refusals():
    from paper_1304_7126_amd import RTContext, capi
    from paper_1304_7126_amd.capi import RTError, lib
    ctx, o = make_pair((8, 8, 8), BCS[0], 1, 0, X=1.0, Y=0.0)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(RTError, match="positive"):
            ctx.set_expansion(bad)
    ctx.set_expansion(0.5)
    dt = ctx.courant_dt()
    nc = 512
    counts = torch.zeros(nc, dtype=torch.int32, device="cuda")
    off = torch.empty(int(lib().rt_tape_offsets_len(ctx._h)), dtype=torch.int64, device="cuda")
    Na = torch.empty(nc, dtype=torch.float64, device="cuda")
    Fa = torch.empty(3 * nc, dtype=torch.float64, device="cuda")
    tr = torch.empty(7 * nc, dtype=torch.float64, device="cuda")
    t = capi.RtTape(Na.data_ptr(), Fa.data_ptr(), counts.data_ptr(), off.data_ptr(), tr.data_ptr(), nc)
    assert lib().rt_step_record(ctx._h, dt, ctypes.byref(t)) == capi.RT_EUNSUPPORTED
    # the transport refuses a step above a dx / (3 c_r)
    with pytest.raises(RTError, match="Courant"):
        ctx.transport(ctx.courant_dt(1.0) * 1.01)
