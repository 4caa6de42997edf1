"""GPU parity without the on-the-spot approximation (Sec. 3.3.2; rt_params.otsa
= 0): case A recombination and recombination cooling, and the photons of
recombinations straight to the ground state added to the group rt_groups.brec
holds for each species (eq. cool_N_cr), through the C ABI against the oracle.

  - one fused rt_step on random states with sources, 1-3 groups (one grey
    group takes every species' photons; three groups take one species each),
    hydrogen-only and H+He, isothermal and with T evolving, GLF and HLL, and
    combined with smoothed RT;
  - split calls equal the fused step bit for bit;
  - forty steps of the Stromgren test and six of a lognormal H+He box;
  - the photon budget closes (the chemistry's net absorption counts the
    emission);
  - an out-of-range group map, the batch and the adjoint are refused.
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


def loaded(n, bc, M, flux, seed, isothermal=False, Y=0.24, smooth=False, fp32=False):
    rng = np.random.default_rng(seed)
    X = 1.0 if Y == 0 else 0.76
    ctx, o = make_pair(n, bc, M, flux, isothermal=isothermal, X=X, Y=Y, otsa=False, smooth=smooth,
                       N_floor=1e-12 if smooth else 0.0, fp32=fp32)
    N, F = random_rad(n, M, rng)
    gs = gas(n, rng)
    if Y == 0:
        gs["xHeII"][:] = 0
        gs["xHeIII"][:] = 0
    if fp32:
        N = N.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    st = {"N": N, "F": F, **gs}
    ctx.load_state(st)
    ijk = np.array([[1, 2, 3], [n[0] - 1, 0, n[2] // 2]], np.int32)
    nd = 10 ** rng.uniform(47, 49, len(ijk))
    ctx.set_sources(ijk, ctx.source_rates(nd))
    return ctx, o, st, ijk, nd


CASES = [(1, 0, BCS[0], True, 0.0, False), (3, 1, BCS[1], False, 0.24, False), (2, 0, BCS[2], False, 0.24, False),
         (1, 1, BCS[2], False, 0.24, False), (3, 0, BCS[0], False, 0.24, True), (1, 0, BCS[1], True, 0.0, True)]


@pytest.mark.parametrize("M,flux,bc,iso,Y,smooth", CASES)
def test_one_step_matches_oracle(M, flux, bc, iso, Y, smooth):
    n = (29, 13, 11)
    ctx, o, st, ijk, nd = loaded(n, bc, M, flux, seed=100 + 7 * M + flux, isothermal=iso, Y=Y, smooth=smooth)
    dt = ctx.courant_dt()
    ctx.step(dt, 1)
    fl, nacc, natt = o.step(st, dt, ijk, o.source_rates(nd), want_counts=True, smooth=smooth)
    st["nacc"], st["natt"] = nacc, natt
    g = ctx.state_numpy()
    chem_compare(g, st)
    same = (g["nacc"] == nacc) & (g["natt"] == natt)
    for gi in range(M):
        assert_close(g["F"][gi], st["F"][gi], 1e-10, 1e-13, f"F[{gi}]", mask=same)
    assert (ctx.stats()["flags"] & ~1) == (fl & ~1)


def test_emission_reaches_the_mapped_groups():
    # hot ionised H + He without absorption: the step adds exactly the
    # oracle's emission to each group (1 group: all species; 3: one each)
    for M in (1, 3):
        n = (9, 8, 7)
        rng = np.random.default_rng(110 + M)
        ctx, o = make_pair(n, BCS[0], M, 0, isothermal=True, otsa=False)
        zero = {"N": np.zeros((M,) + n[::-1]), "F": np.zeros((M, 3) + n[::-1])}
        gs = gas(n, rng)
        gs["T"][:] = 6e4
        st = {**zero, **gs}
        ctx.load_state(st)
        dt = ctx.courant_dt()
        ctx.thermochem(dt)
        o.thermochem(st, dt)
        g = ctx.state_numpy()
        assert np.all(st["N"] > 0) if M == 1 else np.all(st["N"][2] > 0)
        for gi in range(M):
            assert_close(g["N"][gi], st["N"][gi], 1e-10, 1e-14, f"N[{gi}]")


def _lognormal(otsa, smooth=False, fp32=False, n=20, seed=4, steps=3):
    from paper_1304_7126_amd import RTContext
    w = ri.lognormal_box(n, 6.6 * n / 128, 5, steps=steps, seed=seed, flux=ri.FLUX_HLL)
    w.otsa = otsa
    st = ri.initial_state(w)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ctx = RTContext.for_workload(w, fp32=fp32, counters=True, smooth=smooth, N_floor=1e-12 if smooth else 0.0)
    ctx.load_state(st)
    ctx.set_sources(ijk, ctx.source_rates(nd))
    return ctx, w, st, ijk, nd


@pytest.mark.parametrize("fp32,smooth", [(False, False), (True, False), (False, True)])
def test_split_calls_equal_the_fused_step(fp32, smooth):
    a, w, *_ = _lognormal(False, smooth, fp32)
    b, *_ = _lognormal(False, smooth, fp32)
    dt = a.courant_dt()
    for _ in range(w.steps):
        a.step(dt, 1)
        b.inject(dt)
        b.transport(dt)
        b.thermochem(dt)
    ga, gb = a.state_numpy(), b.state_numpy()
    for k in ("N", "F", "xHII", "xHeII", "xHeIII", "T", "nacc", "natt"):
        assert np.array_equal(ga[k], gb[k]), k


def test_lognormal_steps_match_oracle():
    ctx, w, st, ijk, nd = _lognormal(False, steps=6, n=24, seed=5)
    o = oracle.OracleRT.for_workload(w)
    ondot = o.source_rates(nd)
    dt = ctx.courant_dt()
    for _ in range(w.steps):
        ctx.step(dt, 1)
        o.step(st, dt, ijk, ondot)
    g = ctx.state_numpy()
    for k in ("xHII", "xHeII", "xHeIII", "T"):
        assert rel_err(g[k], st[k]) < 1e-9, (k, rel_err(g[k], st[k]))
    for gi in range(w.spectrum.M):
        assert rel_err(g["N"][gi], st["N"][gi]) < 1e-9
        assert rel_err(g["F"][gi], st["F"][gi]) < 1e-9


def test_stromgren_steps_match_oracle():
    from paper_1304_7126_amd import RTContext
    w = ri.stromgren_32(40)
    w.otsa = False
    assert w.brec == (0, -1, -1)
    ijk, nd = ri.workload_sources(w)
    ctx = RTContext.for_workload(w, counters=True)
    ctx.load_state(ri.initial_state(w))
    ctx.set_sources(ijk, ctx.source_rates(nd))
    ctx.step(ctx.courant_dt(), w.steps)
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    ondot = o.source_rates(nd)
    dt = o.courant_dt()
    for _ in range(w.steps):
        o.step(st, dt, ijk, ondot)
    g = ctx.state_numpy()
    for k in ("xHII", "T"):
        assert rel_err(g[k], st[k]) < 1e-10, k
    assert rel_err(1 - g["xHII"], 1 - st["xHII"]) < 1e-9
    assert rel_err(g["N"], st["N"]) < 1e-10
    assert rel_err(g["F"], st["F"]) < 1e-10


@pytest.mark.parametrize("fp32", [False, True])
def test_photon_budget_closes(fp32):
    ctx, o, st, ijk, nd = loaded((19, 17, 13), BCS[1], 3, 1, seed=120, fp32=fp32)
    ctx.set_accounting(True)
    ctx.reset_stats()
    p0 = np.array(ctx.stats()["photons"])
    dt = ctx.courant_dt()
    ctx.step(dt, 15)
    s = ctx.stats()
    p1 = np.array(s["photons"])
    inj, ab, out = (np.array(s[k]) for k in ("injected", "absorbed", "outflow"))
    resid = p1 - (p0 + inj - ab - out)
    tol = 1e-5 if fp32 else 1e-12
    assert np.all(np.abs(resid) <= tol * (p0 + inj)), resid / (p0 + inj)


def test_bad_group_map_batch_and_adjoint_are_refused():
    from paper_1304_7126_amd import RTContext, capi
    from paper_1304_7126_amd.capi import RTError, lib
    from paper_1304_7126_amd.runtime import spectrum_attributes
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV=ri.EDGES_2)
    sN, sE, eb, fr = spectrum_attributes(spec)
    kw = dict(n=(8, 8, 8), dx=1e20, bc=BCS[0], M=2, c_r=ri.C_LIGHT / 100, sigN=sN, sigE=sE, ebar=eb)
    with pytest.raises(RTError, match="brec"):
        RTContext(**kw, otsa=False, brec=(0, 2, 1))
    RTContext(**kw, otsa=True, brec=(0, 2, 1))  # ignored with OTSA
    ctx = RTContext(**{**kw, "M": 1}, otsa=False, brec=(0, 0, 0), X=1.0, Y=0.0, counters=True)
    ctx.group_frac = np.ones(1)
    dt = ctx.courant_dt()
    nc = 512
    counts = torch.zeros(nc, dtype=torch.int32, device="cuda")
    off = torch.empty(int(lib().rt_tape_offsets_len(ctx._h)), dtype=torch.int64, device="cuda")
    Na = torch.empty(nc, dtype=torch.float64, device="cuda")
    Fa = torch.empty(3 * nc, dtype=torch.float64, device="cuda")
    tr = torch.empty(7 * nc, dtype=torch.float64, device="cuda")
    t = capi.RtTape(Na.data_ptr(), Fa.data_ptr(), counts.data_ptr(), off.data_ptr(), tr.data_ptr(), nc)
    assert lib().rt_step_record(ctx._h, dt, ctypes.byref(t)) == capi.RT_EUNSUPPORTED
    from paper_1304_7126_amd.batch import RTBatch
    z = np.zeros((3, 3))
    with pytest.raises(RTError, match="otsa"):
        RTBatch([((8, 8, 8), 1e20, BCS[0])], [(1, ri.C_LIGHT / 100, z, z, np.zeros(3))], otsa=False)
