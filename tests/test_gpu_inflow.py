"""GPU parity of boundary-flux sources (RT_BC_INFLOW faces, rt_set_inflow:
the x = 0 source of Iliev test 3, Sec. 6) and of the HLL flux limit, through
the C ABI against the oracle.

  - one transport step on random states with inflow faces on low and high
    faces of every axis, GLF and HLL, FP64 (and FP32 to its tolerance);
  - an empty box fills with the beam and stays there (HLL, FP64 and FP32);
  - steps of the shadow-clump test (Iliev test 3 on a uniform grid) equal
    the oracle's, the clump casts its shadow at 1 Myr, and at 128^3 (the
    paper's resolution) sampled cells equal the oracle's;
  - the photon budget closes with the inflow counted as negative outflow;
  - rt_set_inflow refuses other faces and bad fluxes.
"""
import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri
from gpu_util import assert_close, rel_err
from test_gpu_parity import C_R, gas, random_rad

pytestmark = pytest.mark.gpu

BC_IN = [(3, 1, 0, 0, 2, 3), (1, 3, 3, 2, 0, 0), (3, 3, 3, 3, 3, 3)]


def pair(n, bc, M, flux, fp32=False, rng=None, c_r=C_R):
    from paper_1304_7126_amd import RTContext
    from paper_1304_7126_amd.runtime import spectrum_attributes
    from oracle import physics
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV={1: ri.EDGES_1, 2: ri.EDGES_2, 3: ri.EDGES_3}[M])
    sN, sE, eb, fr = spectrum_attributes(spec)
    dx = 6.6 * ri.KPC / 64
    inflow = np.zeros((6, M))
    for f in range(6):
        if bc[f] == 3:
            inflow[f] = (10 ** rng.uniform(5, 7)) * fr[:M] / fr[:M].sum()
    ctx = RTContext(n=n, dx=dx, bc=bc, M=M, c_r=c_r, sigN=sN, sigE=sE, ebar=eb, flux=flux, fp32=fp32,
                    counters=True)
    ctx.group_frac = fr[:M]
    for f in range(6):
        if bc[f] == 3:
            ctx.set_inflow(f, inflow[f])
    osN, osE, oeb, ofr = physics.spectrum_attributes(spec)
    o = oracle.OracleRT(n=n, dx=dx, bc=bc, M=M, c_r=c_r, sigN=osN, sigE=osE, ebar=oeb, flux=flux, inflow=inflow)
    return ctx, o, inflow


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("bc", BC_IN)
def test_transport_with_inflow_faces_fp64(flux, bc):
    rng = np.random.default_rng(200 + flux)
    n = (23, 14, 11)
    ctx, o, _ = pair(n, bc, 3, flux, rng=rng)
    N, F = random_rad(n, 3, rng)
    st = {"N": N, "F": F, **gas(n, rng)}
    ctx.load_state(st)
    dt = ctx.courant_dt()
    ctx.transport(dt)
    o.transport(st, dt)
    g = ctx.state_numpy()
    for gi in range(3):
        assert_close(g["N"][gi], st["N"][gi], 1e-12, 1e-14, f"N[{gi}]")
        assert_close(g["F"][gi], st["F"][gi], 1e-12, 1e-14, f"F[{gi}]")
    for _ in range(2):
        ctx.transport(dt)
        o.transport(st, dt)
    g = ctx.state_numpy()
    # Later steps start from states both sides computed: HLL near a beam
    # almost parallel to a face has both wave speeds near zero, where the
    # weights lp/(lp - lm) magnify ulp differences of the speeds, so a flux
    # component that is small against the local radiation (c_r N) is
    # compared on the scale of the field
    for gi in range(3):
        assert_close(g["N"][gi], st["N"][gi], 1e-11, 1e-13, f"N[{gi}]")
        assert_close(g["F"][gi], st["F"][gi], 1e-11, 1e-12, f"F[{gi}]")


@pytest.mark.parametrize("flux", [0, 1])
def test_transport_with_inflow_faces_fp32(flux):
    rng = np.random.default_rng(210 + flux)
    n = (21, 12, 9)
    ctx, o, _ = pair(n, BC_IN[0], 2, flux, fp32=True, rng=rng)
    N, F = random_rad(n, 2, rng, empty_frac=0.0)
    N = N.astype(np.float32).astype(np.float64)
    F = F.astype(np.float32).astype(np.float64)
    st = {"N": N, "F": F, **gas(n, rng)}
    ctx.load_state(st)
    dt = ctx.courant_dt()
    ctx.transport(dt)
    o.transport(st, dt)
    g = ctx.state_numpy()
    for gi in range(2):
        assert rel_err(g["N"][gi], st["N"][gi]) < 1e-5
        for d in range(3):
            assert rel_err(g["F"][gi, d], st["F"][gi, d]) < 1e-5


@pytest.mark.parametrize("fp32", [False, True])
def test_empty_box_fills_with_the_beam(fp32):
    from paper_1304_7126_amd import RTContext
    z = np.zeros((3, 3))
    c_r = ri.C_LIGHT / 10
    ctx = RTContext(n=(12, 4, 4), dx=0.1 * ri.KPC, bc=(3, 1, 0, 0, 0, 0), M=1, c_r=c_r, sigN=z, sigE=z,
                    ebar=np.zeros(3), flux=1, fp32=fp32)
    ctx.group_frac = np.ones(1)
    ctx.set_inflow(0, [1e6])
    shp = (4, 4, 12)
    ctx.load_state({"N": np.zeros((1,) + shp), "F": np.zeros((1, 3) + shp), **gas((12, 4, 4),
                                                                                np.random.default_rng(0))})
    dt = ctx.courant_dt()
    ctx.step(dt, 800)
    g = ctx.state_numpy()
    tol = 1e-5 if fp32 else 1e-12
    assert np.allclose(g["N"][0], 1e6 / c_r, rtol=tol, atol=0), (g["N"][0].min() * c_r, g["N"][0].max() * c_r)
    assert np.allclose(g["F"][0, 0], 1e6, rtol=tol, atol=0)
    assert np.max(np.abs(g["F"][0, 1:])) <= tol * 1e6


def test_shadow_clump_steps_match_oracle_and_cast_the_shadow():
    from paper_1304_7126_amd import RTContext
    w = ri.shadow_clump(32)
    ctx = RTContext.for_workload(w, counters=True)
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    ctx.load_state(st)
    dt = ctx.courant_dt()
    assert dt == o.courant_dt()
    for _ in range(60):
        ctx.step(dt, 1)
        o.step(st, dt)
    g = ctx.state_numpy()
    for k in ("xHII", "T"):
        assert rel_err(g[k], st[k]) < 1e-9, (k, rel_err(g[k], st[k]))
    assert rel_err(1 - g["xHII"], 1 - st["xHII"]) < 1e-8
    for gi in range(3):
        assert rel_err(g["N"][gi], st["N"][gi]) < 1e-9
        assert rel_err(g["F"][gi], st["F"][gi]) < 1e-9
    # on to 1 Myr on the GPU alone: the clump's shadow
    steps = int(round(3.15576e13 / dt))
    ctx.step(dt, steps - 60)
    g = ctx.state_numpy()
    dx = w.dx

    def x_at(x_kpc, y_kpc, z_kpc):
        i, j, k = (int(v * ri.KPC / dx) for v in (x_kpc, y_kpc, z_kpc))
        return g["xHII"][k, j, i]

    assert x_at(2.0, 3.3, 3.3) > 0.9 and x_at(5.0, 3.3, 3.3) < 0.01
    assert x_at(6.3, 3.3, 3.3) < 0.1 and x_at(6.3, 1.0, 3.3) > 0.9


def test_shadow_clump_128_sampled_cells_match_oracle():
    from paper_1304_7126_amd import RTContext
    from test_gpu_fullsize import host_state
    w = ri.shadow_clump(128)
    ctx = RTContext.for_workload(w, counters=True)
    ctx.load_state(ri.initial_state(w))
    dt = ctx.courant_dt()
    ctx.step(dt, 300)
    pre = host_state(ctx)
    ctx.step(dt, 1)
    g = ctx.state_numpy()
    o = oracle.OracleRT.for_workload(w)
    rng = np.random.default_rng(1)
    nc = w.ncell
    # random cells, the inflow face and the light front's neighbourhood
    front = np.flatnonzero((pre["N"][0].ravel() > 0) & (pre["N"][0].ravel() < 0.5 * pre["N"][0].max()))
    cells = np.unique(np.concatenate([rng.integers(0, nc, 2048), np.arange(0, nc, 128)[:2048],
                                      rng.choice(front, 1024)]))
    r = o.step_cells(pre, dt, cells)
    M = w.spectrum.M
    same = (g["nacc"].ravel()[cells] == r["nacc"]) & (g["natt"].ravel()[cells] == r["natt"])
    assert 1 - same.mean() <= 5e-3
    gN = g["N"].reshape(M, -1)[:, cells].T
    gx = g["xHII"].ravel()[cells]
    for gi in range(M):
        sc = np.max(np.abs(r["N"][:, gi]))
        assert np.all(np.abs(gN[same, gi] - r["N"][same, gi]) <= 1e-10 * np.abs(r["N"][same, gi]) + 1e-13 * sc)
    assert np.all(np.abs(gx[same] - r["x"][same, 0]) <= 1e-10 * r["x"][same, 0] + 1e-15)


@pytest.mark.parametrize("fp32", [False, True])
def test_budget_counts_the_inflow(fp32):
    from paper_1304_7126_amd import RTContext
    w = ri.shadow_clump(24)
    ctx = RTContext.for_workload(w, fp32=fp32)
    ctx.load_state(ri.initial_state(w))
    ctx.set_accounting(True)
    ctx.reset_stats()
    dt = ctx.courant_dt()
    ctx.step(dt, 40)
    s = ctx.stats()
    p1 = np.array(s["photons"])
    ab, out = np.array(s["absorbed"]), np.array(s["outflow"])
    # nothing in the box at the start and no point sources: what is there
    # came in through the x = 0 face (negative outflow) and was not absorbed
    assert np.all(out < 0)
    resid = p1 - (0.0 - ab - out)
    assert np.all(np.abs(resid) <= (1e-5 if fp32 else 1e-12) * np.abs(out)), resid / out
    # the face lets in at most F A dt per step (all of it while the first
    # cells are empty of absorbers' photons)
    A = (w.n[1] * w.dx) * (w.n[2] * w.dx)
    fr = ctx.group_frac / ctx.group_frac.sum()
    assert np.all(-out <= 1e6 * fr * A * dt * 40 * (1 + 1e-9))


def test_set_inflow_refusals():
    from paper_1304_7126_amd import RTContext
    from paper_1304_7126_amd.capi import RTError
    z = np.zeros((3, 3))
    ctx = RTContext(n=(4, 4, 4), dx=1e20, bc=(3, 1, 1, 1, 1, 1), M=1, c_r=C_R, sigN=z, sigE=z, ebar=np.zeros(3))
    with pytest.raises(RTError, match="not an RT_BC_INFLOW"):
        ctx.set_inflow(1, [1e6])
    with pytest.raises(RTError, match="finite"):
        ctx.set_inflow(0, [-1.0])
    with pytest.raises(RTError, match="finite"):
        ctx.set_inflow(0, [np.nan])
    ctx.set_inflow(0, [0.0])
