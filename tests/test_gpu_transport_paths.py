"""The two transport kernels give the same bits: the z-marching kernel
(closure and wave speeds once per cell, x/y neighbours through LDS, z
neighbours through registers) against the per-cell stencil, for every
boundary condition, both fluxes, both precisions, tile shapes with ragged
rows, tiles and z chunks; and rt_step on either path (fused per-cell head
or transport then chemistry passes) including smoothed RT, inflow faces and
the photon accounting."""
import numpy as np
import pytest
import torch

import rt_inputs as ri
from test_gpu_parity import BCS, C_R, gas, make_pair, random_rad

pytestmark = pytest.mark.gpu

FIELDS = ("N", "F", "xHII", "xHeII", "xHeIII", "T", "nacc", "natt")


def pair(n, bc, M, flux, fp32, seed, empty_frac=0.2, **kw):
    rng = np.random.default_rng(seed)
    N, F = random_rad(n, M, rng, empty_frac=empty_frac)
    st = {"N": N, "F": F, **gas(n, rng)}
    a, _ = make_pair(n, bc, M, flux, fp32=fp32, **kw)
    b, _ = make_pair(n, bc, M, flux, fp32=fp32, **kw)
    a.load_state(st)
    b.load_state(st)
    a.set_transport_path("cell")
    b.set_transport_path("zmarch")
    return a, b, st


SHAPES = [(37, 21, 19), (64, 5, 40), (1, 9, 17), (8, 1, 3), (130, 3, 2), (256, 6, 9)]


@pytest.mark.parametrize("fp32", [True, False])
@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("bc", BCS + [(3, 1, 1, 2, 0, 0)])
def test_zmarch_transport_equals_per_cell(fp32, flux, bc):
    for k, n in enumerate(SHAPES):
        a, b, st = pair(n, bc, 3, flux, fp32, seed=100 + k)
        if bc[0] == 3:
            for ctx in (a, b):
                ctx.set_inflow(0, [1e6, 5e5, 2e5])
        dt = a.courant_dt()
        for rep in range(2):
            a.transport(dt)
            b.transport(dt)
        ga, gb = a.state_numpy(), b.state_numpy()
        print(f"# transport paths n={n} bc={bc} flux={flux} fp32={fp32}", flush=True)
        for key in ("N", "F"):
            assert np.array_equal(ga[key], gb[key]), (n, key)


@pytest.mark.parametrize("fp32", [True, False])
def test_zmarch_handles_tiny_and_subnormal_densities(fp32):
    rng = np.random.default_rng(7)
    n = (40, 11, 13)
    lo, hi = (-44, -30) if fp32 else (-322, -290)
    N = 10.0 ** rng.uniform(lo, hi, (2,) + n[::-1])
    d = rng.normal(size=(2, 3) + n[::-1])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    F = d * rng.uniform(0.9, 1.0, (2, 1) + n[::-1]) * C_R * N[:, None]
    st = {"N": N, "F": np.ascontiguousarray(F), **gas(n, rng)}
    a, _ = make_pair(n, BCS[1], 2, 1, fp32=fp32)
    b, _ = make_pair(n, BCS[1], 2, 1, fp32=fp32)
    for ctx, p in ((a, "cell"), (b, "zmarch")):
        ctx.load_state(st)
        ctx.set_transport_path(p)
        ctx.transport(ctx.courant_dt())
    ga, gb = a.state_numpy(), b.state_numpy()
    assert np.array_equal(ga["N"], gb["N"]) and np.array_equal(ga["F"], gb["F"])


@pytest.mark.parametrize("fp32,smooth", [(True, False), (False, False), (True, True)])
def test_step_paths_equal(fp32, smooth):
    from paper_1304_7126_amd import RTContext
    w = ri.lognormal_box(24, 6.6 * 24 / 128, 8, steps=5, seed=4)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    floor = 1e-12 if smooth else 0.0
    ctxs = []
    for p in ("cell", "zmarch"):
        c = RTContext.for_workload(w, fp32=fp32, counters=True, smooth=smooth, N_floor=floor)
        c.load_state(ri.initial_state(w))
        c.set_sources(ijk, c.source_rates(nd))
        c.set_transport_path(p)
        c.set_accounting(True)
        c.reset_stats()
        ctxs.append(c)
    dt = ctxs[0].courant_dt()
    for c in ctxs:
        c.step(dt, w.steps)
    ga, gb = ctxs[0].state_numpy(), ctxs[1].state_numpy()
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k]), k
    sa, sb = ctxs[0].stats(), ctxs[1].stats()
    for k in ("substeps_total", "attempts_total", "attempts_max", "flags", "substep_hist", "injected"):
        assert sa[k] == sb[k], k
    # the two kernels sum their accounting partials over different blocks
    for k in ("absorbed", "outflow", "photons"):
        assert np.allclose(sa[k], sb[k], rtol=1e-12 if not fp32 else 1e-9, atol=0), k


def test_zmarch_path_refused_where_it_does_not_fit():
    from paper_1304_7126_amd.capi import RTError
    ctx, _ = make_pair((600, 2, 2), BCS[0], 1, 0, fp32=False)
    with pytest.raises(RTError):
        ctx.set_transport_path("zmarch")
    ctx.set_transport_path("auto")
    rng = np.random.default_rng(1)
    N, F = random_rad((600, 2, 2), 1, rng)
    ctx.load_state({"N": N, "F": F, **gas((600, 2, 2), rng)})
    ctx.transport(ctx.courant_dt())
    assert np.all(np.isfinite(ctx.state_numpy()["N"]))
