"""GPU tests of the photon accounting (rt_set_accounting): per group the
photons injected, absorbed by the chemistry and carried out through the
boundary faces, and the histogram of accepted substeps.

  - budget: photons(t) = photons(t0) + injected - absorbed - outflow over
    many steps, for outflow/reflecting and periodic grids, FP64 and FP32
    transport (the operator split of Sec. 3 has no other source or sink);
  - one step against the oracle: absorbed = sum over cells of the photons
    entering minus leaving the chemistry, outflow = photons lost by the
    transport, histogram = the oracle's accepted-substep counts;
  - the fused step, the split calls and repeated runs give identical sums;
  - every field of rt_get_stats against the oracle's step ledger over
    several steps (photons, ionised hydrogen, largest reduced flux, smallest
    density, injected, absorbed, outflow, substep histogram and totals).
"""
import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri
from test_gpu_parity import BCS, gas, make_pair, random_rad

pytestmark = pytest.mark.gpu


def loaded(n, bc, M, flux, fp32=False, seed=3):
    rng = np.random.default_rng(seed)
    ctx, o = make_pair(n, bc, M, flux, fp32=fp32)
    N, F = random_rad(n, M, rng, empty_frac=0.0)
    st = {"N": N, "F": F, **gas(n, rng)}
    ctx.load_state(st)
    ijk = np.array([[1, 2, 3], [n[0] - 1, 0, n[2] // 2], [1, 2, 3]], np.int32)
    nd = np.array([3e48, 1e49, 2e47])
    ctx.set_sources(ijk, ctx.source_rates(nd))
    return ctx, o, st, ijk, nd


@pytest.mark.parametrize("bc", [BCS[1], BCS[2], BCS[0]])
@pytest.mark.parametrize("fp32", [False, True])
def test_budget_closes_over_many_steps(bc, fp32):
    n = (19, 17, 13)
    ctx, o, st, ijk, nd = loaded(n, bc, 3, 1, fp32=fp32)
    ctx.set_accounting(True)
    ctx.reset_stats()
    p0 = np.array(ctx.stats()["photons"])
    dt = ctx.courant_dt()
    ctx.step(dt, 25)
    s = ctx.stats()
    p1 = np.array(s["photons"])
    inj, ab, out = (np.array(s[k]) for k in ("injected", "absorbed", "outflow"))
    # injected photons are the host sum of rate x dt
    rates = ctx.source_rates(nd)
    assert np.allclose(inj, rates.sum(axis=0) * dt * 25, rtol=1e-14, atol=0)
    scale = p0 + inj
    resid = p1 - (p0 + inj - ab - out)
    # FP32 transport: every cell's update and injection rounds to FP32 once
    # per step; FP64: rounding of the sums only
    tol = 1e-5 if fp32 else 1e-12
    assert np.all(np.abs(resid) <= tol * scale), (resid / scale)
    assert np.all(ab > 0)
    if bc == BCS[0]:
        assert np.all(out == 0.0)  # periodic: no boundary faces
    else:
        assert np.all(out != 0.0)
    # the histogram counts every cell of every step
    h = np.array(s["substep_hist"])
    assert h.sum() == 25 * np.prod(n)
    if h[63] == 0:
        assert (h * np.arange(64)).sum() == s["substeps_total"]


def test_one_step_matches_oracle():
    n = (23, 11, 9)
    ctx, o, st, ijk, nd = loaded(n, BCS[2], 3, 0)
    ctx.set_accounting(True)
    ctx.reset_stats()
    dt = ctx.courant_dt()
    ctx.step(dt, 1)
    s = ctx.stats()
    V = ctx.dx ** 3
    o.inject(st, dt, ijk, o.source_rates(nd))
    n_inj = st["N"].sum(axis=(1, 2, 3)) * V
    o.transport(st, dt)
    n_tr = st["N"].sum(axis=(1, 2, 3)) * V
    _, nacc, _ = o.thermochem(st, dt, want_counts=True)
    n_ch = st["N"].sum(axis=(1, 2, 3)) * V
    assert np.allclose(s["absorbed"], n_tr - n_ch, rtol=1e-10, atol=1e-13 * n_tr.max())
    assert np.allclose(s["outflow"], n_inj - n_tr, rtol=1e-9, atol=1e-12 * n_inj.max())
    h = np.bincount(np.minimum(nacc.ravel(), 63), minlength=64)
    assert np.array_equal(np.array(s["substep_hist"]), h)


def test_split_calls_and_repeats_give_identical_sums():
    n = (21, 13, 11)
    sums = []
    for mode in ("fused", "split", "fused"):
        ctx, o, st, ijk, nd = loaded(n, BCS[1], 2, 1, seed=9)
        ctx.set_accounting(True)
        ctx.reset_stats()
        dt = ctx.courant_dt()
        for _ in range(4):
            if mode == "fused":
                ctx.step(dt, 1)
            else:
                ctx.inject(dt)
                ctx.transport(dt)
                ctx.thermochem(dt)
        s = ctx.stats()
        sums.append((s["injected"], s["absorbed"], s["outflow"], s["substep_hist"], s["photons"]))
    assert sums[0] == sums[2]
    assert sums[0] == sums[1]


def test_chemistry_alone_is_accounted_and_off_means_zero():
    n = (16, 8, 8)
    ctx, o, st, ijk, nd = loaded(n, BCS[0], 1, 0)
    ctx.reset_stats()
    dt = ctx.courant_dt()
    ctx.step(dt, 2)  # accounting off
    s = ctx.stats()
    assert s["absorbed"] == [0.0] and s["outflow"] == [0.0] and s["injected"] == [0.0]
    assert sum(s["substep_hist"]) == 0
    ctx.set_accounting(True)
    p0 = ctx.stats()["photons"][0]
    ctx.thermochem(dt)
    s = ctx.stats()
    assert abs(s["absorbed"][0] - (p0 - s["photons"][0])) <= 1e-13 * p0
    assert sum(s["substep_hist"]) == np.prod(n)


@pytest.mark.parametrize("bc,flux,fp32", [(BCS[2], 1, False), (BCS[1], 0, False), (BCS[0], 1, False),
                                          (BCS[2], 1, True)])
def test_stats_match_oracle_ledger(bc, flux, fp32):
    n = (19, 17, 13)
    ctx, o, st, ijk, nd = loaded(n, bc, 3, flux, fp32=fp32, seed=21)
    if fp32:
        # the oracle starts from the values the FP32 state holds
        st["N"] = st["N"].astype(np.float32).astype(np.float64)
        st["F"] = st["F"].astype(np.float32).astype(np.float64)
        ctx.load_state(st)
    ctx.set_accounting(True)
    ctx.reset_stats()
    dt = ctx.courant_dt()
    steps = 4
    led = None
    for _ in range(steps):
        ctx.step(dt, 1)
        led = o.step_ledger(st, dt, ijk, o.source_rates(nd), led)
    s = ctx.stats()
    g = ctx.state_numpy()
    print(f"# stats vs ledger bc={bc} flux={flux} fp32={fp32}", flush=True)
    if not fp32:
        # trace-matched run: per-cell counters first, then every integer exactly
        assert np.array_equal(g["nacc"], led["nacc"]) and np.array_equal(g["natt"], led["natt"])
        assert np.array_equal(np.array(s["substep_hist"]), led["substep_hist"])
        assert s["substeps_total"] == led["substeps_total"]
        assert s["attempts_total"] == led["attempts_total"]
        assert s["attempts_max"] == led["attempts_max"]
    assert s["flags"] == led["flags"] == 0
    tol = 1e-5 if fp32 else 1e-12
    tot = np.array(led["photons"]) + led["injected"]
    for k in ("photons", "injected"):
        assert np.allclose(s[k], led[k], rtol=tol, atol=0), (k, s[k], led[k])
    for k in ("absorbed", "outflow"):
        # differences of photon totals: bounded relative to the totals
        assert np.all(np.abs(np.array(s[k]) - led[k]) <= tol * np.abs(led[k]) + 10 * tol * tot), (k, s[k], led[k])
    assert s["ionised_H"] == pytest.approx(led["ionised_H"], rel=tol)
    assert s["max_f"] == pytest.approx(led["max_f"], rel=tol)
    assert s["min_N"] == pytest.approx(led["min_N"], rel=tol, abs=0)
    if bc != BCS[0]:
        assert np.all(np.abs(led["outflow"]) > 0)
