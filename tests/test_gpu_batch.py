"""GPU tests of the batched form: every box of a batch equals the same box
stepped alone through rt_step (bit for bit), graph replays equal eager
launches, launch tuning never changes results, and a subset matches the
oracle."""
import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri
from gpu_util import rel_err

pytestmark = pytest.mark.gpu

DX = 6.6 * ri.KPC / 128

FIELDS = ("N", "F", "xHII", "xHeII", "xHeIII", "T", "nacc", "natt")


def small_specs(seed=5, n=6):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        out.append(ri.BoxSpec(side=int(rng.choice([8, 12, 16, 20])), M=int(1 + b % 3),
                              nH=float(10 ** rng.uniform(-4, -1)), n_sources=int(rng.integers(1, 4)),
                              seed=seed * 100 + b))
    return out


def make_batch(specs, fp32, **tune):
    assert torch.cuda.is_available()
    from paper_1304_7126_amd.batch import batch_from_specs
    b, ws, srcs = batch_from_specs(specs, DX, fp32=fp32, counters=True)
    if tune:
        b.set_tuning(**tune)
    return b, ws, srcs


def single(w, srcs, fp32):
    from paper_1304_7126_amd import RTContext
    ctx = RTContext.for_workload(w, fp32=fp32, counters=True)
    ctx.load_state(ri.initial_state(w))
    ijk, nd = srcs
    ctx.set_sources(ijk, ctx.source_rates(nd))
    return ctx


@pytest.mark.parametrize("fp32", [True, False])
def test_batched_boxes_equal_single_box_steps(fp32):
    specs = small_specs()
    b, ws, srcs = make_batch(specs, fp32, head_attempts=2)
    dt = b.courant_dt()
    steps = 5
    b.step(dt, steps)
    for i, w in enumerate(ws):
        ctx = single(w, srcs[i], fp32)
        ctx.set_tuning(2, -1)
        ctx.step(dt, steps)
        g1, g2 = b.state_numpy(i), ctx.state_numpy()
        for k in FIELDS:
            assert np.array_equal(g1[k], g2[k]), (i, k, w.n, w.spectrum.M)


def test_graph_replays_equal_eager_launches():
    specs = small_specs(seed=7)
    a, ws, _ = make_batch(specs, True, use_graph=1)
    e, _, _ = make_batch(specs, True, use_graph=0)
    dt = a.courant_dt()
    for rep in range(4):
        a.step(dt, 1)          # graph replay
        e.step(dt, 1)          # eager launches
        a.synchronize()
        e.synchronize()
        # eager work of the program's own between replays
        junk = torch.ones(1 << 20, device="cuda").sum().item()
        assert junk == float(1 << 20)
        for i in range(len(ws)):
            ga, ge = a.state_numpy(i), e.state_numpy(i)
            for k in FIELDS:
                assert np.array_equal(ga[k], ge[k]), (rep, i, k)
    assert a.stats() == e.stats()


@pytest.mark.parametrize("tune", [dict(head_blocks_per_cu=1, head_attempts=1, tail_blocks=1),
                                  dict(head_blocks_per_cu=8, head_attempts=4, tail_blocks=2048),
                                  dict(head_blocks_per_cu=2, head_attempts=1000, tail_blocks=7)])
def test_batch_tuning_does_not_change_results(tune):
    specs = small_specs(seed=9)
    ref, ws, _ = make_batch(specs, True)
    alt, _, _ = make_batch(specs, True, **tune)
    dt = ref.courant_dt()
    ref.step(dt, 4)
    alt.step(dt, 4)
    for i in range(len(ws)):
        g1, g2 = ref.state_numpy(i), alt.state_numpy(i)
        for k in FIELDS:
            assert np.array_equal(g1[k], g2[k]), (i, k)


def test_batched_subset_matches_oracle():
    specs = small_specs(seed=11, n=4)
    b, ws, srcs = make_batch(specs, False)
    dt = b.courant_dt()
    steps = 4
    b.step(dt, steps)
    for i, w in enumerate(ws):
        o = oracle.OracleRT.for_workload(w)
        st = ri.initial_state(w)
        ijk, nd = srcs[i]
        ondot = o.source_rates(nd)
        for _ in range(steps):
            o.step(st, dt, ijk, ondot)
        g = b.state_numpy(i)
        for k in ("xHII", "xHeII", "xHeIII", "T"):
            assert rel_err(g[k], st[k]) < 1e-9, (i, k)
        assert rel_err(g["N"], st["N"]) < 1e-9
        assert rel_err(g["F"], st["F"]) < 1e-9


def test_autotuner_picks_a_config_and_keeps_state(tmp_path, monkeypatch):
    from paper_1304_7126_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    specs = small_specs(seed=13)
    b, ws, _ = make_batch(specs, True)
    ref, _, _ = make_batch(specs, True)
    dt = b.courant_dt()
    res = autotune.tune_batch(b, dt, trial_steps=1, head_blocks=(1, 4), head_attempts=(1, 3),
                              tail_blocks=(256, 1024))
    assert len(res["config"]) == 3 and not res["cached"]
    again = autotune.tune_batch(b, dt)
    assert again["cached"] and again["config"] == res["config"]
    b.step(dt, 3)
    ref.step(dt, 3)
    for i in range(len(ws)):
        g1, g2 = b.state_numpy(i), ref.state_numpy(i)
        for k in FIELDS:
            assert np.array_equal(g1[k], g2[k]), (i, k)


def test_batching_workload_subset_mixed_matches_oracle():
    # the 64-box batching workload in its own precision (FP32 transport, FP64
    # chemistry): one box of each side 16, 24, 32, 48, 64, 96 is checked
    # against the oracle on sampled cells at step 100 (oracle steps from the
    # batch's pre-step state), the two smallest over their whole 100 steps
    from test_gpu_fullsize import FP32_DARK, FP32_EPS, FP32_FLOOR, compare_sampled, perturbed_oracle, sample_cells
    specs = ri.batch_boxes(64, seed=0)
    b, ws, srcs = make_batch(specs, True)
    dt = b.courant_dt()
    pick = {}
    for i, s in enumerate(specs):
        pick.setdefault(s.side, i)
    assert sorted(pick) == [16, 24, 32, 48, 64, 96]
    steps = 100
    b.step(dt, steps - 1)
    pre = {i: b.state_numpy(i) for i in pick.values()}
    b.step(dt, 1)
    for side, i in sorted(pick.items()):
        w = ws[i]
        print(f"# batch box {i}: side {side}, M = {w.spectrum.M}, n_H {w.nH_mean:.3g}", flush=True)
        g = b.state_numpy(i)
        st = dict(pre[i])
        o = oracle.OracleRT.for_workload(w)
        ijk, nd = srcs[i]
        o.inject(st, dt, ijk, o.source_rates(nd))
        cells = sample_cells(w, ijk, st["natt"].ravel(), 1024, i)
        r = o.step_cells(st, dt, cells)
        # dense boxes amplify the FP32 rounding of the transport: the limits
        # include 10x the oracle's own response to a perturbation of that
        # size; cells behind the fronts hold densities below FP32's range
        compare_sampled(w, st, g, cells, r, 1e-5, spread=perturbed_oracle(o, st, dt, cells, FP32_EPS),
                        dark=FP32_DARK, abs_floor=FP32_FLOOR)
    for side in (16, 24):
        i = pick[side]
        w = ws[i]
        o = oracle.OracleRT.for_workload(w)
        st = ri.initial_state(w)
        ijk, nd = srcs[i]
        ondot = o.source_rates(nd)
        for _ in range(steps):
            o.step(st, dt, ijk, ondot)
        g = b.state_numpy(i)
        # FP32 rounding of N, F once per step, carried through the chemistry
        for k in ("xHII", "xHeII", "xHeIII", "T", "N", "F"):
            assert rel_err(g[k], st[k]) < 1e-5, (side, k, rel_err(g[k], st[k]))
