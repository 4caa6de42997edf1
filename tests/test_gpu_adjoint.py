"""GPU tests of the differentiation form (rt_step_record / rt_step_adjoint
behind torch.autograd.Function, with checkpointing).

  - a recorded step equals rt_step bit for bit and reports no tape mismatch;
  - gradients w.r.t. the log source rates and log densities equal the
    oracle's complex-step directional derivatives (the FP64 reference
    gradient: same branch of the subcycling as the adjoint) on a small box
    with several checkpoint segments, isothermal and with T evolving;
  - on the full differentiation workload (64^3, 16 sources, 300 steps,
    checkpoints every 20 steps) they equal central finite differences
    (h = 1e-6, FP64) of the GPU forward run;
  - the mixed form's gradient (FP32 radiation in the forward steps) stays
    close to the FP64 one on that workload;
  - a backward uses the parameters of its own forward run, whatever the
    context holds by then, and refuses once a later forward run has
    replaced the checkpoints.
"""
import numpy as np
import pytest
import torch

import rt_inputs as ri
from oracle import complex_step as cs
from oracle import physics

pytestmark = pytest.mark.gpu


def make_run(w, every, fp32=False):
    from paper_1304_7126_amd import RTContext
    from paper_1304_7126_amd.adjoint import GradientRun
    ctx = RTContext.for_workload(w, counters=True, fp32=fp32)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    dt = ctx.courant_dt()
    run = GradientRun(ctx, ijk, dt, w.steps, x0=w.xHII0, T0=w.T0, every=every)
    return run, ijk, nd, dt


def params(w, nd):
    st = ri.initial_state(w)
    lnnd = torch.tensor(np.log(nd), dtype=torch.float64)
    lnnH = torch.tensor(np.log(st["nH"]), dtype=torch.float64, device="cuda")
    return st, lnnd, lnnH


@pytest.mark.parametrize("fp32", [False, True])
def test_recorded_steps_equal_rt_step(fp32):
    assert torch.cuda.is_available()
    from paper_1304_7126_amd import capi
    w = ri.grey_box(20, 3.3 * 20 / 64, 6, 12, seed=3)
    run, ijk, nd, dt = make_run(w, every=5, fp32=fp32)
    st, lnnd, lnnH = params(w, nd)
    x_fwd = run.forward(lnnd, lnnH)
    ctx = run.ctx
    fwd = {k: getattr(ctx, k).clone() for k in ("xHII", "T")}
    fwd["N"], fwd["F"] = (a.clone() for a in ctx.radiation())
    # the same steps again through rt_step_record
    g_src, g_nH, *_ = run.backward(torch.zeros_like(x_fwd))
    assert run.last_backward["flags"] & capi.RT_FLAG_TRACE == 0
    # backward ends with the first segment re-recorded: replay everything
    run._restore(run.ckpt[0])
    import ctypes
    from paper_1304_7126_amd.capi import lib
    nc = run.nc
    for k in range(w.steps):
        tot = int(run.counts[k].sum().item()) + nc
        Na = torch.empty(nc, dtype=torch.float64, device="cuda")
        Fa = torch.empty(3 * nc, dtype=torch.float64, device="cuda")
        off = torch.empty(run.off_len, dtype=torch.int64, device="cuda")
        tr = torch.empty(7 * tot, dtype=torch.float64, device="cuda")
        t = capi.RtTape(Na.data_ptr(), Fa.data_ptr(), run.counts[k].data_ptr(), off.data_ptr(), tr.data_ptr(), tot)
        capi.check(lib().rt_step_record(ctx._h, dt, ctypes.byref(t)), ctx._h)
        torch.cuda.synchronize()
        assert int(off[nc].item()) == tot
    N, F = ctx.radiation()
    assert torch.equal(N, fwd["N"]) and torch.equal(F, fwd["F"])
    assert torch.equal(ctx.xHII, fwd["xHII"]) and torch.equal(ctx.T, fwd["T"])
    assert torch.equal(ctx.xHII, x_fwd)
    assert ctx.stats()["flags"] & capi.RT_FLAG_TRACE == 0
    # a zero cotangent gives zero gradients
    assert float(g_src.abs().max()) == 0.0 and float(g_nH.abs().max()) == 0.0


@pytest.mark.parametrize("iso", [True, False])
def test_gradient_equals_oracle_complex_step(iso):
    assert torch.cuda.is_available()
    from paper_1304_7126_amd.adjoint import rt_run
    w = ri.grey_box(12, 3.3 * 12 / 64, 6, 24, seed=1, isothermal=iso)
    run, ijk, nd, dt = make_run(w, every=10)  # segments of 10, 10, 4 steps
    st, lnnd, lnnH = params(w, nd)
    sN, sE, eb, _ = physics.spectrum_attributes(w.spectrum)
    p = cs.CSParams(w.n, w.dx, w.c_r, sN[0][0], sE[0][0], eb[0], iso, X=w.X, gamma=w.gamma, a_exp=w.a_exp,
                    x_min=w.x_min)
    s0 = {"N": st["N"][0], "F": st["F"][0], "xHII": st["xHII"], "T": st["T"]}
    tfin, _ = cs.run(p, s0, dt, w.steps, ijk, ri.perturbed_log_rates(nd, w.seed), np.log(st["nH"]))
    target = torch.tensor(tfin["xHII"].real, device="cuda")

    a = lnnd.clone().requires_grad_(True)
    b = lnnH.clone().requires_grad_(True)
    x = rt_run(run, a, b)
    loss = ((x - target) ** 2).sum()
    loss.backward()
    g_src = a.grad.numpy()
    g_nH = b.grad.cpu().numpy()
    assert np.all(np.isfinite(g_src)) and np.all(np.isfinite(g_nH))

    ln_nH = np.log(st["nH"])
    rng = np.random.default_rng(11)
    checks = [(np.eye(len(nd))[s], None) for s in range(len(nd))]
    checks += [(None, rng.standard_normal(ln_nH.shape)) for _ in range(2)]
    for s in range(2):
        v = np.zeros(ln_nH.shape)
        i, j, k = ijk[s]
        v[k, j, (i + 1) % w.n[0]] = 1.0
        checks.append((None, v))
    scale = max(np.max(np.abs(g_src)), 1e-300)
    for vs, vc in checks:
        ref = cs.directional_derivative(p, s0, dt, w.steps, ijk, np.log(nd), ln_nH, target.cpu().numpy(), vs, vc)
        got = (float(g_src @ vs) if vs is not None else 0.0) + (float(np.sum(g_nH * vc)) if vc is not None else 0.0)
        assert abs(got - ref) <= 1e-8 * abs(ref) + 1e-12 * scale, (vs is not None, got, ref)


def test_gradient_equals_gpu_central_differences_at_full_size():
    """64^3, 16 sources, 300 steps, checkpoints every 20.  Central
    differences with h = 1e-6 (FP64) over all 16 log rates, 4 random
    directions over all log densities, the 16 cells next to the sources and
    16 random cells:
      - frozen schedule (rt_step_replay with the base run's substeps): the
        function the adjoint differentiates, so they must agree closely;
      - free running (rt_step): pairs whose +h or -h run changed any cell's
        substep count cross a jump of the method and are only counted; the
        others must agree as closely."""
    assert torch.cuda.is_available()
    from paper_1304_7126_amd.adjoint import rt_run
    w = ri.grey_64(steps=300, seed=0)
    run, ijk, nd, dt = make_run(w, every=20)
    st, lnnd, lnnH = params(w, nd)
    with torch.no_grad():
        target = run.forward(torch.tensor(ri.perturbed_log_rates(nd, w.seed)), lnnH).clone()
        run.forward(lnnd, lnnH)
        counts0 = run.counts.clone()
        run.record_schedule()

    def loss(x):
        return float(((x - target) ** 2).sum().item())

    a = lnnd.clone().requires_grad_(True)
    b = lnnH.clone().requires_grad_(True)
    x = rt_run(run, a, b)
    L0 = ((x - target) ** 2).sum()
    L0.backward()
    L0 = float(L0.item())
    assert torch.equal(run.counts, counts0)
    g_src = a.grad.numpy().copy()
    g_nH = b.grad.cpu().numpy().copy()
    with torch.no_grad():
        assert abs(loss(run.replay(lnnd, lnnH)) - L0) <= 1e-12 * L0
    h = 1e-6
    rng = np.random.default_rng(21)
    dirs = [(np.eye(len(nd))[s], None) for s in range(len(nd))]
    dirs += [(None, rng.standard_normal(lnnH.shape)) for _ in range(4)]
    for c in ijk[:16]:
        v = np.zeros(lnnH.shape)
        v[c[2], c[1], (c[0] + 1) % w.n[0]] = 1.0
        dirs.append((None, v))
    for _ in range(16):
        v = np.zeros(lnnH.shape)
        v[tuple(rng.integers(0, 64, 3))] = 1.0
        dirs.append((None, v))
    gscale = float(np.max(np.abs(g_src)))
    bad_frozen, bad_free, flipped = [], [], 0
    for vs, vc in dirs:
        da = torch.tensor(vs) if vs is not None else torch.zeros_like(lnnd)
        db = torch.tensor(vc, device="cuda") if vc is not None else torch.zeros_like(lnnH)
        got = (float(g_src @ vs) if vs is not None else 0.0) + (float(np.sum(g_nH * vc)) if vc is not None else 0.0)
        with torch.no_grad():
            fz = (loss(run.replay(lnnd + h * da, lnnH + h * db)) - loss(run.replay(lnnd - h * da, lnnH - h * db))) / (2 * h)
            lp = loss(run.forward(lnnd + h * da, lnnH + h * db))
            same = torch.equal(run.counts, counts0)
            lm = loss(run.forward(lnnd - h * da, lnnH - h * db))
            same = same and torch.equal(run.counts, counts0)
        fd = (lp - lm) / (2 * h)
        tol = 1e-6 * abs(got) + 1e-9 * gscale
        print(f"dir {'src ' if vs is not None else 'cell'} adjoint {got:+.10e} frozen {fz:+.10e} "
              f"free {fd:+.10e} {'same schedule' if same else 'schedule changed'}", flush=True)
        if not abs(got - fz) <= tol:
            bad_frozen.append((got, fz))
        if same:
            if not abs(got - fd) <= tol:
                bad_free.append((got, fd))
        else:
            flipped += 1
    print(f"L = {L0:.6e}; {flipped} of {len(dirs)} free-running pairs changed the substep schedule", flush=True)
    assert not bad_frozen, bad_frozen
    assert not bad_free, bad_free


def test_backward_uses_the_parameters_of_its_forward():
    assert torch.cuda.is_available()
    from paper_1304_7126_amd import capi
    from paper_1304_7126_amd.adjoint import rt_run
    w = ri.grey_box(12, 3.3 * 12 / 64, 4, 10, seed=5)
    run, ijk, nd, dt = make_run(w, every=4)
    st, lnnd, lnnH = params(w, nd)
    target = torch.full_like(lnnH, 0.5)
    with torch.no_grad():
        x = run.forward(lnnd, lnnH)
        g_ref = [t.clone() for t in run.backward(2.0 * (x - target))[:2]]
    a = lnnd.clone().requires_grad_(True)
    b = lnnH.clone().requires_grad_(True)
    loss = ((rt_run(run, a, b) - target) ** 2).sum()
    # something else puts other sources and densities on the context
    # (a finite-difference probe, say) before the backward
    run._set_params(lnnd + 0.3, lnnH - 0.2)
    loss.backward()
    assert torch.equal(a.grad, g_ref[0].cpu()) and torch.equal(b.grad, g_ref[1])
    # a later forward run replaces the checkpoints: the earlier graph refuses
    a1 = lnnd.clone().requires_grad_(True)
    b1 = lnnH.clone().requires_grad_(True)
    l1 = ((rt_run(run, a1, b1) - target) ** 2).sum()
    with torch.no_grad():
        run.forward(lnnd + 0.1, lnnH)
    with pytest.raises(capi.RTError):
        l1.backward()


def test_mixed_gradient_close_to_fp64_at_full_size():
    """C5's workload (64^3, 16 sources, 300 steps, checkpoints every 20)
    differentiated twice: in FP64 and in the mixed form.  The loss uses the
    FP64 target in both.  Compared: L, the 16 source gradients and the
    directional derivatives along 4 random directions over all log
    densities (relative to the FP64 values), and the per-cell density
    gradient (global-normalised)."""
    assert torch.cuda.is_available()
    from paper_1304_7126_amd.adjoint import rt_run
    w = ri.grey_64(steps=300, seed=0)
    res = {}
    target = None
    for fp32 in (False, True):
        run, ijk, nd, dt = make_run(w, every=20, fp32=fp32)
        st, lnnd, lnnH = params(w, nd)
        if target is None:
            with torch.no_grad():
                target = run.forward(torch.tensor(ri.perturbed_log_rates(nd, w.seed)), lnnH).clone()
        a = lnnd.clone().requires_grad_(True)
        b = lnnH.clone().requires_grad_(True)
        L = ((rt_run(run, a, b) - target) ** 2).sum()
        L.backward()
        res[fp32] = (float(L.item()), a.grad.numpy().copy(), b.grad.cpu().numpy().copy(),
                     run.last_backward["flags"])
        run.ctx.close()
        del run
        torch.cuda.empty_cache()
    (L64, gs64, gn64, f64), (L32, gs32, gn32, f32) = res[False], res[True]
    assert f64 == 0 and f32 == 0
    rng = np.random.default_rng(5)
    dirs = [rng.standard_normal(gn64.shape) for _ in range(4)]
    d64 = np.array([np.sum(gn64 * v) for v in dirs])
    d32 = np.array([np.sum(gn32 * v) for v in dirs])
    e_L = abs(L32 - L64) / abs(L64)
    e_src = float(np.max(np.abs(gs32 - gs64)) / np.max(np.abs(gs64)))
    e_src_each = float(np.max(np.abs(gs32 - gs64) / np.abs(gs64)))
    e_dir = float(np.max(np.abs(d32 - d64) / np.abs(d64)))
    e_cell = float(np.max(np.abs(gn32 - gn64)) / np.max(np.abs(gn64)))
    sc = np.max(np.abs(gn64))
    m = np.abs(gn64) > 1e-6 * sc
    rel = np.abs(gn32[m] - gn64[m]) / np.abs(gn64[m])
    print(f"mixed vs FP64 adjoint: L {e_L:.3e}, source gradients e_inf {e_src:.3e} (each {e_src_each:.3e}), "
          f"density directions {e_dir:.3e}, density gradient e_inf {e_cell:.3e}, per-cell p50 "
          f"{np.quantile(rel, 0.5):.3e} p99 {np.quantile(rel, 0.99):.3e} max {rel.max():.3e}", flush=True)
    # measured: loss 9.2e-7, sources 3.1e-6 (each 2.5e-5), directions 7.3e-6
    assert e_L <= 1e-5
    assert e_src <= 1e-4 and e_src_each <= 1e-3 and e_dir <= 1e-4
