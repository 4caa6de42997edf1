#!/usr/bin/env python3
"""Throughput of the explicit M1 RT step on one MI355X.

Workload: 256^3 cells x 3 photon groups (lognormal H+He gas, mean n_H =
1e-3 cm^-3, sigma_ln = 1, 200 sources of 1e47-1e49 photons/s, HLL flux,
c_r = c/100, Courant 0.8), FP32 N/F transport with FP64 thermochemistry.
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line: metric, value (cell-group updates/s over the timed
steps), the roofline of the dominant kernel measured live with HIP events on
the library's stream, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# VALU wave-instructions per second of the chip: 1,024 SIMDs x 2.4 GHz / 4
# cycles per wave64 instruction
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4

# rocprofv3 summaries of the headline command (profiles/, written by
# paper_1304_7126_amd.profiling): kernel durations, HBM byte counters and
# VALU counters of the dominant kernels over the timed launches, one set per
# launch window that is timed (the default 10 warmup + 100 steps: launches
# 11-110; 5 + 20 steps: launches 6-25).  Their figures are used only while
# the kernel sources hash as when they were taken, and only for the window
# they cover.
PROFILE = os.path.join(ROOT, "profiles", "k_chem_all_256cube_3grp")
PROFILE_TRANSPORT = os.path.join(ROOT, "profiles", "k_transport_z_256cube_3grp")
PROFILE_SETS = {PROFILE: [PROFILE, PROFILE + "_launches6to25"],
                PROFILE_TRANSPORT: [PROFILE_TRANSPORT, PROFILE_TRANSPORT + "_launches6to25"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--fp64", action="store_true", help="FP64 transport instead of FP32")
    ap.add_argument("--flux", choices=["hll", "glf"], default="hll")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--head-attempts", type=int, default=0, help="chemistry attempts per cell in the first pass")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost measurement")
    ap.add_argument("--form", choices=["grid", "batch", "adjoint", "shadow", "stromgren", "plain128", "precision",
                                       "oracle-timing"], default="grid",
                    help="grid: the 256^3 x 3 headline; batch: 64 uneven boxes, batched vs one-by-one; "
                         "shadow: Iliev test 3 (dense clump lit from the x = 0 face) at 128^3 to 15 Myr; "
                         "stromgren: 32^3 x 1 FP64 GLF, 100 steps; plain128: 128^3 x 3 FP64 HLL, 50 sources, "
                         "200 steps; precision: mixed vs FP64 GPU vs oracle on the 256^3 workload and its 64^3 "
                         "sub-box; oracle-timing: the CPU oracle at 1 thread and all cores on the configs")
    ap.add_argument("--no-accounting", action="store_true",
                    help="time the headline steps without the photon accounting (a4)")
    ap.add_argument("--transport-path", choices=["auto", "cell", "zmarch"], default="auto")
    ap.add_argument("--chem-path", choices=["auto", "two-pass", "one-pass"], default="auto")
    ap.add_argument("--shadow-myr", type=float, default=15.0, help="simulated time of --form shadow [Myr]")
    ap.add_argument("--smooth", action="store_true", help="time the smoothed RT step (Sec. 4.4) instead")
    ap.add_argument("--n-floor", type=float, default=None,
                    help="photon density floor of the 10%% check (default 0; 1e-12 with --smooth)")
    ap.add_argument("--smooth-steps", type=int, default=30,
                    help="timed steps of the smoothed-vs-plain comparison at floor 1e-12 and of the "
                         "with/without OTSA comparison (0: skip both)")
    ap.add_argument("--expansion", type=float, default=1.0,
                    help="time the step with super-comoving variables at this expansion factor (Sec. 5.4)")
    ap.add_argument("--no-otsa", action="store_true",
                    help="time the step without the on-the-spot approximation (Sec. 3.3.2) instead")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="after the timed region, copy this many MiB device-to-device 3 times "
                         "(reference kernel for HBM byte counters)")
    return ap.parse_args()


def algorithmic_bytes(M, fp32):
    """Bytes one RT step must move per cell: read and write N, F of every
    group once (4 values x 4 or 8 bytes each way) and the gas state x_HII,
    x_HeII, x_HeIII, T (FP64, read and write), plus n_H (read).  The same
    count is the first chemistry pass's when the transport runs on its own:
    it reads N and the gas, writes them, and rescales F (one read, one
    write); the transport moves N, F once each way (rad below)."""
    rb = 4 if fp32 else 8
    rad = 2 * 4 * rb * M
    gas = 2 * 4 * 8 + 8
    return rad, gas


def cpu_baseline(seconds, n_full, M):
    """The oracle on the 64^3 sub-box of the workload's realisation (cells
    [0, 64)^3 with the sources inside them, periodic, same cell size),
    stepped from the initial state until ~`seconds` of wall time, on all the
    host's cores."""
    import oracle
    import rt_inputs as ri
    w = ri.lognormal_box(n_full, 13.2 * n_full / 256, max(1, round(200 * (n_full / 256) ** 3)), steps=1, seed=0)
    ws, st, ijk, nd = ri.subbox(w, min(64, n_full))
    o = oracle.OracleRT.for_workload(ws)
    ndot = o.source_rates(nd)
    dt = o.courant_dt()
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(st, dt, ijk, ndot)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 100:
            break
    n = ws.n[0]
    cgu = ws.ncell * M * steps / el
    return {"value": cgu, "unit": "cell-group updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{n}^3 x {M} groups sub-box [0,{n})^3 of the {n_full}^3 realisation with its "
                      f"{ws.n_sources} sources (periodic), first {steps} RT steps from the initial state, "
                      f"{el:.1f} s wall"}


def grid_run(n, fp32, flux_name, steps, warmup, head_attempts, smooth=False, floor=0.0, nH_mean=1e-3, otsa=True,
             a=1.0, acct=False, path="auto", chem_path="auto"):
    """The lognormal n^3 x 3 workload: build it, run `warmup` steps, reload
    the initial state, then time `steps` rt_step calls from it (injection,
    transport, the chemistry passes and, with acct, the photon accounting and
    its reductions), with the library's HIP events bracketing each kernel on
    its stream and one pair of events around each step (the per-step
    series)."""
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext
    flux = ri.FLUX_HLL if flux_name == "hll" else ri.FLUX_GLF
    w = ri.lognormal_box(n, 13.2 * n / 256, max(1, round(200 * (n / 256) ** 3)), steps=steps, seed=0, flux=flux)
    w.nH_mean = nH_mean
    w.otsa = otsa
    M = w.spectrum.M
    print(f"# building {n}^3 x {M} workload (mean n_H {nH_mean:g}, smooth={smooth}, N_floor={floor:g}, "
          f"otsa={otsa}, accounting={acct})", file=sys.stderr, flush=True)
    st = ri.initial_state(w)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ctx = RTContext.for_workload(w, fp32=fp32, smooth=smooth, N_floor=floor)
    if a != 1.0:
        # the same comoving box at expansion factor a: comoving densities
        st["nH"] = st["nH"] * a ** 3
    ctx.load_state(st)
    if a != 1.0:
        ctx.set_expansion(a)
    ctx.set_sources(ijk, ctx.source_rates(nd))
    ctx.set_transport_path(path)
    ctx.set_chem_path(chem_path)
    dt = ctx.courant_dt()
    if head_attempts > 0:
        ctx.set_tuning(head_attempts, -1)
    print(f"# warmup {warmup} steps", file=sys.stderr, flush=True)
    for _ in range(warmup):
        ctx.step(dt, 1)
    torch.cuda.synchronize()
    # the timed steps are the workload's steps 1..K: back to the initial state
    ctx.load_state(st)
    del st
    ctx.reset_stats()
    ctx.set_accounting(acct)
    ctx.set_timing(True)
    ctx.timing()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        ctx.step(dt, 1)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.timing()
    ctx.set_timing(False)
    s = ctx.stats()
    series = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tm.items()}
    per_step = {k: v[0] / steps for k, v in tm.items()}
    del ctx
    return {"w": w, "M": M, "stats": s, "ms": wall * 1e3 / steps, "cgu": w.ncell * M * steps / wall, "per": per,
            "per_step": per_step, "series": series}


def smoothing_comparison(n, fp32, flux_name, steps, warmup, head_attempts):
    """Smoothed RT (Sec. 4.4) against plain operator splitting on the same
    workload and photon floor (1e-12 cm^-3, far below the densities that
    ionise: c_r sigma N dt ~ 1e-10 there): substeps and time per step, on
    the headline's diffuse gas (mean n_H 1e-3 cm^-3) and on the same box
    with 100 times denser gas, where the sources' photons are absorbed
    within a step (the case the section describes)."""
    out = {"N_floor": 1e-12, "timed_steps": steps, "warmup": warmup}
    for name, nH in (("diffuse", 1e-3), ("dense", 1e-1)):
        d = {"mean_nH": nH}
        for smooth in (False, True):
            r = grid_run(n, fp32, flux_name, steps, warmup, head_attempts, smooth, 1e-12, nH)
            s = r["stats"]
            nc = r["w"].ncell
            d["smoothed" if smooth else "plain"] = {
                "value": r["cgu"], "unit": "cell-group updates/s", "ms_per_step": r["ms"],
                "substeps_per_cell_step": s["substeps_total"] / (nc * steps),
                "attempts_per_cell_step": s["attempts_total"] / (nc * steps), "attempts_max": s["attempts_max"],
                "flags": s["flags"], "ms_per_launch": {k: r["per"][k] for k in ("inject", "head", "tail")}}
        d["substep_ratio_plain_over_smoothed"] = (d["plain"]["substeps_per_cell_step"] /
                                                  d["smoothed"]["substeps_per_cell_step"])
        d["time_ratio_plain_over_smoothed"] = d["plain"]["ms_per_step"] / d["smoothed"]["ms_per_step"]
        out[name] = d
    return out


def otsa_comparison(n, fp32, flux_name, steps, warmup, head_attempts):
    """The headline workload with and without the on-the-spot approximation
    (Sec. 3.3.2: case A rates and recombination photons into the group
    holding each species' threshold), same steps timed."""
    out = {"timed_steps": steps, "warmup": warmup}
    for otsa in (True, False):
        r = grid_run(n, fp32, flux_name, steps, warmup, head_attempts, otsa=otsa)
        s = r["stats"]
        nc = r["w"].ncell
        out["otsa" if otsa else "case_A_with_emission"] = {
            "value": r["cgu"], "unit": "cell-group updates/s", "ms_per_step": r["ms"],
            "substeps_per_cell_step": s["substeps_total"] / (nc * steps),
            "attempts_max": s["attempts_max"], "flags": s["flags"],
            "ms_per_launch": {k: r["per"][k] for k in ("inject", "head", "tail")}}
    out["time_ratio"] = out["case_A_with_emission"]["ms_per_step"] / out["otsa"]["ms_per_step"]
    # the same comoving box at a = 1/8 (super-comoving variables, Sec. 5.4):
    # 512x denser gas in physical units, photons in a^3 N
    a = 0.125
    r = grid_run(n, fp32, flux_name, steps, warmup, head_attempts, a=a)
    s = r["stats"]
    nc = r["w"].ncell
    out["super_comoving_a_0.125"] = {
        "value": r["cgu"], "unit": "cell-group updates/s", "ms_per_step": r["ms"],
        "substeps_per_cell_step": s["substeps_total"] / (nc * steps), "attempts_max": s["attempts_max"],
        "flags": s["flags"], "ms_per_launch": {k: r["per"][k] for k in ("inject", "head", "tail")}}
    return out


def bench_shadow(args):
    """Iliev test 3 (Sec. 6) on a uniform 128^3 grid: a flux of 1e6 photons
    s^-1 cm^-2 enters through the x = 0 face, a clump of 200x denser gas
    traps the I-front and casts a shadow; HLL, three groups, c_r = c/10, run
    to 15 Myr.  Reports the step rate and the quantities the paper plots:
    the I-front position on the axis (x_HII = 0.5, relative to the clump
    centre, in units of the clump's Stromgren length 0.78 kpc) and the mean
    ionised fraction and temperature inside the clump at 1, 3 and 15 Myr."""
    import numpy as np
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext
    w = ri.shadow_clump(128)
    st = ri.initial_state(w)
    ctx = RTContext.for_workload(w)
    ctx.load_state(st)
    ctx.set_chem_path(args.chem_path)
    ctx.set_transport_path(args.transport_path)
    inside = st["nH"] > 1e-3
    del st
    dt = ctx.courant_dt()
    myr = 3.15576e13
    marks = sorted({m for m in (1.0, 3.0, args.shadow_myr) if m <= args.shadow_myr})
    targets = [int(round(m * myr / dt)) for m in marks]
    n = w.n[0]
    dx = w.dx
    xs = (np.arange(n) + 0.5) * dx

    def snapshot(t_myr):
        x = ctx.xHII.cpu().numpy()
        T = ctx.T.cpu().numpy()
        axis = x[n // 2, n // 2, :]
        # the I-front: the last x_HII = 0.5 crossing on the axis before the
        # neutral gas (the clump or the shadow behind it)
        k = int(np.argmax(axis < 0.5)) if np.any(axis < 0.5) else n - 1
        if 0 < k < n and axis[k] < 0.5 <= axis[k - 1]:
            xf = xs[k - 1] + (axis[k - 1] - 0.5) / (axis[k - 1] - axis[k]) * dx
        else:
            xf = xs[k]
        return {"t_Myr": t_myr, "ifront_x_kpc": xf / ri.KPC,
                "ifront_rel_clump_centre_over_lS": (xf / ri.KPC - 5.0) / 0.78,
                "clump_mean_xHII": float(x[inside].mean()), "clump_mean_T": float(T[inside].mean()),
                "shadow_xHII": float(x[n // 2, n // 2, int(6.3 * ri.KPC / dx)]),
                "beside_xHII": float(x[n // 2, int(1.0 * ri.KPC / dx), int(6.3 * ri.KPC / dx)])}

    print(f"# shadow clump 128^3: {targets[-1]} steps of {dt:.4g} s", file=sys.stderr, flush=True)
    ctx.step(dt, 10)
    torch.cuda.synchronize()
    ctx.reset_stats()
    done, snaps, wall = 10, [], 0.0
    chunk = 1000
    for tgt, m in zip(targets, marks):
        while done < tgt:
            k = min(chunk, tgt - done)
            t0 = time.perf_counter()
            ctx.step(dt, k)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            done += k
            print(f"# step {done} / {targets[-1]}", file=sys.stderr, flush=True)
        snaps.append(snapshot(m))
    s = ctx.stats()
    timed = done - 10
    cgu = w.ncell * w.spectrum.M * timed / wall
    print(json.dumps({"metric": "RT cell-group updates/s, Iliev test 3 (shadow) at 128^3 x 3 groups", "value": cgu,
                      "unit": "cell-group updates/s", "n_gpus": 1, "steps": timed, "warmup": 10,
                      "ms_per_step": wall * 1e3 / timed, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "Iliev test 3 on a uniform 128^3 grid: 6.6 kpc, n_H 2e-4 / clump 4e-2, "
                                             "F = 1e6 s^-1 cm^-2 from x = 0, HLL, 3 groups, c_r = c/10, FP64"},
                      "substeps_per_cell_step": s["substeps_total"] / (w.ncell * timed),
                      "attempts_max": s["attempts_max"], "flags": s["flags"], "snapshots": snaps}), flush=True)


def bench_batch(args):
    """The batching form: 64 periodic boxes (sides 16-96, 1-3 groups, uniform
    densities, 1-8 sources; FP32 transport, FP64 chemistry, GLF), advanced as
    one autotuned batch (one graph launch per step) and, for comparison, one
    box at a time through rt_step, in the same precision and in plain FP64;
    the batched result is compared with both after the same steps."""
    import numpy as np
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext, autotune
    from paper_1304_7126_amd.batch import batch_from_specs
    specs = ri.batch_boxes(64, seed=0)
    dx = 6.6 * ri.KPC / 128
    b, ws, srcs = batch_from_specs(specs, dx, fp32=True)
    cg = sum(w.ncell * w.spectrum.M for w in ws)
    dt = b.courant_dt()
    tune = autotune.tune_batch(b, dt, trial_steps=2, use_cache=False)
    b.step(dt, args.warmup)
    b.synchronize()
    b.reset_stats()
    t0 = time.perf_counter()
    b.step(dt, args.steps)
    b.synchronize()
    wall_b = time.perf_counter() - t0
    st = b.stats()
    fields = ("N", "F", "xHII", "xHeII", "xHeIII", "T")
    res_b = [{k: b.state_numpy(i)[k] for k in fields} for i in range(len(ws))]
    del b
    torch.cuda.empty_cache()

    def one_by_one(fp32):
        ctxs = []
        for w, (ijk, nd) in zip(ws, srcs):
            c = RTContext.for_workload(w, fp32=fp32)
            c.load_state(ri.initial_state(w))
            c.set_sources(ijk, c.source_rates(nd))
            ctxs.append(c)
        for _ in range(args.warmup):
            for c in ctxs:
                c.step(dt, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for c in ctxs:
                c.step(dt, 1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res = [c.state_numpy() for c in ctxs]
        for c in ctxs:
            c.close()
        torch.cuda.empty_cache()
        return wall, res

    wall_u, res_u = one_by_one(True)
    same = all(np.array_equal(rb[k], ru[k]) for rb, ru in zip(res_b, res_u) for k in fields)
    wall_64, res_64 = one_by_one(False)
    # e_inf of the batched (mixed) result against plain FP64, worst box
    err = {k: max(float(np.max(np.abs(rb[k] - r6[k])) / max(np.max(np.abs(r6[k])), 1e-300))
                  for rb, r6 in zip(res_b, res_64)) for k in fields}
    out = {"metric": "RT cell-group updates/s, 64 uneven boxes (batching form)",
           "value": cg * args.steps / wall_b, "unit": "cell-group updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall_b * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 transport / f64 chemistry", "data": "synthetic",
           "config": {"workload": "64 periodic boxes, sides {16..96}, 1-3 groups, GLF", "cells": sum(w.ncell for w in ws),
                      "cell_groups": cg, "tuning": tune["config"]},
           "one_by_one": {"value": cg * args.steps / wall_u, "ms_per_step": wall_u * 1e3 / args.steps,
                          "identical_to_batched": same},
           "speedup_vs_one_by_one": wall_u / wall_b,
           "one_by_one_fp64": {"value": cg * args.steps / wall_64, "ms_per_step": wall_64 * 1e3 / args.steps,
                               "batched_e_inf_vs_fp64": err},
           "speedup_vs_one_by_one_fp64": wall_64 / wall_b,
           "chem": {"attempts_per_cell_step": st["attempts_total"] / (sum(w.ncell for w in ws) * args.steps),
                    "flags": st["flags"]}}
    print(json.dumps(out), flush=True)


def adjoint_cost(steps=300, every=20):
    """Cost of the gradient of L = sum (x_HII - target)^2 after `steps`
    steps of the differentiation workload (64^3, one grey group, hydrogen
    only, 16 sources, FP64) with checkpoints every `every` steps, against
    the plain forward run (rt_step, no checkpoints) on the same GPU; and the
    same gradient in the mixed form (FP32 radiation in the forward steps)
    with its cost and its distance from the FP64 gradient."""
    import numpy as np
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext
    from paper_1304_7126_amd.adjoint import GradientRun

    w = ri.grey_64(steps=steps)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    st = ri.initial_state(w)
    lnnd = torch.tensor(np.log(nd), dtype=torch.float64)
    lnnH = torch.tensor(np.log(st["nH"]), dtype=torch.float64, device="cuda")

    def t_plain(fp32):
        plain = RTContext.for_workload(w, fp32=fp32)
        dt = plain.courant_dt()
        best = None
        for _ in range(3):
            plain.load_state(st)
            plain.set_sources(ijk, nd.reshape(-1, 1))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plain.step(dt, steps)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        plain.close()
        return best, dt

    target = None
    out = {}
    grads = {}
    for fp32 in (False, True):
        tp, dt = t_plain(fp32)
        ctx = RTContext.for_workload(w, counters=True, fp32=fp32)
        run = GradientRun(ctx, ijk, dt, steps, x0=w.xHII0, T0=w.T0, every=every)
        if target is None:
            target = run.forward(torch.tensor(ri.perturbed_log_rates(nd, w.seed)), lnnH).clone()
        times = []
        for _ in range(2):  # the first pass warms the allocator
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = run.forward(lnnd, lnnH)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g_src, g_nH = run.backward(2.0 * (x - target))[:2]
            torch.cuda.synchronize()
            times.append((t1 - t0, time.perf_counter() - t1))
        tf, tb = times[-1]
        grads[fp32] = (float(((x - target) ** 2).sum().item()), g_src.cpu().numpy(), g_nH.cpu().numpy())
        out["mixed" if fp32 else "fp64"] = {
            "forward_ms": tp * 1e3, "forward_checkpointed_ms": tf * 1e3, "backward_ms": tb * 1e3,
            "ratio": (tf + tb) / tp, "backward_only_ratio": tb / tp,
            "trace_entries_max": run.last_backward.get("trace_entries_max"),
            "grad_finite": bool(torch.isfinite(g_src).all().item() and torch.isfinite(g_nH).all().item())}
        ctx.close()
        del run, ctx
        torch.cuda.empty_cache()
    (L64, s64, n64), (L32, s32, n32) = grads[False], grads[True]
    rng = np.random.default_rng(5)
    dirs = [rng.standard_normal(n64.shape) for _ in range(4)]
    d64 = np.array([np.sum(n64 * v) for v in dirs])
    d32 = np.array([np.sum(n32 * v) for v in dirs])
    out["mixed_vs_fp64"] = {"loss": abs(L32 - L64) / abs(L64),
                            "source_gradients_e_inf": float(np.max(np.abs(s32 - s64)) / np.max(np.abs(s64))),
                            "source_gradients_max_rel": float(np.max(np.abs(s32 - s64) / np.abs(s64))),
                            "density_directions_max_rel": float(np.max(np.abs(d32 - d64) / np.abs(d64))),
                            "density_gradient_e_inf": float(np.max(np.abs(n32 - n64)) / np.max(np.abs(n64)))}
    f = out["fp64"]
    return {"workload": f"grey {w.n[0]}^3 x 1 group, H only, 16 sources, {steps} steps, checkpoints every {every}, "
                        "GLF, FP64 (and the mixed form)",
            "forward_ms": f["forward_ms"], "forward_checkpointed_ms": f["forward_checkpointed_ms"],
            "backward_ms": f["backward_ms"], "ratio": f["ratio"], "backward_only_ratio": f["backward_only_ratio"],
            "trace_entries_max": f["trace_entries_max"], "grad_finite": f["grad_finite"],
            "mixed": out["mixed"], "mixed_vs_fp64": out["mixed_vs_fp64"]}


def host_cpu():
    """Model name and logical CPUs of this host, and the threads the oracle
    may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity_cpus": avail}


def field_errors(a, b, M):
    """Error of state a against state b per field and group: the global-
    normalised e_inf = max|a-b| / max|b| and the distribution of the per-cell
    relative error over the cells with |b| > 1e-6 max|b| (quantiles and the
    fraction above 1e-5 and 1e-10); x_HI = 1 - x_HII as well."""
    import numpy as np

    def one(x, y):
        x = np.asarray(x, np.float64).ravel()
        y = np.asarray(y, np.float64).ravel()
        sc = float(np.max(np.abs(y)))
        if sc == 0.0:
            return {"e_inf": float(np.max(np.abs(x))), "cells": 0}
        m = np.abs(y) > 1e-6 * sc
        rel = np.abs(x[m] - y[m]) / np.abs(y[m])
        q = np.quantile(rel, [0.5, 0.9, 0.99, 0.999]) if rel.size else [0.0] * 4
        return {"e_inf": float(np.max(np.abs(x - y)) / sc), "cells": int(rel.size),
                "rel_p50": float(q[0]), "rel_p90": float(q[1]), "rel_p99": float(q[2]), "rel_p999": float(q[3]),
                "rel_max": float(rel.max()) if rel.size else 0.0,
                "frac_above_1e-5": float(np.mean(rel > 1e-5)) if rel.size else 0.0,
                "frac_above_1e-10": float(np.mean(rel > 1e-10)) if rel.size else 0.0}

    out = {}
    for g in range(M):
        out[f"N{g}"] = one(a["N"][g], b["N"][g])
        out[f"F{g}"] = one(a["F"][g], b["F"][g])
    for k in ("xHII", "xHeII", "xHeIII", "T"):
        out[k] = one(a[k], b[k])
    out["xHI"] = one(1.0 - np.asarray(a["xHII"]), 1.0 - np.asarray(b["xHII"]))
    return out


def timed_config(w, fp32, steps, warmup, ijk, nd, st=None, acct=False, chem_path="auto", path="auto"):
    """Run a workload on the GPU: `warmup` steps, back to the initial state,
    then `steps` timed rt_step calls.  Returns (context, ms per step, per-step
    series, stats)."""
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext
    st = st if st is not None else ri.initial_state(w)
    ctx = RTContext.for_workload(w, fp32=fp32)
    ctx.load_state(st)
    ctx.set_sources(ijk, ctx.source_rates(nd))
    ctx.set_chem_path(chem_path)
    ctx.set_transport_path(path)
    dt = ctx.courant_dt()
    if warmup > 0:
        ctx.step(dt, warmup)
        torch.cuda.synchronize()
        ctx.load_state(st)
    ctx.reset_stats()
    ctx.set_accounting(acct)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        ctx.step(dt, 1)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    series = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ctx, dt, wall * 1e3 / steps, series, ctx.stats()


def oracle_run(w, st, ijk, nd, steps, threads, label, dt=None, progress_every=1):
    """The oracle over `steps` steps from st (modified in place) on `threads`
    threads: (seconds, cell-group updates/s)."""
    import oracle
    oracle.set_threads(threads)
    o = oracle.OracleRT.for_workload(w)
    ndot = o.source_rates(nd) if ijk is not None and len(ijk) else None
    dt = dt if dt is not None else o.courant_dt()
    t_tot = 0.0
    for k in range(steps):
        t0 = time.perf_counter()
        o.step(st, dt, ijk if ndot is not None else None, ndot)
        t_tot += time.perf_counter() - t0
        if (k + 1) % progress_every == 0 or k + 1 == steps:
            print(f"# oracle {label}: step {k + 1}/{steps} on {threads} threads, {t_tot:.1f} s", file=sys.stderr,
                  flush=True)
    return t_tot, w.ncell * w.spectrum.M * steps / t_tot


def line(metric, value, unit, steps, warmup, ms, dtype, workload, higher=True, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": {"workload": workload}}
    out.update(extra)
    return out


def stromgren_radius(xHII, dx):
    """Radius of the sphere whose volume is the ionised volume of the full
    sphere the corner octant stands for."""
    import numpy as np
    V = 8.0 * float(np.sum(xHII)) * dx ** 3
    return (3.0 * V / (4.0 * np.pi)) ** (1.0 / 3.0)


def bench_stromgren(args):
    """C1: the isothermal H II region (Iliev test 1) on 32^3 x 1 group, FP64,
    GLF, 100 steps from the initial state; the ionised radius against the
    I-front law r_S (1 - exp(-t/t_rec))^(1/3) with case B recombination at
    1e4 K, and the oracle on the same steps."""
    import numpy as np

    import oracle
    import rt_inputs as ri
    steps = args.steps
    w = ri.stromgren_32(steps)
    ijk, nd = ri.workload_sources(w)
    ctx, dt, ms, series, s = timed_config(w, False, steps, args.warmup, ijk, nd, chem_path=args.chem_path,
                                          path=args.transport_path)
    g = ctx.state_numpy()
    nH = w.nH_mean
    alpha_B = 2.59e-13
    Ndot = 5e48
    rS = (3.0 * Ndot / (4.0 * np.pi * nH ** 2 * alpha_B)) ** (1.0 / 3.0)
    t = steps * dt
    t_rec = 1.0 / (alpha_B * nH)
    rI = stromgren_radius(g["xHII"], w.dx)
    st = ri.initial_state(w)
    t_o, cgu_o = oracle_run(w, st, ijk, nd, steps, oracle.threads(), "C1", dt=dt, progress_every=steps)
    err = field_errors(g, st, 1)
    print(json.dumps(line("RT cell-group updates/s, Stromgren sphere 32^3 x 1 group (FP64, GLF)",
                          w.ncell * steps / (ms * 1e-3 * steps), "cell-group updates/s", steps, args.warmup, ms,
                          "f64", "Iliev test 1: 32^3, 6.6 kpc, n_H 1e-3, x_HII 1.2e-3, T 1e4 K fixed, 13.6 eV, "
                                 "5e48/s corner source (1/8 injected), GLF, c_r = c/100",
                          series_ms=[round(v, 4) for v in series],
                          ifront={"t_Myr": t / 3.15576e13, "r_I_over_r_S": rI / rS,
                                  "law": float((1.0 - np.exp(-t / t_rec)) ** (1.0 / 3.0)), "alpha_B": alpha_B},
                          oracle={"seconds": t_o, "cgu_per_s": cgu_o, "threads": oracle.threads()},
                          gpu_vs_oracle={k: v["e_inf"] for k, v in err.items()})), flush=True)


def bench_plain128(args):
    """C2: 128^3 x 3 groups, FP64, HLL, 50 sources, 200 steps from the
    initial state; per-step series and the chemistry counters."""
    import rt_inputs as ri
    steps = 200 if args.steps == 100 else args.steps
    w = ri.lognormal_128(steps)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ctx, dt, ms, series, s = timed_config(w, False, steps, args.warmup, ijk, nd, chem_path=args.chem_path,
                                          path=args.transport_path)
    print(json.dumps(line("RT cell-group updates/s, 128^3 x 3 groups (FP64, HLL, 50 sources)",
                          w.ncell * 3 / (ms * 1e-3), "cell-group updates/s", steps, args.warmup, ms, "f64",
                          "lognormal 128^3 x 3 groups, 6.6 kpc, sigma_ln 1, mean n_H 1e-3, 50 sources, HLL, "
                          "c_r = c/100, FP64",
                          series_ms=[round(v, 4) for v in series],
                          chem={"substeps_per_cell_step": s["substeps_total"] / (w.ncell * steps),
                                "attempts_max": s["attempts_max"], "flags": s["flags"]})), flush=True)


def bench_precision(args):
    """C3's precision protocol: (i) mixed vs FP64 GPU on the full 256^3 grid
    after 100 steps; (ii) oracle vs FP64 GPU vs mixed GPU on the 64^3
    sub-box (cells [0,64)^3 and the sources in them, periodic) after 100
    steps.  Every comparison gives e_inf and the per-cell error
    distribution."""
    import torch

    import oracle
    import rt_inputs as ri
    steps = args.steps
    w = ri.lognormal_box(args.n, 13.2 * args.n / 256, max(1, round(200 * (args.n / 256) ** 3)), steps=steps,
                         seed=0)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    res, ms = {}, {}
    for fp32 in (False, True):
        print(f"# full grid {w.n[0]}^3, fp32={fp32}", file=sys.stderr, flush=True)
        ctx, dt, ms[fp32], _, _ = timed_config(w, fp32, steps, 0, ijk, nd)
        res[fp32] = ctx.state_numpy()
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    full = field_errors(res[True], res[False], 3)
    del res
    ws, st, sijk, snd = ri.subbox(w, 64)
    sub = {}
    for fp32 in (False, True):
        ctx, dt_s, _, _, _ = timed_config(ws, fp32, steps, 0, sijk, snd, st=st)
        sub[fp32] = ctx.state_numpy()
        ctx.close()
    ost = {k: v.copy() for k, v in st.items()}
    t_o, cgu_o = oracle_run(ws, ost, sijk, snd, steps, oracle.threads(), "C3 sub-box", dt=dt_s, progress_every=10)
    out = line("e_inf of the mixed-precision RT step (FP32 transport, FP64 chemistry) against FP64",
               max(v["e_inf"] for v in full.values()), "relative", steps, 0, ms[True], "f32 transport / f64 chemistry",
               f"lognormal {w.n[0]}^3 x 3 groups, {w.n_sources} sources, HLL, {steps} steps; 64^3 sub-box with "
               f"{ws.n_sources} sources", higher=False,
               full_grid={"mixed_vs_fp64_gpu": full, "ms_per_step": {"fp64": ms[False], "mixed": ms[True]}},
               subbox={"fp64_gpu_vs_oracle": field_errors(sub[False], ost, 3),
                       "mixed_gpu_vs_oracle": field_errors(sub[True], ost, 3),
                       "mixed_gpu_vs_fp64_gpu": field_errors(sub[True], sub[False], 3),
                       "oracle_seconds": t_o, "oracle_threads": oracle.threads()})
    print(json.dumps(out), flush=True)


def bench_oracle_timing(args):
    """The oracle's own throughput on this host at 1 thread and on all the
    threads it may use: C1 (100 steps), C2 (200 steps on all threads, the
    first 20 on one), the C3 64^3 sub-box (100 steps), late steps of the
    full 256^3 C3 grid from the FP64 GPU state after step 97 (3 on all
    threads, compared with the GPU's steps 98-100; 1 on one thread), and
    C5's forward run (300 steps)."""
    import torch

    import oracle
    import rt_inputs as ri
    full_threads = oracle.threads()
    out = {"host": host_cpu(), "threads_all": full_threads, "unit": "cell-group updates/s"}
    runs = {}

    def both(name, w, mk_state, ijk, nd, steps_all, steps_one, dt=None):
        r = {}
        for th, k in ((full_threads, steps_all), (1, steps_one)):
            st = mk_state()
            t, cgu = oracle_run(w, st, ijk, nd, k, th, f"{name}", dt=dt)
            r[f"threads_{th}"] = {"steps": k, "seconds": t, "value": cgu}
        runs[name] = r

    w1 = ri.stromgren_32(100)
    i1, n1 = ri.workload_sources(w1)
    both("C1 stromgren 32^3 x 1", w1, lambda: ri.initial_state(w1), i1, n1, 100, 100)
    w2 = ri.lognormal_128(200)
    i2, n2 = ri.random_sources(w2.n, w2.n_sources, w2.seed)
    both("C2 lognormal 128^3 x 3", w2, lambda: ri.initial_state(w2), i2, n2, 200, 20)
    w3 = ri.lognormal_256(100)
    ws, st3, si, sn = ri.subbox(w3, 64)
    both("C3 64^3 sub-box x 3", ws, lambda: {k: v.copy() for k, v in st3.items()}, si, sn, 100, 100)
    w5 = ri.grey_64(300)
    i5, n5 = ri.random_sources(w5.n, w5.n_sources, w5.seed)
    both("C5 grey 64^3 x 1 forward", w5, lambda: ri.initial_state(w5), i5, n5, 300, 300)
    # C3 late steps: the FP64 GPU state after 97 steps, then 3 steps on both
    from paper_1304_7126_amd import RTContext
    i3, n3 = ri.random_sources(w3.n, w3.n_sources, w3.seed)
    ctx = RTContext.for_workload(w3)
    ctx.load_state(ri.initial_state(w3))
    ctx.set_sources(i3, ctx.source_rates(n3))
    dt3 = ctx.courant_dt()
    ctx.step(dt3, 97)
    s97 = ctx.state_numpy()
    s97["nH"] = ctx.nH.cpu().numpy()
    ctx.step(dt3, 3)
    g100 = ctx.state_numpy()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    r = {}
    # one thread takes step 98 only (a minute or more of host time)
    for th, k in ((1, 1), (full_threads, 3)):
        st = {key: v.copy() for key, v in s97.items()}
        t, cgu = oracle_run(w3, st, i3, n3, k, th, "C3 256^3 from step 97", dt=dt3)
        r[f"threads_{th}"] = {"steps": k, "seconds": t, "value": cgu}
    r["fp64_gpu_vs_oracle_after_step_100"] = {k: v["e_inf"] for k, v in field_errors(g100, st, 3).items()}
    runs["C3 256^3 x 3 steps 98-100"] = r
    out["runs"] = runs
    print(json.dumps(out), flush=True)


def profile_figures(path, expect_window=None):
    """Figures of a profiles/ summary if it exists and its kernel-source hash
    is the current one (else None), with the reason."""
    from paper_1304_7126_amd import profiling
    f = profiling.read_figures(path)
    if f is None:
        return None, "missing"
    if f.get("kernel_source_hash") != profiling.kernel_source_hash():
        return None, "kernel sources changed since the profile was taken"
    if expect_window is not None and f.get("window") != list(expect_window):
        return None, f"profile window {f.get('window')} is not the timed launches {list(expect_window)}"
    return f, "ok"


def kernel_roofline(name, bytes_per_launch, ms_live, prefix, window, default_config):
    """Roofline entry of one kernel: algorithmic bytes over the live average
    launch duration against 8 TB/s, the profile's average duration over the
    same launches, the HBM bytes the counters saw, and the VALU figures."""
    achieved = bytes_per_launch / (ms_live * 1e-3) / 1e9
    r = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": bytes_per_launch,
         "ms_per_launch": ms_live}
    if not default_config:
        r["profile"] = "not the profiled configuration"
        return r
    # the summary set taken over these launches, if there is one
    for cand in PROFILE_SETS.get(prefix, [prefix]):
        if profile_figures(cand + "_kernel_stats.md", window)[0] is not None:
            prefix = cand
            break
    st, why = profile_figures(prefix + "_kernel_stats.md", window)
    by, why_b = profile_figures(prefix + "_pmc_bytes.md", window)
    va, why_v = profile_figures(prefix + "_pmc_valu.md", window)
    mx, _ = profile_figures(prefix + "_pmc_mix.md", window)
    r["profile"] = {"kernel_stats": os.path.relpath(prefix + "_kernel_stats.md", ROOT), "status": why}
    if st is not None:
        t = st["avg_us"] * 1e-6
        r["profile"].update({"avg_us": st["avg_us"], "frac_from_profile": bytes_per_launch / t / 1e9 / HBM_PEAK_GBS,
                             "live_over_profile": ms_live * 1e-3 / t})
    if by is not None:
        r["traffic"] = by["read_bytes"] + by["write_bytes"]
        r["traffic_read"] = by["read_bytes"]
        r["traffic_write"] = by["write_bytes"]
        r["traffic_over_algorithmic"] = r["traffic"] / bytes_per_launch
        r["traffic_source"] = os.path.relpath(prefix + "_pmc_bytes.md", ROOT)
    else:
        r["traffic_status"] = why_b
    if va is not None and st is not None:
        t = st["avg_us"] * 1e-6
        lane = va["SQ_THREAD_CYCLES_VALU"] / (64.0 * va["SQ_ACTIVE_INST_VALU"])
        alu = {"valu_issue_frac": va["SQ_INSTS_VALU"] / t / VALU_ISSUE_PEAK, "lane_util": lane,
               "wait_frac": va["SQ_WAIT_ANY"] / va["SQ_WAVE_CYCLES"],
               "source": os.path.relpath(prefix + "_pmc_valu.md", ROOT)}
        if mx is not None:
            f64 = sum(mx.get(f"SQ_INSTS_VALU_{k}_F64", 0.0) for k in ("ADD", "MUL", "FMA", "TRANS"))
            f32 = sum(mx.get(f"SQ_INSTS_VALU_{k}_F32", 0.0) for k in ("ADD", "MUL", "FMA", "TRANS"))
            fl64 = 64.0 * lane * (f64 + mx.get("SQ_INSTS_VALU_FMA_F64", 0.0)) / t
            alu.update({"fp64_instr_frac": f64 / va["SQ_INSTS_VALU"], "fp32_instr_frac": f32 / va["SQ_INSTS_VALU"],
                        "fp64_TFLOPs_active_lanes": fl64 / 1e12, "fp64_peak_TFLOPs": FP64_VECTOR_PEAK_TFLOPS,
                        "fp64_frac": fl64 / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                        "mix_source": os.path.relpath(prefix + "_pmc_mix.md", ROOT)})
        r["alu"] = alu
    else:
        r["alu_status"] = why_v
    return r


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the RT step is not sharded across GPUs, "
                                   "so --gpus must be 1"}))
        sys.exit(2)
    forms = {"batch": bench_batch, "shadow": bench_shadow, "stromgren": bench_stromgren,
             "plain128": bench_plain128, "precision": bench_precision, "oracle-timing": bench_oracle_timing}
    if args.form in forms:
        return forms[args.form](args)
    if args.form == "adjoint":
        a = adjoint_cost()
        print(json.dumps({"metric": "adjoint/forward cost ratio (checkpointed forward + reverse sweep over plain "
                          "forward)", "value": a["ratio"], "unit": "x",
                          "n_gpus": 1, "steps": 300, "warmup": 1, "ms_per_step": a["backward_ms"] / 300,
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": a["workload"]}, "adjoint": a}), flush=True)
        return
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fp32 = not args.fp64
    n = args.n
    acct = not args.no_accounting
    floor = args.n_floor if args.n_floor is not None else (1e-12 if args.smooth else 0.0)
    r = grid_run(n, fp32, args.flux, args.steps, args.warmup, args.head_attempts, args.smooth, floor,
                 otsa=not args.no_otsa, a=args.expansion, acct=acct, path=args.transport_path,
                 chem_path=args.chem_path)
    w, M, K, s, ms, cgu, per = r["w"], r["M"], args.steps, r["stats"], r["ms"], r["cgu"], r["per"]

    rad, gas = algorithmic_bytes(M, fp32)
    default_config = (fp32 and n == 256 and args.flux == "hll" and not args.smooth and floor == 0.0
                      and not args.no_otsa and args.expansion == 1.0 and acct and args.head_attempts == 0
                      and args.transport_path == "auto" and args.chem_path == "auto")
    window = (args.warmup + 1, args.warmup + K)
    split = per["transport"] > 0.0
    # the dominant kernel: the chemistry (one persistent pass after the
    # z-marching transport; on the per-cell path the head pass, fused with
    # the transport); it reads N, F and the gas state of every cell and
    # writes them back, the step's algorithmic traffic.  Its timing class
    # also holds the two small launches before it (counter reset, list of
    # long chains)
    one_pass = split and per["tail"] == 0.0
    name = ("k_chem_all (one-pass chemistry)" if one_pass else
            "k_head (first chemistry pass)" if split else "k_head (first chemistry pass, fused with the transport)")
    roof = kernel_roofline(name, w.ncell * (rad + gas), per["head"], PROFILE, window, default_config)
    roof["ms_per_launch_all"] = per
    roof["ms_per_step_by_class"] = r["per_step"]
    roof["step_algorithmic_GBps"] = w.ncell * (rad + gas) / (ms * 1e-3) / 1e9
    roof["step_frac"] = roof["step_algorithmic_GBps"] / HBM_PEAK_GBS
    if split:
        roof["transport"] = kernel_roofline("k_transport_z", w.ncell * rad, per["transport"], PROFILE_TRANSPORT,
                                            window, default_config)
    wl = f"lognormal {n}^3 x {M} groups, {w.n_sources} sources, {args.flux.upper()}, c_r=c/100, {K} steps"
    if args.smooth or floor > 0:
        wl += f"{', smoothed RT' if args.smooth else ''}, N_floor={floor:g}"
    if args.no_otsa:
        wl += ", no OTSA (case A, recombination photons)"
    if args.expansion != 1.0:
        wl += f", super-comoving at a={args.expansion:g}"
    if not acct:
        wl += ", no photon accounting"
    series = r["series"]
    out = {
        "metric": "RT cell-group updates/s at 256^3 x 3 groups; adjoint/forward cost ratio",
        "value": cgu,
        "unit": "cell-group updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 transport / f64 chemistry" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": wl,
                   "grid": [n, n, n], "groups": M, "flux": args.flux, "precision": "mixed" if fp32 else "fp64",
                   "smooth": bool(args.smooth), "otsa": not args.no_otsa, "N_floor": floor,
                   "photon_accounting": acct, "timed_steps": f"1-{K} from the initial state"},
        "series_ms": [round(v, 4) for v in series],
        "series_summary": {"first10_ms": sum(series[:10]) / min(10, K), "last10_ms": sum(series[-10:]) / min(10, K),
                           "max_ms": max(series), "min_ms": min(series)},
        "chem": {"substeps_per_cell_step": s["substeps_total"] / (w.ncell * K),
                 "attempts_per_cell_step": s["attempts_total"] / (w.ncell * K),
                 "attempts_max": s["attempts_max"], "flags": s["flags"]},
        "roofline": roof,
    }
    if acct:
        out["photon_budget"] = {k: s[k] for k in ("injected", "absorbed", "outflow", "photons") if k in s}
    torch.cuda.empty_cache()
    if args.smooth_steps > 0 and not args.smooth and not args.no_otsa and args.expansion == 1.0:
        out["smoothing"] = smoothing_comparison(n, fp32, args.flux, args.smooth_steps, args.warmup,
                                                args.head_attempts)
        torch.cuda.empty_cache()
        out["recombination_photons"] = otsa_comparison(n, fp32, args.flux, args.smooth_steps, args.warmup,
                                                       args.head_attempts)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        print("# adjoint cost (64^3 differentiation workload)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_cost()
        torch.cuda.empty_cache()
    if args.copy_calibration > 0:
        nb = args.copy_calibration * (1 << 20)
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": nb, "write": nb, "launches": 3}
        del a, b
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, n, M)
        out["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
