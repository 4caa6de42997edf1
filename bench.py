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

# Counter measurements of k_head<float, 3, 1, 1> on this workload (steps
# 101-105), valid for the kernel sources they were taken with
# (profiles/k_head_fused_256cube_3grp_pmc_bytes.md and _pmc_valu.md).
KERNEL_SOURCES = ("rt_kernels.hip", "rt_cell.h", "rt_device.h", "rt_internal.h")
COUNTERS_SOURCE_HASH = "49b77b76363506d5"
COUNTERS = {"read_bytes": 2534411 * 2 * 1024, "write_bytes": 3102981 * 1024, "valu_wave_instr": 3.1734e+09,
            "lane_util": 0.669, "fp64_flops_all_lanes": 1.173e+11, "ms": 5.595}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1304_7126_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
    ap.add_argument("--form", choices=["grid", "batch", "adjoint", "shadow"], default="grid",
                    help="grid: the 256^3 x 3 headline; batch: 64 uneven boxes, batched vs one-by-one; "
                         "shadow: Iliev test 3 (dense clump lit from the x = 0 face) at 128^3 to 15 Myr")
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
    x_HeII, x_HeIII, T (FP64, read and write), plus n_H (read)."""
    rb = 4 if fp32 else 8
    rad = 2 * 4 * rb * M
    gas = 2 * 4 * 8 + 8
    return rad, gas


def cpu_baseline(seconds, n_full, M):
    """The oracle on a 64^3 box of the same recipe (same cell size, sources
    scaled with volume), stepped until ~`seconds` of wall time."""
    import numpy as np

    import oracle
    import rt_inputs as ri
    n = 64
    w = ri.lognormal_box(n, 13.2 * n / n_full, max(1, round(200 * (n / n_full) ** 3)), steps=1, seed=0)
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ndot = o.source_rates(nd)
    dt = o.courant_dt()
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(st, dt, ijk, ndot)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    cgu = w.ncell * M * steps / el
    return {"value": cgu, "unit": "cell-group updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{n}^3 x {M} groups lognormal box (same recipe and cell size), first {steps} RT steps "
                      f"from the initial state, {el:.1f} s wall"}


def grid_run(n, fp32, flux_name, steps, warmup, head_attempts, smooth=False, floor=0.0, nH_mean=1e-3, otsa=True,
             a=1.0):
    """The lognormal n^3 x 3 workload: build it, run `warmup` steps, then time
    `steps` rt_step calls (injection, transport fused with the first
    chemistry pass, the compacted tail), with the library's HIP events
    bracketing each kernel on its stream."""
    import torch

    import rt_inputs as ri
    from paper_1304_7126_amd import RTContext
    flux = ri.FLUX_HLL if flux_name == "hll" else ri.FLUX_GLF
    w = ri.lognormal_box(n, 13.2 * n / 256, max(1, round(200 * (n / 256) ** 3)), steps=steps, seed=0, flux=flux)
    w.nH_mean = nH_mean
    w.otsa = otsa
    M = w.spectrum.M
    print(f"# building {n}^3 x {M} workload (mean n_H {nH_mean:g}, smooth={smooth}, N_floor={floor:g}, "
          f"otsa={otsa})", file=sys.stderr, flush=True)
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
    dt = ctx.courant_dt()
    if head_attempts > 0:
        ctx.set_tuning(head_attempts, -1)
    del st
    print(f"# warmup {warmup} steps", file=sys.stderr, flush=True)
    for _ in range(warmup):
        ctx.step(dt, 1)
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.set_timing(True)
    ctx.timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.timing()
    ctx.set_timing(False)
    s = ctx.stats()
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tm.items()}
    del ctx
    return {"w": w, "M": M, "stats": s, "ms": wall * 1e3 / steps, "cgu": w.ncell * M * steps / wall, "per": per}


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
    the plain forward run (rt_step, no checkpoints) on the same GPU."""
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
    plain = RTContext.for_workload(w)
    dt = plain.courant_dt()
    ctx = RTContext.for_workload(w, counters=True)
    run = GradientRun(ctx, ijk, dt, steps, x0=w.xHII0, T0=w.T0, every=every)

    def t_plain():
        plain.load_state(st)
        plain.set_sources(ijk, nd.reshape(-1, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain.step(dt, steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    target = run.forward(torch.tensor(ri.perturbed_log_rates(nd, w.seed)), lnnH).clone()
    tp = min(t_plain() for _ in range(3))
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
    return {"workload": f"grey {w.n[0]}^3 x 1 group, H only, 16 sources, {steps} steps, checkpoints every {every}, "
                        "GLF, FP64",
            "forward_ms": tp * 1e3, "forward_checkpointed_ms": tf * 1e3, "backward_ms": tb * 1e3,
            "ratio": (tf + tb) / tp, "backward_only_ratio": tb / tp,
            "trace_entries_max": run.last_backward.get("trace_entries_max"),
            "grad_finite": bool(torch.isfinite(g_src).all().item() and torch.isfinite(g_nH).all().item())}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.form == "batch":
        return bench_batch(args)
    if args.form == "shadow":
        return bench_shadow(args)
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
    floor = args.n_floor if args.n_floor is not None else (1e-12 if args.smooth else 0.0)
    r = grid_run(n, fp32, args.flux, args.steps, args.warmup, args.head_attempts, args.smooth, floor,
                 otsa=not args.no_otsa, a=args.expansion)
    w, M, K, s, ms, cgu, per = r["w"], r["M"], args.steps, r["stats"], r["ms"], r["cgu"], r["per"]

    rad, gas = algorithmic_bytes(M, fp32)
    step_bytes = w.ncell * (rad + gas)
    # the fused head kernel reads the source radiation set and the gas state
    # and writes the destination set and the gas state: the step's
    # algorithmic traffic; the tail re-touches only the queued cells
    t_head = per["head"]
    achieved = step_bytes / (t_head * 1e-3) / 1e9
    counters_valid = (kernel_source_hash() == COUNTERS_SOURCE_HASH and fp32 and n == 256 and args.flux == "hll"
                      and not args.smooth and floor == 0.0 and not args.no_otsa and args.expansion == 1.0)
    traffic = COUNTERS["read_bytes"] + COUNTERS["write_bytes"] if counters_valid else None
    # the kernel is bound by its VALU issue rate: counter figures over steps
    # 101-105 (instruction counts grow with the step as fronts develop),
    # divided by the duration of those same launches
    alu = None
    if counters_valid:
        t_c = COUNTERS["ms"] * 1e-3
        alu = {"valu_issue_frac": COUNTERS["valu_wave_instr"] / t_c / VALU_ISSUE_PEAK,
               "lane_util": COUNTERS["lane_util"],
               "fp64_active_lane_TFLOPs": COUNTERS["fp64_flops_all_lanes"] * COUNTERS["lane_util"] / t_c / 1e12,
               "fp64_peak_TFLOPs": FP64_VECTOR_PEAK_TFLOPS,
               "steps": "101-105", "ms_per_launch": COUNTERS["ms"],
               "source": "profiles/k_head_fused_256cube_3grp_pmc_valu.md"}
    roof = {"kernel": "k_head (transport fused with the first chemistry pass)", "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_source": "profiles/k_head_fused_256cube_3grp_pmc_bytes.md" if traffic else None,
            "alu": alu, "bytes_per_launch": step_bytes,
            "ms_per_launch": {"inject": per["inject"], "head": per["head"], "tail": per["tail"]},
            "step_algorithmic_GBps": step_bytes / (ms * 1e-3) / 1e9,
            "step_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    wl = f"lognormal {n}^3 x {M} groups, 200 sources, {args.flux.upper()}, c_r=c/100"
    if args.smooth or floor > 0:
        wl += f"{', smoothed RT' if args.smooth else ''}, N_floor={floor:g}"
    if args.no_otsa:
        wl += ", no OTSA (case A, recombination photons)"
    if args.expansion != 1.0:
        wl += f", super-comoving at a={args.expansion:g}"
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
                   "parallelism": "1 GPU"},
        "chem": {"substeps_per_cell_step": s["substeps_total"] / (w.ncell * K),
                 "attempts_per_cell_step": s["attempts_total"] / (w.ncell * K),
                 "attempts_max": s["attempts_max"], "flags": s["flags"]},
        "roofline": roof,
    }
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
