"""Autotuner for the launch shape of the RT step.

It times candidate launch configurations on the caller's own workload (the
state is snapshotted and restored between candidates, so the tuning leaves
the simulation untouched; results never depend on the configuration) and
caches the winner in a JSON file keyed by a signature of the workload and the
GPU.  Tunables: for the single-grid step, the chemistry attempts per cell in
the fused first pass; for the batched step, also the persistent head grid
(blocks per compute unit) and the tail grid."""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import torch

CACHE = os.environ.get("RTM1_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rtm1_tune.json"))


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    except OSError:
        pass


def _gpu_name():
    try:
        return torch.cuda.get_device_name()
    except Exception:
        return "unknown"


def batch_signature(batch):
    shapes = sorted((b.n, b.M) for b in batch.boxes)
    h = hashlib.sha1(json.dumps([shapes, batch.fp32, _gpu_name()]).encode()).hexdigest()[:16]
    return "batch:" + h


def tune_batch(batch, dt, trial_steps=3, head_blocks=(2, 4, 8), head_attempts=(1, 2, 3, 4),
               tail_blocks=(512, 1024, 2048), use_cache=True, verbose=False):
    """Pick the fastest (head_blocks_per_cu, head_attempts, tail_blocks) for
    this batch by timing `trial_steps` graph-launched steps of each candidate
    from the same snapshot.  Applies and returns the winner."""
    key = batch_signature(batch)
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]["config"]
        batch.set_tuning(*best, 1)
        return {"config": best, "cached": True}
    snap = batch.snapshot()
    results = []
    for hb, ha, tb in itertools.product(head_blocks, head_attempts, tail_blocks):
        batch.restore(snap)
        batch.set_tuning(hb, ha, tb, 1)
        batch.step(dt, 1)  # graph capture and warm-up
        batch.synchronize()
        t0 = time.perf_counter()
        batch.step(dt, trial_steps)
        batch.synchronize()
        t = (time.perf_counter() - t0) / trial_steps
        results.append((t, (hb, ha, tb)))
        if verbose:
            print(f"  tune hb={hb} K={ha} tb={tb}: {t * 1e3:.3f} ms/step", flush=True)
    batch.restore(snap)
    results.sort()
    best = list(results[0][1])
    batch.set_tuning(*best, 1)
    if use_cache:
        cache[key] = {"config": best, "ms_per_step": results[0][0] * 1e3}
        _save(cache)
    return {"config": best, "cached": False, "trials": [(r[0] * 1e3, r[1]) for r in results]}


def tune_grid(ctx, dt, trial_steps=3, head_attempts=(1, 2, 3, 4, 6), verbose=False):
    """Pick the fastest head_attempts for a single-grid context (state is
    restored afterwards)."""
    torch.cuda.synchronize()
    saved = [t.clone() for t in (ctx.N, ctx.F, ctx.xHII, ctx.xHeII, ctx.xHeIII, ctx.T)]
    cur = ctx.current
    res = []
    for K in head_attempts:
        for t, s in zip((ctx.N, ctx.F, ctx.xHII, ctx.xHeII, ctx.xHeIII, ctx.T), saved):
            t.copy_(s)
        from .capi import lib
        lib().rt_set_current(ctx._h, cur)
        ctx.set_tuning(K, -1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(dt, trial_steps)
        torch.cuda.synchronize()
        res.append(((time.perf_counter() - t0) / trial_steps, K))
        if verbose:
            print(f"  tune K={K}: {res[-1][0] * 1e3:.3f} ms/step", flush=True)
    for t, s in zip((ctx.N, ctx.F, ctx.xHII, ctx.xHeII, ctx.xHeIII, ctx.T), saved):
        t.copy_(s)
    from .capi import lib
    lib().rt_set_current(ctx._h, cur)
    res.sort()
    ctx.set_tuning(res[0][1], -1)
    return {"head_attempts": res[0][1], "trials": [(r[0] * 1e3, r[1]) for r in res]}
