"""Precision form: FP32 N/F transport with FP64 chemistry against the FP64
oracle and the FP64 GPU path, field by field, on a 64^3 box of the 256^3
benchmark recipe (same cell size, density statistics and source rates).

The errors are written to precision_errors.json (in gpurun_out/ when that
folder exists) and bounded here:
  FP64 GPU vs oracle : e_inf <= 1e-10 on every field (measured ~1e-12)
  mixed  vs oracle   : e_inf <= 2e-6 on every field (measured <= 3.4e-7)
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri

pytestmark = pytest.mark.gpu

STEPS = 30


def errors(a, b):
    """global-normalised e_inf and the largest per-cell relative error over
    cells with |b| > 1e-6 max|b|."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    sc = np.max(np.abs(b))
    if sc == 0:
        return {"e_inf": float(np.max(np.abs(a))), "rel_max": 0.0}
    m = np.abs(b) > 1e-6 * sc
    rel = np.abs(a[m] - b[m]) / np.abs(b[m])
    return {"e_inf": float(np.max(np.abs(a - b)) / sc), "rel_max": float(rel.max()) if rel.size else 0.0,
            "rel_p99": float(np.quantile(rel, 0.99)) if rel.size else 0.0}


def field_errors(g, st, M):
    out = {}
    for gi in range(M):
        out[f"N{gi}"] = errors(g["N"][gi], st["N"][gi])
        out[f"F{gi}"] = errors(g["F"][gi], st["F"][gi])
    for k in ("xHII", "xHeII", "xHeIII", "T"):
        out[k] = errors(g[k], st[k])
    out["xHI"] = errors(1 - g["xHII"], 1 - st["xHII"])
    return out


def test_precision_form_errors_against_fp64():
    assert torch.cuda.is_available()
    from paper_1304_7126_amd import RTContext
    w = ri.lognormal_box(64, 13.2 * 64 / 256, 3, steps=STEPS, seed=0)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    res = {}
    for fp32 in (False, True):
        ctx = RTContext.for_workload(w, fp32=fp32)
        ctx.load_state(ri.initial_state(w))
        ctx.set_sources(ijk, ctx.source_rates(nd))
        dt = ctx.courant_dt()
        ctx.step(dt, STEPS)
        res[fp32] = ctx.state_numpy()
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    ondot = o.source_rates(nd)
    for _ in range(STEPS):
        o.step(st, dt, ijk, ondot)
    M = w.spectrum.M
    report = {"workload": f"lognormal 64^3 x {M} groups, same recipe as 256^3, {STEPS} steps",
              "fp64_gpu_vs_oracle": field_errors(res[False], st, M),
              "mixed_gpu_vs_oracle": field_errors(res[True], st, M),
              "mixed_gpu_vs_fp64_gpu": field_errors(res[True], res[False], M)}
    out_dir = "gpurun_out" if os.path.isdir("gpurun_out") else "."
    with open(os.path.join(out_dir, "precision_errors.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report["mixed_gpu_vs_oracle"]), flush=True)
    for k, v in report["fp64_gpu_vs_oracle"].items():
        assert v["e_inf"] <= 1e-10, (k, v)
    for k, v in report["mixed_gpu_vs_oracle"].items():
        assert v["e_inf"] <= 2e-6, (k, v)
