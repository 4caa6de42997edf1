"""Parity at the benchmark's full size: 256^3 x 3 groups in the launch
configuration bench.py times (rt_step: injection, the z-marching transport,
the one-pass chemistry, the photon accounting), plain, smoothed and without
OTSA, and the dense-gas variant; 128^3 x 3 in FP64 over 200 steps.  After
some steps on the GPU the pre-step
state is copied to the host, the oracle steps sampled cells one by one from
it (or_step_cells), and the GPU's next rt_step is compared on those cells."""
import numpy as np
import pytest
import torch

import oracle
import rt_inputs as ri

pytestmark = pytest.mark.gpu


def host_state(ctx):
    torch.cuda.synchronize()
    N, F = ctx.radiation()
    return {"N": N.double().cpu().numpy(), "F": F.double().cpu().numpy(),
            "xHII": ctx.xHII.cpu().numpy(), "xHeII": ctx.xHeII.cpu().numpy(),
            "xHeIII": ctx.xHeIII.cpu().numpy(), "T": ctx.T.cpu().numpy(), "nH": ctx.nH.cpu().numpy()}


# FP32 transport: photon densities and fluxes below ~10x the smallest
# normal FP32 number (1.2e-38) are held as subnormals, without relative
# precision; where some group's density is below 1e-30 over a cell's whole
# stencil, the transport of that group is at the bottom of the format
FP32_FLOOR = 1e-37
FP32_DARK = 1e-30
# relative rounding of the FP32 transport's result: a few ulps (2^-21 = 4
# ulps of FP32) over its ~50 operations per group
FP32_EPS = 2.0 ** -21


def run_and_sample(w, steps_before, fp32=False, smooth=False, floor=0.0, nsample=2048, ctx=None, done=0,
                   spread_eps=None, dark=None):
    """Run the workload on the GPU to `steps_before` steps (continuing `ctx`
    after `done` steps if given), copy the pre-step state to the host, take
    one more rt_step, and compare it on sampled cells (random cells, the
    1,024 cells with most attempts in the previous step, the source cells
    and their neighbours) with the oracle stepping those cells one by one
    from the same pre-step state.  Returns the context for a later call."""
    assert torch.cuda.is_available()
    from paper_1304_7126_amd import RTContext
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    if ctx is None:
        ctx = RTContext.for_workload(w, fp32=fp32, counters=True, smooth=smooth, N_floor=floor)
        ctx.load_state(ri.initial_state(w))
        ctx.set_sources(ijk, ctx.source_rates(nd))
        ctx.set_accounting(True)
    dt = ctx.courant_dt()
    if steps_before > done:
        ctx.step(dt, steps_before - done)
    pre = host_state(ctx)
    natt_prev = ctx.natt.cpu().numpy().ravel()
    ctx.step(dt, 1)
    g = ctx.state_numpy()
    print(f"# {w.n[0]}^3 mean n_H {w.nH_mean:g} fp32={fp32} smooth={smooth} otsa={w.otsa}: step "
          f"{steps_before + 1} sampled", flush=True)

    o = oracle.OracleRT.for_workload(w, N_floor=floor)
    assert o.courant_dt() == dt
    N_pre = pre["N"].copy() if smooth else None
    o.inject(pre, dt, ijk, o.source_rates(nd))
    cells = sample_cells(w, ijk, natt_prev if steps_before > 0 else None, nsample, steps_before)
    r = o.step_cells(pre, dt, cells, N_pre=N_pre)
    spread = perturbed_oracle(o, pre, dt, cells, spread_eps, N_pre=N_pre) if spread_eps else None
    compare_sampled(w, pre, g, cells, r, 1e-5 if fp32 else 1e-10, spread=spread, dark=dark,
                    abs_floor=FP32_FLOOR if fp32 else 0.0)
    return ctx, r


def sample_cells(w, ijk, natt_prev, nsample, seed):
    """Random cells, the 1,024 cells with most attempts in the previous
    step (if known), the source cells and their +x and +y neighbours."""
    rng = np.random.default_rng(seed)
    nc = w.ncell
    src_cells = (ijk[:, 0] + w.n[0] * (ijk[:, 1] + w.n[1] * ijk[:, 2])).astype(np.int64)
    heavy = np.argsort(natt_prev)[-1024:] if natt_prev is not None else np.zeros(0, np.int64)
    return np.unique(np.concatenate([rng.integers(0, nc, nsample), heavy, src_cells,
                                     np.minimum(src_cells + 1, nc - 1), np.minimum(src_cells + w.n[0], nc - 1)]))


def perturbed_oracle(o, pre, dt, cells, eps, seed=1, N_pre=None):
    """The oracle's step of the sampled cells from the injected pre-step
    state with every N and F value scaled by 1 +- eps, once with random signs
    and once all by 1 + eps (rounding that is the same across a stencil, as
    that of the FP32 constants): the spread of the results measures how
    strongly the step amplifies a relative perturbation of its input of
    that size."""
    rng = np.random.default_rng(seed)
    out = []
    for signs in ("random", "same"):
        p = dict(pre)
        for k in ("N", "F"):
            sg = rng.choice([-1.0, 1.0], pre[k].shape) if signs == "random" else 1.0
            p[k] = pre[k] * (1 + eps * sg)
        out.append(o.step_cells(p, dt, cells, N_pre=N_pre))
    return out


def compare_sampled(w, pre, g, cells, r, tol, spread=None, K=10.0, dark=None, abs_floor=0.0):
    """The GPU's step (g: whole-grid state after it) against the oracle's
    results r on the sampled cells, from the injected pre-step state pre.

    Cells whose accepted-substep and attempt counts match the oracle's are
    compared field by field; the others (a 10%-rule decision taken on the
    other side of its threshold) are counted.  With `spread` (the oracle's
    results from inputs perturbed by the rounding of the GPU's transport
    precision, see perturbed_oracle) every limit grows by K times the
    oracle's largest change, and cells whose counts a perturbation changes
    may also change on the GPU.  With `dark`, cells where some group's
    photon density is below it over the whole 7-point stencil (densities at
    the bottom of the floating-point range of the transport, whose rounding
    differs between implementations) may take other substep counts; their
    gas state must still agree (to 1e-8, or the limits of tol and spread).
    abs_floor: absolute slack on N and F for values below the normal range
    of the transport's format."""
    M = w.spectrum.M
    gN = g["N"].reshape(M, -1)[:, cells].T
    gF = g["F"].reshape(M, 3, -1)[:, :, cells].transpose(2, 0, 1)
    gx = np.stack([g[k].ravel()[cells] for k in ("xHII", "xHeII", "xHeIII")], axis=1)
    gT = g["T"].ravel()[cells]
    same = (g["nacc"].ravel()[cells] == r["nacc"]) & (g["natt"].ravel()[cells] == r["natt"])
    # max of the injected pre-step N over each sampled cell's periodic stencil
    nx, ny, nz = w.n
    ix, iy, iz = cells % nx, (cells // nx) % ny, cells // (nx * ny)
    nstencil = []
    for gi in range(M):
        Ng = pre["N"][gi]
        m = Ng[iz, iy, ix].copy()
        for dz, dy, dx_ in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            m = np.maximum(m, Ng[(iz + dz) % nz, (iy + dy) % ny, (ix + dx_) % nx])
        nstencil.append(m)
    ds = {k: np.zeros_like(v, dtype=np.float64) for k, v in r.items() if k in ("N", "F", "x", "T")}
    free = np.zeros_like(same)
    for sp in spread or ():
        for k in ds:
            ds[k] = np.maximum(ds[k], K * np.abs(sp[k] - r[k]))
        free |= (sp["nacc"] != r["nacc"]) | (sp["natt"] != r["natt"])
    if dark is not None:
        dk = np.any(np.stack(nstencil, axis=1) < dark, axis=1)
        fd = ~same & dk
        if np.any(fd):
            # another substep schedule integrates the same equations with the
            # 10% rule's error control: the results differ by a fraction of
            # the step's change
            gtol = max(tol, 1e-8)
            for q, k in enumerate(("xHII", "xHeII", "xHeIII")):
                err = np.abs(gx[fd, q] - r["x"][fd, q])
                chg = np.abs(r["x"][fd, q] - pre[k].ravel()[cells][fd])
                assert np.all(err <= 0.1 * chg + gtol * np.abs(r["x"][fd, q]) + 1e-15 + ds["x"][fd, q]), \
                    ("dark x", q, err.max())
            chg = np.abs(r["T"][fd] - pre["T"].ravel()[cells][fd])
            assert np.all(np.abs(gT[fd] - r["T"][fd]) <= 0.1 * chg + gtol * r["T"][fd] + ds["T"][fd]), "dark T"
        free |= dk
    flip = 1 - (same | free).mean()
    print(f"sampled {cells.size} cells: {int((~same).sum())} with other counts, {int(free.sum())} allowed to "
          f"(flip fraction outside them {flip:.2e})", flush=True)
    assert flip <= 5e-3, flip
    # Near full ionisation x_HI = 1 - x is ill-conditioned: x agrees to a few
    # ulps (~1e-16 absolute), so x_HI and with it the absorption factor
    # 1/(1 + h c sigma n_HI) of every substep differ by ~1e-16/x_HI relative;
    # over the step's optical depth (<~ 100) N and F pick up ~1e-14/x_HI.
    xhi = np.maximum(1.0 - r["x"][:, 0], 1e-6)
    rtol = tol + 1e-14 / xhi
    for gi in range(M):
        sc = np.max(np.abs(r["N"][:, gi]))
        err = np.abs(gN[same, gi] - r["N"][same, gi])
        # the transport rounds on the scale of the stencil's densities (FP32:
        # ~1e-6 of them); FP64 keeps the tighter global floor alone
        lim = (rtol[same] * np.abs(r["N"][same, gi]) + tol * 1e-3 * sc + ds["N"][same, gi] + abs_floor
               + (tol * nstencil[gi][same] if tol >= 1e-6 else 0.0))
        iw = np.argmax(np.where(lim > 0, err / np.where(lim > 0, lim, 1.0), 0.0))
        print(f"N{gi}: worst err/limit {err[iw] / lim[iw]:.3g} (x_HI {xhi[same][iw]:.3g})", flush=True)
        assert np.all(err <= lim), (gi, err.max())
        # F on the scale of the local radiation: the transport update adds
        # terms of order c_r N of the stencil, so |F| << c_r N comes out of
        # a cancellation; the error is bounded relative to |F| and, as a
        # reduced-flux error, relative to c_r max(N over the 7-point stencil)
        Fn = np.linalg.norm(r["F"][same, gi], axis=1)
        errF = np.linalg.norm(gF[same, gi] - r["F"][same, gi], axis=1)
        limF = (rtol[same] * Fn + tol * w.c_r * nstencil[gi][same] + np.linalg.norm(ds["F"][same, gi], axis=1)
                + abs_floor)
        iw = np.argmax(np.where(limF > 0, errF / np.where(limF > 0, limF, 1.0), 0.0))
        print(f"F{gi}: worst err/limit {errF[iw] / limF[iw]:.3g} (|F| {Fn[iw]:.3g}, c_r N_stencil "
              f"{w.c_r * nstencil[gi][same][iw]:.3g}, x_HI {xhi[same][iw]:.3g})", flush=True)
        assert np.all(errF <= limF), (gi, errF.max())
    for q in range(3):
        err = np.abs(gx[same, q] - r["x"][same, q])
        assert np.all(err <= tol * np.abs(r["x"][same, q]) + 1e-15 + ds["x"][same, q]), (q, err.max())
    assert np.all(np.abs(gT[same] - r["T"][same]) <= tol * r["T"][same] + ds["T"][same])
    # x_HI = 1 - x near full ionisation
    xhi_err = np.abs((1 - gx[same, 0]) - (1 - r["x"][same, 0]))
    assert np.all(xhi_err <= tol * 1e3 * np.maximum(1 - r["x"][same, 0], 1e-6) + ds["x"][same, 0])


# smoothed RT (Sec. 4.4) runs with a photon floor of 1e-12 cm^-3; otsa =
# False: case A with recombination photons (Sec. 3.3.2)
@pytest.mark.parametrize("fp32,smooth,otsa", [(False, False, True), (True, False, True), (True, True, True),
                                              (True, False, False)])
def test_256_cubed_sampled_cells_match_oracle(fp32, smooth, otsa):
    w = ri.lognormal_256(steps=12)
    w.otsa = otsa
    floor = 1e-12 if smooth else 0.0
    ctx, r = run_and_sample(w, w.steps, fp32=fp32, smooth=smooth, floor=floor)
    assert int(r["natt"].max()) > 10  # the sample contains subcycling cells


@pytest.mark.parametrize("fp32,floor", [(False, 1e-12), (True, 1e-12), (False, 0.0)])
def test_256_cubed_dense_gas_sampled_cells_match_oracle(fp32, floor):
    # the benchmark's dense variant (mean n_H 0.1): the sources' photons are
    # absorbed within a step, I-fronts are one cell wide and the cells next
    # to them subcycle hundreds of times; no photon density goes negative.
    # The chemistry there amplifies a relative change of its photon input
    # by up to ~1e3 (measured on the oracle), so FP32 transport is held to
    # the oracle's own response to FP32 rounding of its input.  Without a
    # photon floor the dark cells behind the fronts carry densities at the
    # bottom of the FP64 range (1e-160 to 1e-323), which the 10% rule
    # subcycles thousands of times: their substep counts depend on the
    # rounding of those numbers and may differ, their gas state may not.
    w = ri.lognormal_256(steps=12)
    w.nH_mean = 0.1
    ctx, r = run_and_sample(w, w.steps, fp32=fp32, floor=floor, spread_eps=FP32_EPS if fp32 else None,
                            dark=FP32_DARK if fp32 else (1e-150 if floor == 0.0 else None))
    assert int(r["natt"].max()) > 50
    s = ctx.stats()
    assert s["flags"] == 0, s["flags"]
    assert s["min_N"] >= 0.0


def test_128_cubed_plain_fp64_at_steps_1_100_200():
    # the 128^3 x 3 workload of the plain method in FP64 (HLL, 50 sources,
    # 200 steps): sampled cells against the oracle at the first, the 100th
    # and the last step; no anomaly flag over the run
    w = ri.lognormal_128(steps=200)
    ctx, r = run_and_sample(w, 0)
    done = 1
    for k in (99, 199):
        ctx, r = run_and_sample(w, k, ctx=ctx, done=done)
        done = k + 1
    assert int(r["natt"].max()) > 10
    s = ctx.stats()
    assert s["flags"] == 0, s["flags"]
    assert s["min_N"] >= 0.0
