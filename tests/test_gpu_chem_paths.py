"""The one-pass chemistry kernel (persistent lanes that take the next cell
as soon as theirs has filled dt_RT, long chains of the previous pass first)
against the two-pass chemistry (a lockstep head pass, then the queued cells
in a persistent tail): the same bits in every field and the same counters,
for both precisions, one to three groups, smoothed RT and the case without
the on-the-spot approximation, over several steps of the split rt_step and
for rt_thermochem alone; with non-finite cells; with a list of long chains
larger than the room it has; and on a grid large enough (over the 262,144
lanes of the first fill) that most cells reach their lane as a refill."""
import numpy as np
import pytest
import torch

import rt_inputs as ri
from test_gpu_parity import gas, make_pair, random_rad

pytestmark = pytest.mark.gpu

FIELDS = ("N", "F", "xHII", "xHeII", "xHeIII", "T", "nacc", "natt")
COUNTS = ("substeps_total", "attempts_total", "attempts_max", "flags", "substep_hist")


def compare(a, b):
    ga, gb = a.state_numpy(), b.state_numpy()
    for k in FIELDS:
        assert np.array_equal(ga[k], gb[k], equal_nan=True), k
    sa, sb = a.stats(), b.stats()
    for k in COUNTS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    for k in ("injected", "absorbed", "outflow", "photons"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k
    return sa


def lognormal_pair(n, fp32, nH_mean, smooth=False, otsa=True, steps=4, spectrum=None, queue_cap=None):
    from paper_1304_7126_amd import RTContext
    w = ri.lognormal_box(n, 6.6 * n / 128, 6, steps=steps, seed=5, spectrum=spectrum)
    w.nH_mean = nH_mean
    w.otsa = otsa
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ctxs = []
    for path in ("two-pass", "one-pass"):
        c = RTContext.for_workload(w, fp32=fp32, counters=True, smooth=smooth, N_floor=1e-12 if smooth else 0.0)
        c.load_state(ri.initial_state(w))
        c.set_sources(ijk, c.source_rates(nd))
        c.set_transport_path("zmarch")
        c.set_chem_path(path)
        c.set_accounting(True)
        if queue_cap is not None:
            c.set_tuning(-1, queue_cap)
        c.reset_stats()
        ctxs.append(c)
    return w, ctxs


@pytest.mark.parametrize("fp32", [True, False])
@pytest.mark.parametrize("M", [1, 2, 3])
def test_one_pass_equals_two_pass_step(fp32, M):
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV={1: ri.EDGES_1, 2: ri.EDGES_2, 3: ri.EDGES_3}[M])
    # dense gas: I-front cells take tens to hundreds of attempts, so the
    # list of long chains is in use from the second step on
    w, (a, b) = lognormal_pair(24, fp32, 0.1, spectrum=spec, steps=6)
    dt = a.courant_dt()
    for _ in range(w.steps):
        a.step(dt, 1)
        b.step(dt, 1)
    s = compare(a, b)
    print(f"# one-pass vs two-pass M={M} fp32={fp32}: attempts max {s['attempts_max']}", flush=True)
    assert s["attempts_max"] >= 48


@pytest.mark.parametrize("smooth,otsa", [(True, True), (False, False), (True, False)])
def test_one_pass_equals_two_pass_variants(smooth, otsa):
    w, (a, b) = lognormal_pair(20, True, 0.03, smooth=smooth, otsa=otsa, steps=5)
    dt = a.courant_dt()
    for _ in range(w.steps):
        a.step(dt, 1)
        b.step(dt, 1)
    compare(a, b)


def test_one_pass_with_a_list_larger_than_its_room():
    # a queue of 7 cells: most long chains are not listed and go through
    # the sweep over all cells like any other
    w, (a, b) = lognormal_pair(24, True, 0.1, steps=6, queue_cap=7)
    dt = a.courant_dt()
    for _ in range(w.steps):
        a.step(dt, 1)
        b.step(dt, 1)
    s = compare(a, b)
    assert s["attempts_max"] >= 48


@pytest.mark.parametrize("fp32", [True, False])
def test_one_pass_thermochem_alone_with_a_nonfinite_cell(fp32):
    rng = np.random.default_rng(3)
    n = (37, 21, 19)
    N, F = random_rad(n, 3, rng)
    st = {"N": N, "F": F, **gas(n, rng)}
    st["T"][4, 5, 6] = np.nan
    st["N"][1, 7, 3, 2] = np.inf
    # a cell whose flux alone is not finite (the one-pass kernel finds it
    # only when it writes the cell)
    st["F"][2, 1, 10, 11, 12] = np.nan
    ctxs = []
    for path in ("two-pass", "one-pass"):
        c, _ = make_pair(n, (0,) * 6, 3, 1, fp32=fp32)
        c.load_state(st)
        c.set_chem_path(path)
        c.set_accounting(True)
        c.reset_stats()
        ctxs.append(c)
    dt = ctxs[0].courant_dt()
    for c in ctxs:
        for _ in range(3):
            c.thermochem(dt)
    s = compare(*ctxs)
    assert s["flags"] & 2


@pytest.mark.parametrize("fp32", [True, False])
def test_one_pass_refills_on_a_large_grid(fp32):
    # 96^3 cells: 3.4x the lanes of the first fill, so that most cells are
    # taken by lanes whose previous cell is done
    w, (a, b) = lognormal_pair(96, fp32, 0.03, steps=3)
    for c in (a, b):
        st = c.state_numpy()
        st["nH"] = c.nH.cpu().numpy()
        # non-finite inputs late in the grid: a flux, a density, a temperature
        st["F"][1, 2, 90, 91, 92] = np.nan
        st["N"][0, 80, 3, 4] = np.inf
        st["T"][70, 60, 50] = np.nan
        c.load_state(st)
    dt = a.courant_dt()
    for _ in range(w.steps):
        a.step(dt, 1)
        b.step(dt, 1)
    s = compare(a, b)
    assert s["flags"] & 2
