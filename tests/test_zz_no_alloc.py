"""rt_step_noalloc (the step in the library's static per-GPU scratch array,
for callers that cannot allocate) against rt_step with bound scratch: the
same bits on two calls in a row, the second on a smaller grid (the array
keeps the first call's contents), in mixed precision and FP64, on both
transport paths; grids too large for the array and contexts without
scratch are refused."""
import numpy as np
import pytest
import torch

import rt_inputs as ri

pytestmark = pytest.mark.gpu

FIELDS = ("N", "F", "xHII", "xHeII", "xHeIII", "T", "nacc", "natt")


def ctx_pair(n, fp32, path, nsrc):
    from paper_1304_7126_amd import RTContext
    w = ri.lognormal_box(n, 6.6 * n / 128, nsrc, steps=5, seed=n)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    st = ri.initial_state(w)
    out = []
    for scratch in (True, False):
        c = RTContext.for_workload(w, fp32=fp32, counters=True, scratch=scratch)
        c.load_state(st)
        c.set_sources(ijk, c.source_rates(nd))
        c.set_transport_path(path)
        out.append(c)
    return w, out


@pytest.mark.parametrize("fp32,path", [(True, "auto"), (False, "auto"), (True, "cell")])
def test_step_noalloc_equals_step_on_two_calls(fp32, path):
    assert torch.cuda.is_available()
    for n, nsrc in ((40, 12), (24, 5)):
        w, (ref, na) = ctx_pair(n, fp32, path, nsrc)
        dt = ref.courant_dt()
        print(f"# noalloc {n}^3 fp32={fp32} path={path}", flush=True)
        ref.step(dt, w.steps)
        na.step_noalloc(dt, w.steps)
        ga, gb = ref.state_numpy(), na.state_numpy()
        for k in FIELDS:
            assert np.array_equal(ga[k], gb[k]), (n, k)
        assert int(gb["natt"].max()) > 10  # cells subcycled (the queue was used)


def test_step_noalloc_refuses_what_it_cannot_hold():
    from paper_1304_7126_amd import RTContext
    from paper_1304_7126_amd.capi import RTError
    w = ri.lognormal_box(24, 6.6 * 24 / 128, 3, steps=1, seed=2)
    c = RTContext.for_workload(w, fp32=True, scratch=False)
    c.load_state(ri.initial_state(w))
    with pytest.raises(RTError):
        c.step(c.courant_dt(), 1)  # no scratch bound
    with pytest.raises(RTError):
        c.stats()
    c.step_noalloc(c.courant_dt(), 1)
    # 512 x 512 x 256 cells need more than the 64 MiB array beside the queue
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV=ri.EDGES_1)
    from paper_1304_7126_amd.runtime import spectrum_attributes
    sN, sE, eb, _ = spectrum_attributes(spec)
    big = RTContext(n=(512, 512, 256), dx=1e20, bc=(0,) * 6, M=1, c_r=3e8, sigN=sN, sigE=sE, ebar=eb, fp32=True,
                    scratch=False)
    with pytest.raises(RTError, match="static buffer"):
        big.step_noalloc(big.courant_dt(), 1)
