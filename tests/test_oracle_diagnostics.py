"""Pins of the oracle's step diagnostics: the photon budget of the operator
split (Sec. 3) -- photons per group, injected, carried out through the
boundary faces, absorbed by the chemistry -- and the substep histogram.

  - the boundary outflow (a sum of face fluxes at the grid's boundary
    faces) equals the change of the photon total over a transport step (a
    different computation: the transport's interior fluxes cancel in pairs);
  - a reflecting face carries no photons; a periodic grid has no boundary;
  - over many steps the ledger closes: photons(t) = photons(0) + injected -
    absorbed - outflow;
  - the histogram counts every cell once per step and its first moment is
    the substep total.
"""
import numpy as np
import pytest

import oracle
import rt_inputs as ri
from oracle import physics

C_R = ri.C_LIGHT / 100
DX = 6.6 * ri.KPC / 128


def make(n, bc, M=3, flux=1, Y=0.24):
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV={1: ri.EDGES_1, 2: ri.EDGES_2, 3: ri.EDGES_3}[M])
    sN, sE, eb, fr = physics.spectrum_attributes(spec)
    o = oracle.OracleRT(n=n, dx=DX, bc=bc, M=M, c_r=C_R, sigN=sN, sigE=sE, ebar=eb, flux=flux,
                        X=1 - Y, Y=Y)
    o.group_frac = fr[:M]
    return o


def state(n, M, rng, empty_frac=0.2):
    nx, ny, nz = n
    shp = (nz, ny, nx)
    N = 10 ** rng.uniform(-8, -3, (M,) + shp)
    N[rng.uniform(size=N.shape) < empty_frac] = 0.0
    d = rng.normal(size=(M, 3) + shp)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    F = d * rng.uniform(0, 1, (M, 1) + shp) * C_R * N[:, None]
    return {"N": N, "F": np.ascontiguousarray(F), "nH": 1e-3 * np.exp(rng.normal(0, 1, shp)),
            "xHII": 10 ** rng.uniform(-6, 0, shp), "xHeII": rng.uniform(0, 0.3, shp),
            "xHeIII": rng.uniform(0, 0.3, shp), "T": 10 ** rng.uniform(2, 4.7, shp)}


BCS = [(1,) * 6, (2, 1, 2, 1, 2, 1), (1, 1, 0, 0, 2, 2)]


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("bc", BCS)
def test_boundary_outflow_is_the_transport_loss(oracle_mod, bc, flux):
    rng = np.random.default_rng(11)
    n = (9, 7, 6)
    o = make(n, bc, flux=flux)
    st = state(n, 3, rng)
    dt = o.courant_dt()
    p0 = o.diagnostics(st)["photons"]
    out = o.boundary_outflow(st, dt)
    o.transport(st, dt)
    p1 = o.diagnostics(st)["photons"]
    assert np.all(np.abs((p0 - p1) - out) <= 1e-12 * p0), (p0 - p1, out)
    assert np.all(out != 0.0)


@pytest.mark.parametrize("flux", [0, 1])
def test_reflecting_and_periodic_faces_carry_nothing(oracle_mod, flux):
    rng = np.random.default_rng(12)
    n = (6, 5, 7)
    st = state(n, 3, rng)
    p = make(n, (2,) * 6, flux=flux).diagnostics(st)["photons"]
    out = make(n, (2,) * 6, flux=flux).boundary_outflow(st, 1e11)
    assert np.all(np.abs(out) <= 1e-12 * p)
    assert np.all(make(n, (0,) * 6, flux=flux).boundary_outflow(st, 1e11) == 0.0)


def test_inflow_face_counts_entering_photons_negative(oracle_mod):
    n = (6, 4, 4)
    o = oracle.OracleRT(n=n, dx=DX, bc=(3, 1, 1, 1, 1, 1), M=1, c_r=C_R, sigN=np.zeros((3, 3)),
                        sigE=np.zeros((3, 3)), ebar=np.zeros(3), flux=1, inflow=[[1e6], [0], [0], [0], [0], [0]])
    z = np.zeros((4, 4, 6))
    st = {"N": np.zeros((1, 4, 4, 6)), "F": np.zeros((1, 3, 4, 4, 6)), "xHII": z + 1, "xHeII": z.copy(),
          "xHeIII": z.copy(), "T": z + 1e4, "nH": z + 1e-3}
    dt = o.courant_dt()
    out = o.boundary_outflow(st, dt)
    # an empty grid lets in exactly F A dt through the lit face
    assert out[0] == pytest.approx(-1e6 * 16 * DX * DX * dt, rel=1e-14)


def test_diagnostics_are_the_plain_sums(oracle_mod):
    rng = np.random.default_rng(13)
    n = (8, 6, 5)
    o = make(n, (0,) * 6, M=2)
    st = state(n, 2, rng)
    dg = o.diagnostics(st)
    V = DX ** 3
    assert np.allclose(dg["photons"][:2], st["N"].reshape(2, -1).sum(axis=1) * V, rtol=1e-13, atol=0)
    assert dg["photons"][2] == 0.0
    assert dg["ionised_H"] == pytest.approx((st["xHII"] * st["nH"]).sum() * V, rel=1e-13)
    pos = st["N"] > 0
    f = np.linalg.norm(st["F"], axis=1)[pos] / (C_R * st["N"][pos])
    assert dg["max_f"] == pytest.approx(f.max(), rel=1e-14)
    assert dg["min_N"] == st["N"].min() == 0.0


@pytest.mark.parametrize("bc", [BCS[0], BCS[2]])
def test_ledger_closes_over_many_steps(oracle_mod, bc):
    rng = np.random.default_rng(14)
    n = (10, 8, 7)
    o = make(n, bc)
    st = state(n, 3, rng)
    ijk = np.array([[1, 2, 3], [9, 0, 3], [1, 2, 3]], np.int32)
    nd = o.source_rates(np.array([3e48, 1e49, 2e47]))
    dt = o.courant_dt()
    p0 = o.diagnostics(st)["photons"]
    led = None
    steps = 8
    for _ in range(steps):
        led = o.step_ledger(st, dt, ijk, nd, led)
    resid = led["photons"] - (p0 + led["injected"] - led["absorbed"] - led["outflow"])
    assert np.all(np.abs(resid) <= 1e-12 * (p0 + led["injected"]))
    assert np.all(led["absorbed"] > 0) and np.all(led["outflow"] != 0)
    assert np.allclose(led["injected"], nd.sum(axis=0) * dt * steps, rtol=1e-15, atol=0)
    h = led["substep_hist"]
    assert h.sum() == steps * np.prod(n)
    if h[63] == 0:
        assert (h * np.arange(64)).sum() == led["substeps_total"]
    assert led["attempts_total"] >= led["substeps_total"] and led["attempts_max"] >= 1
    assert led["flags"] == 0
