"""Pins of the oracle's boundary-flux source (the x = 0 face of Iliev test 3,
Sec. 6): a face whose ghost cell holds a beam of photon flux F entering the
box (N = F / c_r, reduced flux 1).

  - without absorbers the box fills with the beam, N = F / c_r and
    F_x = F everywhere, for HLL and GLF, and the face lets in F A dt per
    step;
  - a plane I-front in neutral hydrogen moves at c_r F / (n c_r + F), the
    speed photon counting gives when the ionised region holds the beam at
    N = F / c_r (the front is limited by the reduced light speed, as Sec. 6
    notes for test 3);
  - a dense clump casts a shadow: at 1 Myr the gas behind it on the axis is
    neutral while the gas beside it at the same depth is ionised, and the
    clump's core is neutral.
"""
import math

import numpy as np
import pytest

import oracle
import rt_inputs as ri

C = 2.99792458e10
KPC = ri.KPC


def beam_box(nx, flux, sig=0.0, isothermal=True, nH=2e-4, c_r=C / 10, dx=0.1 * KPC):
    s = np.zeros((3, 3))
    s[0, 0] = sig
    inflow = np.zeros((6, 1))
    inflow[0, 0] = 1e6
    bc = (ri.BC_INFLOW, ri.BC_OUTFLOW, 0, 0, 0, 0)
    o = oracle.OracleRT(n=(nx, 2, 2), dx=dx, bc=bc, M=1, c_r=c_r, sigN=s, sigE=s.copy(),
                        ebar=np.array([13.6 * 1.602176634e-12, 0, 0]), flux=flux, isothermal=isothermal,
                        X=1.0, Y=0.0, inflow=inflow)
    shp = (2, 2, nx)
    st = {"N": np.zeros((1,) + shp), "F": np.zeros((1, 3) + shp), "nH": np.full(shp, nH),
          "xHII": np.full(shp, 1e-6), "xHeII": np.zeros(shp), "xHeIII": np.zeros(shp), "T": np.full(shp, 1e4)}
    return o, st


@pytest.mark.parametrize("flux", [ri.FLUX_HLL, ri.FLUX_GLF])
def test_empty_box_fills_with_the_beam(oracle_mod, flux):
    o, st = beam_box(12, flux)
    dt = o.courant_dt()
    for _ in range(800):
        o.transport(st, dt)
    c_r = C / 10
    assert np.allclose(st["N"][0], 1e6 / c_r, rtol=1e-12, atol=0)
    assert np.allclose(st["F"][0, 0], 1e6, rtol=1e-12, atol=0)
    assert np.max(np.abs(st["F"][0, 1:])) < 1e-12 * 1e6
    # one more step changes nothing: what enters leaves through x = L
    N0 = st["N"].copy()
    o.transport(st, dt)
    assert np.allclose(st["N"], N0, rtol=1e-14, atol=0)


def test_first_step_lets_in_F_A_dt(oracle_mod):
    o, st = beam_box(12, ri.FLUX_HLL)
    dt = o.courant_dt()
    o.transport(st, dt)
    dx = o.dx
    entered = st["N"].sum() * dx ** 3
    assert entered == pytest.approx(1e6 * (2 * dx) * (2 * dx) * dt, rel=1e-12)
    # the HLL beam enters the first cell only (upwind in x)
    assert np.all(st["N"][0, :, :, 1:] == 0.0)


def test_plane_front_follows_the_finite_light_speed_law(oracle_mod):
    # n = 2e-4 and F = 1e6 of test 3's diffuse gas: F / (n c_r) = 1.67, so
    # the front moves at 0.625 c_r; sigma = 6.3e-18 (mean free path 0.26 kpc)
    nx, dx = 96, 0.05 * KPC
    o, st = beam_box(nx, ri.FLUX_HLL, sig=6.3e-18, dx=dx)
    dt = o.courant_dt()
    c_r, n, F = C / 10, 2e-4, 1e6
    v = c_r * F / (n * c_r + F)
    t = 0.0
    for k in range(1, 301):
        assert o.step(st, dt) == 0
        t += dt
        if k % 100 == 0:
            # ionised column along x (the front's position)
            R = st["xHII"][0, 0].sum() * dx
            assert abs(R - v * t) < 2.0 * dx, (k, R / dx, v * t / dx)


def test_dense_clump_casts_a_shadow(oracle_mod):
    w = ri.shadow_clump(32)
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    dt = o.courant_dt(w.courant)
    steps = int(round(1.0 * 3.15576e13 / dt))  # 1 Myr
    worst = 0.0
    for _ in range(steps):
        # HLL is not positive in 3D: a cell in the shadow may dip below zero
        # by ~1e-25 of the beam's density (flag bit 3), nothing more
        assert o.step(st, dt) & ~8 == 0
        worst = min(worst, st["N"].min() / st["N"].max())
    assert worst > -1e-20
    dx = w.dx

    def x_at(x_kpc, y_kpc, z_kpc):
        i, j, k = (int(v * KPC / dx) for v in (x_kpc, y_kpc, z_kpc))
        return st["xHII"][k, j, i]

    assert x_at(2.0, 3.3, 3.3) > 0.9     # diffuse gas in front of the clump
    assert x_at(5.0, 3.3, 3.3) < 0.01    # clump core
    assert x_at(6.3, 3.3, 3.3) < 0.1     # behind the clump on the axis
    assert x_at(6.3, 1.0, 3.3) > 0.9     # beside it, same depth
    assert x_at(6.3, 3.3, 5.6) > 0.9
