"""Pins of the oracle's super-comoving RT variables (Sec. 5.4): the state
holds N~ = a^3 N, F~ = a^4 F (units with H_0 L = 1) and a^3 n_H on a grid of
comoving cell width; a step converts to physical variables, steps cells of
width a dx, and converts back.

  - the transport written in the new variables (light speed a c_r, step
    dt / a^2, comoving dx) gives the same result as the physical transport,
    the invariance the section states, for GLF and HLL;
  - a = 1 is the static step;
  - held fixed across a change of a, N~ and F~ dilute the physical N as
    a^-3 and F as a^-4 (photon counts per comoving cell do not change);
  - the Compton term of the chemistry works with the CMB temperature
    2.727 / a.
"""
import numpy as np
import pytest

import oracle
import rt_inputs as ri
from oracle import physics

C_R = ri.C_LIGHT / 100


def box(flux, c_r=C_R, dx=6.6 * ri.KPC / 32, sig=True, **kw):
    spec = ri.Spectrum(kind="bb", T_bb=1e5, edges_eV=ri.EDGES_2)
    sN, sE, eb, fr = physics.spectrum_attributes(spec)
    if not sig:
        sN, sE = np.zeros((3, 3)), np.zeros((3, 3))
    o = oracle.OracleRT(n=(11, 9, 7), dx=dx, bc=(0, 0, 1, 2, 1, 1), M=2, c_r=c_r, sigN=sN, sigE=sE, ebar=eb,
                        flux=flux, **kw)
    o.group_frac = fr[:2]
    return o


def random_state(rng, n=(11, 9, 7), M=2):
    nx, ny, nz = n
    N = 10 ** rng.uniform(-8, -3, (M, nz, ny, nx))
    d = rng.normal(size=(M, 3, nz, ny, nx))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    F = d * rng.uniform(0, 1, (M, 1, nz, ny, nx)) * C_R * N[:, None]
    shp = (nz, ny, nx)
    return {"N": N, "F": F, "nH": 1e-3 * np.exp(rng.normal(0, 1, shp)), "xHII": 10 ** rng.uniform(-4, 0, shp),
            "xHeII": np.zeros(shp), "xHeIII": np.zeros(shp), "T": 10 ** rng.uniform(2, 4.5, shp)}


@pytest.mark.parametrize("flux", [ri.FLUX_GLF, ri.FLUX_HLL])
@pytest.mark.parametrize("a", [0.3, 0.07])
def test_transport_in_the_new_variables_equals_the_physical_one(oracle_mod, flux, a):
    rng = np.random.default_rng(31)
    o = box(flux)
    st = random_state(rng)
    tl = {"N": st["N"] * a ** 3, "F": st["F"] * a ** 4}
    dt = o.courant_dt(0.8, a)
    # physical: cells of width a dx
    ophys = box(flux, dx=a * o.dx)
    phys = {"N": st["N"].copy(), "F": st["F"].copy()}
    ophys.transport(phys, dt)
    # super-comoving: c~ = a c_r, dt~ = dt / a^2, comoving dx
    otl = box(flux, c_r=a * C_R)
    otl.transport(tl, dt / a ** 2)
    assert np.allclose(tl["N"] / a ** 3, phys["N"], rtol=1e-12, atol=1e-14 * phys["N"].max())
    assert np.allclose(tl["F"] / a ** 4, phys["F"], rtol=1e-11, atol=1e-13 * np.abs(phys["F"]).max())


def test_a_one_is_the_static_step(oracle_mod):
    rng = np.random.default_rng(32)
    o = box(0)
    s1 = random_state(rng)
    s2 = oracle.copy_state(s1)
    ijk = np.array([[3, 4, 5]], np.int32)
    nd = o.source_rates(np.array([2e48]))
    dt = o.courant_dt()
    o.step(s1, dt, ijk, nd)
    o.step(s2, dt, ijk, nd, a=1.0)
    for k in s1:
        assert np.array_equal(s1[k], s2[k]), k


def test_fixed_comoving_radiation_dilutes_with_expansion(oracle_mod):
    # uniform radiation, no absorbers, periodic along x and y: the steps
    # leave N~ and F~ alone at every a, so physical N, F fall as a^-3, a^-4
    o = box(1, sig=False)
    o.p.bc[2] = o.p.bc[3] = o.p.bc[4] = o.p.bc[5] = 0
    shp = (7, 9, 11)
    st = {"N": np.full((2,) + shp, 1e-4), "F": np.zeros((2, 3) + shp), "nH": np.full(shp, 1e-3),
          "xHII": np.full(shp, 0.5), "xHeII": np.zeros(shp), "xHeIII": np.zeros(shp), "T": np.full(shp, 1e4)}
    # reduced flux F~ / (a c_r N~) = 0.2 at a = 0.25, falling as 1 / a after
    st["F"][:, 0] = 0.2 * 0.25 * C_R * 1e-4
    N0, F0 = st["N"].copy(), st["F"].copy()
    for a in (0.25, 0.5, 1.0):
        o.step(st, o.courant_dt(0.8, a), a=a)
        assert np.allclose(st["N"], N0, rtol=1e-13) and np.allclose(st["F"], F0, rtol=1e-13)
    # physical densities: N~ / a^3 and F~ / a^4
    assert np.allclose((st["N"] / 0.25 ** 3) / (st["N"] / 1.0 ** 3), 64.0)
    assert np.allclose((st["F"][:, 0] / 0.25 ** 4) / (st["F"][:, 0] / 1.0 ** 4), 256.0)


@pytest.mark.parametrize("a,T0", [(0.1, 5.0), (1.0, 100.0)])
def test_compton_term_uses_the_cmb_temperature_at_a(oracle_mod, a, T0):
    # fully ionised hydrogen so dilute (1e-10 cm^-3) that it neither
    # recombines nor cools otherwise within the step: Compton exchange drives
    # T towards the CMB temperature 2.727 / a (27.3 K for a = 0.1: the 5 K
    # gas heats; 2.7 K for a = 1: the 100 K gas cools), never past it
    s = np.zeros((3, 3))
    o = oracle.OracleRT(n=(1, 1, 1), dx=1e20, bc=(0,) * 6, M=1, c_r=C_R, sigN=s, sigE=s, ebar=np.zeros(3),
                        isothermal=False, X=1.0, Y=0.0)
    st = {"N": np.zeros((1, 1, 1, 1)), "F": np.zeros((1, 3, 1, 1, 1)), "nH": np.full((1, 1, 1), 1e-10 * a ** 3),
          "xHII": np.ones((1, 1, 1)), "xHeII": np.zeros((1, 1, 1)), "xHeIII": np.zeros((1, 1, 1)),
          "T": np.full((1, 1, 1), T0)}
    o.step(st, 3e16, a=a)
    T1 = float(st["T"][0, 0, 0])
    Tcmb = 2.727 / a
    assert st["xHII"][0, 0, 0] > 1 - 1e-4
    assert min(T0, Tcmb) < T1 < max(T0, Tcmb), (T1, Tcmb)
    assert abs(T1 - T0) > 1e-4 * abs(Tcmb - T0)
