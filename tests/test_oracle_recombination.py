"""Pins of the oracle without the on-the-spot approximation (Sec. 3.3.2): case
A recombination, case A recombination cooling, and the photons of
recombinations straight to the ground state added to the group b^rec of the
recombining species (eq. cool_N_cr).

  - optically thin (no absorption): the collisional ionisation equilibrium
    is the case A one, and the photon density grows by exactly
    (alpha_A - alpha_B) n_HII n_e dt per step once x is there;
  - optically thick: the emitted photons are absorbed in the cell, and the
    equilibrium is the case B one, i.e. what the OTSA assumes (Sec. 3.3.2),
    with N = C / D;
  - each species' photons land in the group holding its threshold;
  - the Stromgren test without OTSA stays within a few per cent of the OTSA
    front (inside the ionised region the emitted photons are re-absorbed).
"""
import math

import numpy as np
import pytest

import oracle
import rt_inputs as ri

C = 2.99792458e10
C_R = C / 100
EV = 1.602176634e-12
SIG = 6.3e-18


def cell(M=1, sig=0.0, Y=0.0, brec=(0, 0, 0), otsa=False, isothermal=True):
    s = np.zeros((3, 3))
    s[:M, 0] = sig
    eb = np.zeros(3)
    eb[:M] = 18.0 * EV
    return oracle.OracleRT(n=(1, 1, 1), dx=1e20, bc=(0,) * 6, M=M, c_r=C_R, sigN=s, sigE=s.copy(), ebar=eb,
                           isothermal=isothermal, X=1.0 - Y, Y=Y, otsa=otsa, brec=brec)


def relax(o, dt, nH, N, F, x, T, n):
    for _ in range(n):
        r = o.thermo_cell(dt, nH, N, F, x, T)
        assert r["flags"] == 0
        N, F, x = r["N"], r["F"], r["x"]
    return r


@pytest.mark.parametrize("T", [2e4, 5e4])
def test_optically_thin_equilibrium_is_case_A(oracle_mod, T):
    o = cell(sig=0.0)
    b = oracle.rate("beta_HI", T)[0]
    aA = oracle.rate("alphaA_HII", T)[0]
    aB = oracle.rate("alphaB_HII", T)[0]
    r = relax(o, 3e13, 1.0, [0.0], [0, 0, 0], [0.5, 0, 0], T, 400)
    x = r["x"][0]
    assert abs(x / (b / (aA + b)) - 1) < 1e-6, (x, b / (aA + b))
    # one more step at equilibrium: no absorption, so the recombination
    # photons simply add up, (alpha_A - alpha_B) n_HII n_e dt
    dt = 3e13
    r2 = o.thermo_cell(dt, 1.0, r["N"], r["F"], r["x"], T)
    dN = r2["N"][0] - r["N"][0]
    assert abs(dN / ((aA - aB) * x * x * dt) - 1) < 1e-6
    # the flux gets none of it (isotropic emission)
    assert np.array_equal(r2["F"], r["F"])


@pytest.mark.parametrize("T", [2e4, 5e4])
def test_optically_thick_equilibrium_is_case_B(oracle_mod, T):
    o = cell(sig=SIG)
    b = oracle.rate("beta_HI", T)[0]
    aA = oracle.rate("alphaA_HII", T)[0]
    aB = oracle.rate("alphaB_HII", T)[0]
    r = relax(o, 3e13, 1.0, [0.0], [0, 0, 0], [0.5, 0, 0], T, 400)
    x = r["x"][0]
    # every emitted photon ionises an atom of the same cell: net
    # recombination at alpha_B, the equilibrium the OTSA assumes
    assert abs(x / (b / (aB + b)) - 1) < 1e-6, (x, b / (aB + b))
    Crec = (aA - aB) * x * x
    D = C_R * SIG * (1 - x)
    assert abs(r["N"][0] * D / Crec - 1) < 1e-6
    # the OTSA run reaches the same state without photons
    ro = relax(cell(sig=SIG, otsa=True), 3e13, 1.0, [0.0], [0, 0, 0], [0.5, 0, 0], T, 400)
    assert abs(ro["x"][0] / x - 1) < 1e-6 and ro["N"][0] == 0.0


def test_each_species_emits_into_its_group(oracle_mod):
    # H + He at 6e4 K in case A collisional equilibrium, no absorption; the
    # three groups of EDGES_3 receive the HII, HeII and HeIII photons
    T, nH, Y = 6e4, 1.0, 0.24
    groups = ri.recombination_groups(ri.Spectrum(kind="bb", edges_eV=ri.EDGES_3))
    assert groups == (0, 1, 2)
    o = cell(M=3, Y=Y, brec=groups)
    r = relax(o, 3e13, nH, [0.0] * 3, [0.0] * 9, [0.5, 0.3, 0.3], T, 600)
    x, y2, y3 = r["x"]
    nHe = nH * Y / (4 * (1 - Y))
    ne = x * nH + (y2 + 2 * y3) * nHe
    dt = 3e13
    r2 = o.thermo_cell(dt, nH, r["N"], r["F"], r["x"], T)
    assert np.allclose(r2["x"], r["x"], rtol=1e-7, atol=0)  # at equilibrium
    em = [(oracle.rate("alphaA_" + s, T)[0] - oracle.rate("alphaB_" + s, T)[0]) * n * ne
          for s, n in (("HII", x * nH), ("HeII", y2 * nHe), ("HeIII", y3 * nHe))]
    assert min(em) > 0
    for g in range(3):
        assert abs((r2["N"][g] - r["N"][g]) / (em[g] * dt) - 1) < 1e-6, g
    # one group from 13.6 eV up: all three into it
    g1 = ri.recombination_groups(ri.Spectrum(kind="bb", edges_eV=ri.EDGES_1))
    assert g1 == (0, 0, 0)
    o1 = cell(M=1, Y=Y, brec=g1)
    r1 = o1.thermo_cell(dt, nH, [0.0], [0.0] * 3, r["x"], T)
    assert abs(r1["N"][0] / (sum(em) * dt) - 1) < 1e-6


def test_otsa_ignores_the_group_map_and_emits_nothing(oracle_mod):
    a = cell(sig=SIG, otsa=True, brec=(0, 0, 0)).thermo_cell(3e13, 1.0, [1e-8], [0, 0, 0], [0.3, 0, 0], 3e4)
    b = cell(sig=SIG, otsa=True, brec=(-1, -1, -1)).thermo_cell(3e13, 1.0, [1e-8], [0, 0, 0], [0.3, 0, 0], 3e4)
    assert all(np.array_equal(np.asarray(a[k]), np.asarray(b[k])) for k in a)
    # and without OTSA, a map pointing nowhere emits nothing: case A alone
    c = cell(sig=0.0, otsa=False, brec=(-1, -1, -1)).thermo_cell(3e13, 1.0, [0.0], [0, 0, 0], [0.3, 0, 0], 3e4)
    assert c["N"][0] == 0.0


def test_stromgren_front_without_otsa(oracle_mod):
    w = ri.stromgren_32(100)
    w.n = (20, 20, 20)
    ijk, nd = ri.workload_sources(w)
    radii = {}
    for otsa in (True, False):
        w.otsa = otsa
        o = oracle.OracleRT.for_workload(w)
        st = ri.initial_state(w)
        ndot = o.source_rates(nd)
        dt = o.courant_dt(w.courant)
        for _ in range(100):
            assert o.step(st, dt, ijk, ndot) == 0
        radii[otsa] = (3 * 8 * st["xHII"].sum() * w.dx ** 3 / (4 * math.pi)) ** (1 / 3)
        if not otsa:
            assert st["N"].min() >= 0.0
    # at 1.8 Myr << t_rec hardly any atom has recombined yet: the fronts
    # agree closely, and the case A one is not ahead
    assert radii[False] <= radii[True] * (1 + 1e-9)
    assert abs(radii[False] / radii[True] - 1) < 0.02, radii
