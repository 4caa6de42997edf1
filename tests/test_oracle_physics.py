"""Pins of the oracle's host physics and rate coefficients against what the
paper prints, closed forms, physical scaling laws and brute force."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import physics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
KPC = 3.0856775814913673e21
MYR = 3.15576e13
C = 2.99792458e10


# ---------------------------------------------------------------- rates ----
def test_alpha_B_printed_value(oracle_mod):
    # Sec. 4.2 quotes alpha_B ~ 2.6e-13 at 1e4 K
    v, _ = oracle.rate("alphaB_HII", 1e4)
    assert abs(v / GOLD["alpha_B_1e4K"]["value"] - 1) < 0.01


def test_iliev1_stromgren_numbers(oracle_mod):
    # Sec. 6, test 1: r_S = 5.4 kpc and t_rec = 122.4 Myr for n_H = 1e-3, Ndot = 5e48
    aB, _ = oracle.rate("alphaB_HII", 1e4)
    rs = physics.stromgren_radius(5e48, 1e-3, aB) / KPC
    tr = physics.t_rec(1e-3, aB) / MYR
    assert abs(rs - GOLD["iliev1_r_S_kpc"]["value"]) < 0.05
    assert abs(tr / GOLD["iliev1_t_rec_Myr"]["value"] - 1) < 0.003


def test_c_red_table_rows():
    # Table c_red, computed with the paper's alpha_B = 2.6e-13 and the full light speed
    for row in GOLD["c_red_table"]["rows"]:
        rs = physics.stromgren_radius(row["Ndot"], row["nH"], 2.6e-13)
        tr = physics.t_rec(row["nH"], 2.6e-13)
        tc = rs / C
        q = tc / tr
        # printed to one or two significant figures
        assert abs(math.log10(rs / KPC / row["r_S_kpc"])) < 0.12, row
        assert abs(math.log10(tr / MYR / row["t_rec_Myr"])) < 0.12, row
        assert abs(math.log10(tc / MYR / row["t_cross_Myr"])) < 0.12, row
        assert abs(math.log10(q / row["q"])) < 0.12, row


def test_courant_dt_iliev(oracle_mod):
    # Sec. 6 intro: 6.6 kpc / 128 cells, f_c = 1e-2 -> Delta t ~ 4,500 yr
    dt = oracle.lib().or_courant_dt(6.6 * KPC / 128, C / 100, 0.8)
    assert abs(dt / 3.15576e7 / GOLD["iliev1_dt_yr_fine"]["value"] - 1) < 0.01


RATES = [n for n in oracle.RATE_NAMES]


@pytest.mark.parametrize("name", RATES)
def test_rate_derivative_matches_finite_difference(oracle_mod, name):
    for T in (50.0, 3e3, 1e4, 7e4, 3e5, 2e6):
        v, d = oracle.rate(name, T)
        h = T * 1e-6
        vp, _ = oracle.rate(name, T + h)
        vm, _ = oracle.rate(name, T - h)
        fd = (vp - vm) / (2 * h)
        scale = max(abs(d), abs(v) / T, 1e-300)
        assert abs(fd - d) <= 1e-5 * scale, (name, T, d, fd)


def test_rates_positive(oracle_mod):
    for name in RATES:
        if name == "varpi":
            continue
        for T in (10.0, 1e3, 1e4, 1e5, 1e7):
            v, _ = oracle.rate(name, T)
            assert v >= 0.0 and np.isfinite(v), (name, T)


def test_cen_family_shares_form(oracle_mod):
    # beta_j and zeta_j share one functional form (App. E.1, E.3): constant ratio
    pairs = [("zeta_HI", "beta_HI", 1.27e-21 / 5.85e-11), ("zeta_HeI", "beta_HeI", 9.38e-22 / 2.38e-11),
             ("zeta_HeII", "beta_HeII", 4.95e-22 / 5.68e-12)]
    for z, b, ratio in pairs:
        for T in (3e3, 3e4, 3e5, 3e6):
            assert abs(oracle.rate(z, T)[0] / oracle.rate(b, T)[0] / ratio - 1) < 1e-12


def test_hydrogenic_scaling_of_HeIII(oracle_mod):
    # HeIII recombination is hydrogenic with Z = 2: alpha(Z, T) = Z alpha(1, T T_HI/T_HeII)
    # where T_HI/T_HeII = 315614/1263030 (~1/Z^2); cooling scales as Z^3 T/T'.
    s = 315614.0 / 1263030.0
    for T in (1e3, 1e4, 1e5, 1e6):
        for case in ("A", "B"):
            a3 = oracle.rate(f"alpha{case}_HeIII", T)[0]
            a1 = oracle.rate(f"alpha{case}_HII", T * s)[0]
            assert abs(a3 / (2.0 * a1) - 1) < 1e-12
            e3 = oracle.rate(f"eta{case}_HeIII", T)[0]
            e1 = oracle.rate(f"eta{case}_HII", T * s)[0]
            assert abs(e3 / (8.0 * e1 / s) - 1) < 1e-12


def test_eta_HeII_is_kT_alpha(oracle_mod):
    kB = 1.380649e-16
    for T in (1e3, 1e4, 1e5):
        for case in ("A", "B"):
            assert abs(oracle.rate(f"eta{case}_HeII", T)[0] / (kB * T * oracle.rate(f"alpha{case}_HeII", T)[0]) - 1) < 1e-14


def test_case_A_exceeds_case_B_and_literature(oracle_mod):
    # case A counts ground-state recombinations as well: alpha_A > alpha_B.
    # Osterbrock & Ferland (2006) at 1e4 K: alpha_A = 4.18e-13, alpha_B = 2.59e-13
    for T in (1e3, 1e4, 1e5):
        assert oracle.rate("alphaA_HII", T)[0] > oracle.rate("alphaB_HII", T)[0]
    assert abs(oracle.rate("alphaA_HII", 1e4)[0] / 4.18e-13 - 1) < 0.05
    assert abs(oracle.rate("alphaB_HII", 1e4)[0] / 2.59e-13 - 1) < 0.01


def test_compton_vanishes_at_cmb_temperature(oracle_mod):
    for a in (1.0, 0.5, 0.1):
        v, _ = oracle.rate("varpi", 2.727 / a, a_exp=a)
        assert v == 0.0
        assert oracle.rate("varpi", 2.0 * 2.727 / a, a_exp=a)[0] > 0
        assert oracle.rate("varpi", 0.5 * 2.727 / a, a_exp=a)[0] < 0


# ------------------------------------------------------- cross sections ----
def test_verner_threshold_values():
    # Iliev test 1 uses sigma_HI = 6.3e-18 cm^2 at 13.6 eV
    s = float(physics.sigma_verner(13.6, 0))
    assert abs(s / GOLD["iliev1_sigma_HI"]["value"] - 1) < 0.01
    # hydrogenic HeII: sigma(Z) at threshold = sigma_HI / Z^2
    assert abs(float(physics.sigma_verner(54.42, 2)) / (s / 4.0) - 1) < 0.01
    # HeI threshold ~7.4e-18 cm^2 (Verner et al. 1996) with eps0 = 13.61 eV
    assert abs(float(physics.sigma_verner(24.59, 1)) / 7.43e-18 - 1) < 0.01
    # zero below threshold
    for j, e in enumerate(physics.EPS_ION_EV):
        assert float(physics.sigma_verner(e * 0.999, j)) == 0.0


def test_group_attributes_against_brute_force():
    edges = (13.6, 24.59, 54.42, np.inf)
    sigN, sigE, ebar, frac = physics.group_attributes(1e5, edges)
    assert abs(frac.sum() - 1) < 1e-12
    # brute force: trapezoid on a dense logarithmic grid per group
    kT = physics.KB_EV * 1e5
    for i in range(3):
        lo, hi = edges[i], min(edges[i + 1], 13.6 * 400)
        ee = np.geomspace(lo, hi, 400001)
        JJ = ee ** 3 / np.expm1(ee / kT)
        n_i = np.trapezoid(JJ / ee, ee)
        e_i = np.trapezoid(JJ, ee)
        assert abs(ebar[i] / physics.EV / (e_i / n_i) - 1) < 1e-6
        for j in range(3):
            s = physics.sigma_verner(ee, j)
            bn = np.trapezoid(s * JJ / ee, ee) / n_i
            be = np.trapezoid(s * JJ, ee) / e_i
            assert abs(sigN[i, j] - bn) <= 1e-5 * sigN[i].max()
            assert abs(sigE[i, j] - be) <= 1e-5 * sigE[i].max()
    # mean energy within each group lies inside the group
    for i in range(3):
        assert edges[i] < ebar[i] / physics.EV < edges[i + 1]


def test_grey_group_is_photon_weighted_mean_of_three():
    s3, e3, eb3, f3 = physics.group_attributes(1e5, (13.6, 24.59, 54.42, np.inf))
    s1, e1, eb1, f1 = physics.group_attributes(1e5, (13.6, np.inf))
    for j in range(3):
        assert abs(s1[0, j] - np.dot(f3, s3[:, j])) <= 1e-10 * s1[0, j]
    assert abs(eb1[0] - np.dot(f3, eb3)) <= 1e-10 * eb1[0]


# ---------------------------------------------------------- closure -------
def test_eddington_closure_invariants(oracle_mod):
    rng = np.random.default_rng(3)
    c = 3e8
    # chi(0) = 1/3 -> D = I/3 ; f = 1 -> D = n n
    D = oracle.eddington(1.0, np.zeros(3), c)
    assert np.allclose(D, np.eye(3) / 3, rtol=0, atol=1e-16)
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    D = oracle.eddington(2.0, 2.0 * c * n, c)
    assert np.allclose(D, np.outer(n, n), rtol=0, atol=1e-15)
    for _ in range(200):
        N = rng.uniform(0.1, 10)
        F = rng.normal(size=3)
        F *= rng.uniform(0, 1.2) * c * N / np.linalg.norm(F)
        D = oracle.eddington(N, F, c)
        assert abs(np.trace(D) - 1) < 1e-14
        assert np.allclose(D, D.T, atol=1e-16)
        f = min(np.linalg.norm(F) / (c * N), 1.0)
        chi = (3 + 4 * f * f) / (5 + 2 * math.sqrt(4 - 3 * f * f))
        nn = F / np.linalg.norm(F)
        # the Eddington factor is the eigenvalue along the flux direction
        assert abs(nn @ D @ nn - chi) < 1e-14
        assert 1 / 3 - 1e-15 <= chi <= 1 + 1e-15


# ---------------------------------------------------------- HLL table -----
def test_hll_table_closed_forms():
    tab = physics.hll_table()
    nf, nth = tab.shape[:2]
    fs = np.linspace(0, 1, nf)
    ths = np.linspace(0, np.pi, nth)
    # f = 0: wave speeds +-1/sqrt(3) for any angle
    assert np.allclose(tab[0, :, 0], -1 / math.sqrt(3), atol=1e-14)
    assert np.allclose(tab[0, :, 1], 1 / math.sqrt(3), atol=1e-14)
    # theta = 0: the 1D M1 system U = (N, F), G = (F, chi N) with Jacobian
    # [[0, 1], [chi - f chi', chi']] -> lambda = (chi' +- sqrt(chi'^2 + 4 (chi - f chi')))/2
    for i in range(nf - 1):
        f = fs[i]
        r = math.sqrt(4 - 3 * f * f)
        chi = (3 + 4 * f * f) / (5 + 2 * r)
        dchi = (8 * f * (5 + 2 * r) + 6 * f * (3 + 4 * f * f) / r) / (5 + 2 * r) ** 2
        disc = math.sqrt(dchi * dchi + 4 * (chi - f * dchi))
        lo, hi = 0.5 * (dchi - disc), 0.5 * (dchi + disc)
        assert abs(tab[i, 0, 1] - hi) < 1e-12, (f, tab[i, 0], lo, hi)
        # the smaller longitudinal root may sit above the transverse speeds
        assert tab[i, 0, 0] <= lo + 1e-12
    # mirror symmetry theta -> pi - theta swaps and negates the extremes
    assert np.allclose(tab[:, ::-1, 0], -tab[:, :, 1], atol=1e-12)
    # bounded by the light speed, ordered
    assert np.all(np.abs(tab) <= 1 + 1e-12)
    assert np.all(tab[..., 0] <= tab[..., 1] + 1e-15)
    # f -> 1 limit: all eigenvalues tend to cos(theta) like sqrt(1 - f)
    J = physics.m1_jacobian(1 - 1e-8, ths)
    ev = np.linalg.eigvals(J).real
    assert np.max(np.abs(ev - np.cos(ths)[:, None])) < 3e-4
    assert np.allclose(tab[-1, :, 0], np.cos(ths)) and np.allclose(tab[-1, :, 1], np.cos(ths))


def test_jacobian_complex_step_matches_finite_difference():
    rng = np.random.default_rng(1)
    for _ in range(20):
        f, th = rng.uniform(0.05, 0.95), rng.uniform(0, np.pi)
        J = physics.m1_jacobian(f, th)
        U = np.array([1.0, f * math.cos(th), f * math.sin(th), 0.0])
        h = 1e-6
        for k in range(4):
            Up = U.astype(complex).copy(); Up[k] += h
            Um = U.astype(complex).copy(); Um[k] -= h
            fd = (physics._flux_x_complex(Up).real - physics._flux_x_complex(Um).real) / (2 * h)
            assert np.allclose(fd, J[:, k], atol=1e-8)
