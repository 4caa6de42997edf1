"""Pins of the oracle's smoothed RT (Sec. 4.4): the chemistry starts from the
photon density and flux before injection and transport and receives their
change as constant rates (eqs. thchem_N_smooth, thchem_F_smooth,
smoothrate1, smoothrate2).

  - without photo-absorption the smoothed step leaves exactly the photon
    density and flux of injection and transport (the limit the section
    states), on a grid with sources, over several steps;
  - a cell with constant absorption settles on the steady state of
    eq. thchem_N_smooth, N = Ndot / D and F = Fdot / D, and stays between
    the exact solution and its start on the way there (backward Euler lags
    the exact exponential);
  - the two situations the section describes: a strong source in dense
    neutral gas needs far fewer substeps with smoothing, a strong source in
    ionised gas needs more;
  - the Stromgren test is unchanged by smoothing (the paper reports no
    discernible effect on its tests), and the photon budget still closes.
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


def one_cell(isothermal=True, sig=SIG):
    s = np.zeros((3, 3))
    s[0, 0] = sig
    eb = np.array([18.0 * EV, 0, 0])
    return oracle.OracleRT(n=(1, 1, 1), dx=1e20, bc=(0,) * 6, M=1, c_r=C_R, sigN=s, sigE=s.copy(), ebar=eb,
                           isothermal=isothermal, X=1.0, Y=0.0)


def test_no_absorption_gives_the_transport_result(oracle_mod):
    w = ri.stromgren_32(4)
    w.n = (10, 9, 8)
    w.bc = (ri.BC_OUTFLOW, ri.BC_REFLECT, ri.BC_PERIODIC, ri.BC_PERIODIC, ri.BC_REFLECT, ri.BC_OUTFLOW)
    o = oracle.OracleRT.for_workload(w)
    o.p.sigN[0][0] = o.p.sigN[0][1] = o.p.sigN[0][2] = 0.0
    rng = np.random.default_rng(5)
    st = ri.initial_state(w)
    st["N"] = rng.uniform(0.0, 1e-3, st["N"].shape)
    st["F"] = rng.uniform(-0.3, 0.3, st["F"].shape) * C_R * st["N"][:, None]
    ijk = np.array([[0, 0, 0], [5, 4, 3]], np.int32)
    ndot = o.source_rates(np.array([5e48, 1e48]))
    dt = o.courant_dt()
    sm = oracle.copy_state(st)
    for _ in range(4):
        o.inject(st, dt, ijk, ndot)
        o.transport(st, dt)
        assert o.step(sm, dt, ijk, ndot, smooth=True) == 0
        # the transport result, as the chemistry left it (N + sum h Ndot)
        Ns = np.max(np.abs(st["N"]))
        assert np.max(np.abs(sm["N"] - st["N"])) <= 1e-13 * Ns
        assert np.max(np.abs(sm["F"] - st["F"])) <= 1e-13 * C_R * Ns
        st["N"], st["F"] = sm["N"].copy(), sm["F"].copy()
        st["xHII"], st["T"] = sm["xHII"].copy(), sm["T"].copy()


@pytest.mark.parametrize("start", [3.0, 0.2])
def test_constant_absorption_settles_on_the_steady_state(oracle_mod, start):
    # x_HII stays at 1.2e-3 (photons far fewer than atoms), so D is constant
    nH, x = 1e-3, 1.2e-3
    D = C_R * SIG * (1 - x) * nH
    o = one_cell()
    Ndot = 1e-24 * D  # steady state 1e-24 photons / cm^3
    Fdot = np.array([0.4, -0.2, 0.1]) * C_R * Ndot
    Nss, Fss = Ndot / D, Fdot / D
    # long step: the steady state (eq. thchem_N_smooth with dN/dt = 0), with
    # D from the final x_HII (it drifts by 3e-5 of itself towards CIE)
    r = o.thermo_cell(200.0 / D, nH, [start * Nss], start * Fss, [x, 0, 0], 1e4, Nr=[Ndot], Fr=Fdot)
    assert r["flags"] == 0 and r["nacc"] > 5
    assert abs(r["x"][0] / x - 1) < 1e-4
    Df = C_R * SIG * (1 - r["x"][0]) * nH
    assert abs(r["N"][0] / (Ndot / Df) - 1) < 1e-7
    assert np.allclose(r["F"], Fdot / Df, rtol=1e-7, atol=0)
    # short step: exact solution N_ss + (N0 - N_ss) exp(-D t); the implicit
    # substeps decay more slowly than the exponential, never past N_ss
    dt = 1.5 / D
    r = o.thermo_cell(dt, nH, [start * Nss], start * Fss, [x, 0, 0], 1e4, Nr=[Ndot], Fr=Fdot)
    exact = Nss + (start - 1.0) * Nss * math.exp(-1.5)
    lo, hi = sorted((exact, start * Nss))
    assert lo <= r["N"][0] <= hi
    assert abs(r["N"][0] - exact) < 0.05 * abs(start - 1.0) * Nss
    for d in range(3):
        ex = Fss[d] + (start - 1.0) * Fss[d] * math.exp(-1.5)
        lo, hi = sorted((ex, start * Fss[d]))
        assert lo - 1e-12 * abs(ex) <= r["F"][d] <= hi + 1e-12 * abs(ex)


def test_zero_start_single_substep_closed_form(oracle_mod):
    # A cell without photons at the start of the step skips the photon
    # check; with one accepted substep of dt the photon update is
    # (0 + dt Ndot) / (1 + dt D), the plain result N' / (1 + dt D).
    nH, x = 1e-3, 1.2e-3
    D = C_R * SIG * (1 - x) * nH
    o = one_cell()
    dt = 0.05 / D
    Ndot = 1e-24 * D
    r = o.thermo_cell(dt, nH, [0.0], [0, 0, 0], [x, 0, 0], 1e4, Nr=[Ndot], Fr=[C_R * Ndot, 0, 0])
    assert r["nacc"] == 1 and r["natt"] == 1
    assert r["N"][0] == pytest.approx(dt * Ndot / (1 + dt * D), rel=1e-14)
    assert r["F"][0] == pytest.approx(C_R * dt * Ndot / (1 + dt * D), rel=1e-14)
    plain = o.thermo_cell(dt, nH, [dt * Ndot], [C_R * dt * Ndot, 0, 0], [x, 0, 0], 1e4)
    assert r["N"][0] == pytest.approx(plain["N"][0], rel=1e-14)


@pytest.mark.parametrize("isothermal", [True, False])
def test_dense_neutral_source_cell_needs_fewer_substeps(oracle_mod, isothermal):
    # Sec. 4.4: strong source, dense neutral gas, depletion time << dt.
    # Without smoothing the photons are burnt off in thousands of 10%
    # substeps; with them fed in gradually the cell settles quickly.
    o = one_cell(isothermal)
    dt = 0.8 * 3.086e18 / (3 * C_R)
    T0 = 1e4 if isothermal else 100.0
    for nH, frac in [(100.0, 0.01), (100.0, 0.1)]:
        Np = frac * nH
        plain = o.thermo_cell(dt, nH, [Np], [0, 0, 0], [1e-6, 0, 0], T0)
        sm = o.thermo_cell(dt, nH, [0.0], [0, 0, 0], [1e-6, 0, 0], T0, Nr=[Np / dt])
        assert plain["flags"] == 0 and sm["flags"] == 0
        assert sm["nacc"] * 10 < plain["nacc"], (sm["nacc"], plain["nacc"])
        # both ionise the same amount within the 10% scheme's accuracy
        assert abs(sm["x"][0] / plain["x"][0] - 1) < 0.05
        # smoothing leaves a reservoir of photons, plain depletes the cell
        assert sm["N"][0] > 1e3 * plain["N"][0]


def test_ionised_gas_with_strong_source_needs_more_substeps(oracle_mod):
    # Sec. 4.4: with long gas time scales the plain step hardly subcycles,
    # while the smoothed one must feed the photons in through many substeps
    o = one_cell()
    dt = 0.8 * 3.086e18 / (3 * C_R)
    nH = 1e-3
    Np = 10 * nH
    plain = o.thermo_cell(dt, nH, [Np], [0, 0, 0], [1.0, 0, 0], 1e4)
    sm = o.thermo_cell(dt, nH, [Np / 10], [0, 0, 0], [1.0, 0, 0], 1e4, Nr=[0.9 * Np / dt])
    assert plain["nacc"] <= 2
    assert sm["nacc"] > 5 * plain["nacc"]
    assert sm["N"][0] == pytest.approx(plain["N"][0], rel=1e-3)


def test_negative_rate_below_the_floor_stops_at_zero(oracle_mod):
    # Photons leaving a neutral cell: Ndot < 0 and strong absorption put the
    # steady state Ndot / D below zero.  Above N_floor the 10% check keeps N
    # positive; at or below it the update stops at zero instead of creeping
    # towards it in ever shorter substeps.
    nH, x = 1e-3, 1.2e-3
    D = C_R * SIG * (1 - x) * nH
    dt = 20.0 / D
    s = np.zeros((3, 3))
    s[0, 0] = SIG
    o = oracle.OracleRT(n=(1, 1, 1), dx=1e20, bc=(0,) * 6, M=1, c_r=C_R, sigN=s, sigE=s.copy(),
                        ebar=np.array([18.0 * EV, 0, 0]), isothermal=True, X=1.0, Y=0.0, N_floor=1e-20)
    N0 = 1e-16
    r = o.thermo_cell(dt, nH, [N0], [0.5 * C_R * N0, 0, 0], [x, 0, 0], 1e4, Nr=[-0.4 * N0 / dt],
                      Fr=[-0.2 * C_R * N0 / dt, 0, 0])
    assert r["flags"] == 0
    assert r["N"][0] == 0.0
    assert r["nacc"] < 200
    # the flux follows its own linear update, which has no sign constraint
    assert np.all(np.isfinite(r["F"]))


def test_stromgren_front_and_budget_unchanged_by_smoothing(oracle_mod):
    # N_floor 1e-16 (far below the 1e-4 cm^-3 of the ionised region): the
    # GLF leak ahead of the front is not worth 10% substeps, and without a
    # floor the smoothed update needs billions of them there
    w = ri.stromgren_32(60)
    w.n = (16, 16, 16)
    o = oracle.OracleRT.for_workload(w, N_floor=1e-16)
    ijk, nd = ri.workload_sources(w)
    ndot = o.source_rates(nd)
    dt = o.courant_dt(w.courant)
    res = {}
    for smooth in (False, True):
        st = ri.initial_state(w)
        tot = 0
        for _ in range(60):
            fl, nacc, _ = o.step(st, dt, ijk, ndot, want_counts=True, smooth=smooth)
            assert fl == 0
            tot += int(nacc.sum())
        res[smooth] = (st, tot)
    a, b = res[False][0], res[True][0]
    V = w.dx ** 3
    ra = (3 * 8 * a["xHII"].sum() * V / (4 * math.pi)) ** (1 / 3)
    rb = (3 * 8 * b["xHII"].sum() * V / (4 * math.pi)) ** (1 / 3)
    assert abs(ra - rb) < 0.25 * w.dx, (ra / w.dx, rb / w.dx)
    # fewer substeps with smoothing (2.5x here)
    assert res[True][1] < 0.6 * res[False][1], (res[True][1], res[False][1])
    # injected = in box + absorbed; ionisations match the absorbed photons
    # to the 10% level of the scheme (no outflow yet: the front is inside)
    injected = ndot.sum() * dt * 60
    absorbed = injected - b["N"].sum() * V
    ionised = (b["xHII"].sum() - ri.initial_state(w)["xHII"].sum()) * V * w.nH_mean
    assert abs(ionised / absorbed - 1) < 0.1


def test_selected_cells_equal_the_whole_grid_step(oracle_mod):
    # the sampled-cell step (transport of the listed cells, then their
    # smoothed chemistry) against the whole-grid smoothed step
    w = ri.lognormal_box(12, 6.6 * 12 / 128, 4, steps=1, seed=3)
    o = oracle.OracleRT.for_workload(w, N_floor=1e-12)
    st = ri.initial_state(w)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    ndot = o.source_rates(nd)
    dt = o.courant_dt()
    for _ in range(3):
        o.step(st, dt, ijk, ndot, smooth=True)
    pre = oracle.copy_state(st)
    inj = oracle.copy_state(st)
    o.inject(inj, dt, ijk, ndot)
    fl, nacc, natt = o.step(st, dt, ijk, ndot, want_counts=True, smooth=True)
    cells = np.arange(0, 12 ** 3, 7)
    r = o.step_cells(inj, dt, cells, N_pre=pre["N"])
    assert r["flags"] == fl
    N = st["N"].reshape(w.spectrum.M, -1)[:, cells].T
    assert np.array_equal(r["N"], N)
    assert np.array_equal(r["nacc"], nacc.ravel()[cells])
    assert np.array_equal(r["x"][:, 0], st["xHII"].ravel()[cells])
    F = st["F"].reshape(w.spectrum.M, 3, -1)[:, :, cells].transpose(2, 0, 1)
    assert np.array_equal(r["F"], F)
