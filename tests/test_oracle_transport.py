"""Pins of the oracle's transport step (Sec. 3.2): conservation, exact
special cases (axis beams under HLL are 1D upwind advection), symmetry,
realisability, and a brute-force face-by-face transcription on tiny grids."""
import math

import numpy as np
import pytest

import oracle
from oracle import physics

C_R = 2.99792458e8
DX = 1e20
ZERO3 = np.zeros((3, 3))


def make(n, bc, flux=0, hll=None, M=1):
    return oracle.OracleRT(n=n, dx=DX, bc=bc, M=M, c_r=C_R, sigN=ZERO3, sigE=ZERO3,
                           ebar=np.zeros(3), flux=flux, hll=hll)


def random_state(n, M, rng, fmax=1.0):
    nx, ny, nz = n
    N = rng.uniform(0.1, 1.0, (M, nz, ny, nx))
    d = rng.normal(size=(M, 3, nz, ny, nx))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = rng.uniform(0, fmax, (M, 1, nz, ny, nx))
    F = d * f * C_R * N[:, None]
    z = np.zeros((nz, ny, nx))
    return {"N": N, "F": np.ascontiguousarray(F), "xHII": z + 1, "xHeII": z.copy(),
            "xHeIII": z.copy(), "T": z + 1e4, "nH": z + 1e-3}


@pytest.mark.parametrize("flux", [0, 1])
def test_periodic_free_streaming_conserves_photons_and_flux(oracle_mod, flux):
    rng = np.random.default_rng(0)
    n = (6, 5, 4)
    o = make(n, (0,) * 6, flux=flux, M=2)
    st = random_state(n, 2, rng)
    dt = o.courant_dt()
    N0 = st["N"].sum(axis=(1, 2, 3))
    F0 = st["F"].sum(axis=(2, 3, 4))
    for _ in range(20):
        o.transport(st, dt)
    assert np.allclose(st["N"].sum(axis=(1, 2, 3)), N0, rtol=1e-13, atol=0)
    Fs = st["F"].sum(axis=(2, 3, 4))
    assert np.all(np.abs(Fs - F0) <= 1e-12 * C_R * N0[:, None])


def test_closed_reflecting_box_conserves_photons(oracle_mod):
    rng = np.random.default_rng(1)
    n = (5, 4, 3)
    o = make(n, (2,) * 6)
    st = random_state(n, 1, rng)
    dt = o.courant_dt()
    N0 = st["N"].sum()
    for _ in range(10):
        o.transport(st, dt)
    assert abs(st["N"].sum() / N0 - 1) < 1e-13


@pytest.mark.parametrize("flux", [0, 1])
def test_uniform_state_stays_uniform(oracle_mod, flux):
    n = (4, 4, 4)
    o = make(n, (0,) * 6, flux=flux)
    z = np.zeros((1,) + n)
    st = {"N": z + 0.3, "F": np.ascontiguousarray(np.stack([z + 0.2 * C_R * 0.3, z - 0.1 * C_R * 0.3,
                                                           z + 0.05 * C_R * 0.3], axis=1))}
    N0, F0 = st["N"].copy(), st["F"].copy()
    o.transport(st, o.courant_dt())
    assert np.allclose(st["N"], N0, rtol=1e-15, atol=0)
    assert np.allclose(st["F"], F0, rtol=1e-14, atol=0)


def test_hll_axis_beam_is_1d_upwind_advection(oracle_mod):
    # Sec. 3.2: with HLL an axis-aligned beam is retained perfectly.  A beam
    # (f = 1 along +x) into empty space is exact first-order upwind advection
    # at Courant number nu = c dt/dx.
    n = (24, 3, 2)
    o = make(n, (1, 1, 0, 0, 0, 0), flux=1, hll=oracle.hll_table())
    dt = o.courant_dt()
    nu = C_R * dt / DX
    prof = np.zeros(n[0])
    prof[:4] = [1.0, 0.8, 0.5, 0.2]
    N = np.zeros((1, n[2], n[1], n[0])) + prof
    F = np.zeros((1, 3, n[2], n[1], n[0]))
    F[0, 0] = C_R * N[0]
    st = {"N": N, "F": F}
    ref = prof.copy()
    for _ in range(30):
        o.transport(st, dt)
        new = ref.copy()
        new[1:] = ref[1:] - nu * (ref[1:] - ref[:-1])
        new[0] = ref[0] - nu * (ref[0] - ref[0])  # outflow ghost copies cell 0: no net change
        ref = new
    assert np.allclose(st["N"][0], ref[None, None, :], rtol=1e-12, atol=1e-15)
    assert np.allclose(st["F"][0, 0], C_R * ref[None, None, :], rtol=1e-12, atol=1e-15 * C_R)
    assert np.all(np.abs(st["F"][0, 1:]) < 1e-12 * C_R)


def test_glf_equals_hll_with_light_speed_eigenvalues(oracle_mod):
    # eq. (glf) is HLL with lambda- = -c, lambda+ = +c
    tab = np.zeros((101, 101, 2))
    tab[..., 0] = -1.0
    tab[..., 1] = 1.0
    rng = np.random.default_rng(2)
    o_glf = make((3, 3, 3), (0,) * 6, flux=0)
    o_hll = make((3, 3, 3), (0,) * 6, flux=1, hll=tab)
    for _ in range(100):
        UL = np.r_[rng.uniform(0.1, 1), rng.normal(size=3) * 0.4 * C_R]
        UR = np.r_[rng.uniform(0.1, 1), rng.normal(size=3) * 0.4 * C_R]
        for d in range(3):
            a = o_glf.face_flux(d, UL, UR)
            b = o_hll.face_flux(d, UL, UR)
            assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * C_R)


def test_glf_point_source_keeps_cubic_symmetry(oracle_mod):
    n = (9, 9, 9)
    o = make(n, (1,) * 6)
    st = {"N": np.zeros((1, 9, 9, 9)), "F": np.zeros((1, 3, 9, 9, 9))}
    dt = o.courant_dt()
    for _ in range(6):
        o.inject(st, dt, np.array([[4, 4, 4]], np.int32), np.array([[1e50]]))
        o.transport(st, dt)
    N = st["N"][0]
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0)]:
        assert np.allclose(N, N.transpose(perm), rtol=1e-12, atol=0)
    assert np.allclose(N, N[::-1, ::-1, ::-1], rtol=1e-12, atol=0)
    # F points outward: Fx antisymmetric in x
    assert np.allclose(st["F"][0, 0], -st["F"][0, 0][:, :, ::-1], rtol=1e-12, atol=1e-30)


def test_glf_realisability(oracle_mod):
    # GLF at 3 c dt / dx <= 1 keeps N >= 0 and f <= 1
    rng = np.random.default_rng(4)
    n = (6, 6, 6)
    o = make(n, (0,) * 6)
    st = random_state(n, 1, rng, fmax=1.0)
    a = rng.uniform(0, 1, st["N"].shape) ** 6  # many near-empty cells
    st["N"] *= a
    st["F"] *= (a * rng.uniform(0, 1, a.shape))[:, None]
    for _ in range(10):
        o.transport(st, o.courant_dt())
        N = st["N"][0]
        Fn = np.linalg.norm(st["F"][0], axis=0)
        assert N.min() >= 0
        assert np.all(Fn <= C_R * N * (1 + 1e-12) + 1e-300)


def _brute_transport(n, bc, N, F, dt, c):
    """Face-centred brute force GLF: loop over every interface once, build its
    flux from the two states, then scatter it to both neighbours."""
    nx, ny, nz = n
    U = np.concatenate([N[:, None], F], axis=1)[0]  # (4, nz, ny, nx)
    out = U.copy()

    def G(u, d):
        Nn, Fv = u[0], u[1:]
        Fn = np.linalg.norm(Fv)
        f = min(Fn / (c * Nn), 1.0) if Nn > 0 else 0.0
        chi = (3 + 4 * f * f) / (5 + 2 * math.sqrt(4 - 3 * f * f))
        nv = Fv / Fn if Fn > 0 else np.zeros(3)
        P = Nn * ((1 - chi) / 2 * np.eye(3) + (3 * chi - 1) / 2 * np.outer(nv, nv))
        return np.r_[Fv[d], c * c * P[d]]

    dims = (nx, ny, nz)
    for d in range(3):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    idx = [x, y, z]
                    # interface on the + side of this cell
                    j = idx[d] + 1
                    right = list(idx)
                    uL = U[:, z, y, x].copy()
                    if j < dims[d]:
                        right[d] = j
                        uR = U[:, right[2], right[1], right[0]].copy()
                        own_right = True
                    else:
                        kind = bc[2 * d + 1]
                        if kind == 0:
                            right[d] = 0
                            uR = U[:, right[2], right[1], right[0]].copy()
                            own_right = True
                        else:
                            uR = uL.copy()
                            if kind == 2:
                                uR[1 + d] *= -1
                            own_right = False
                    phi = 0.5 * (G(uL, d) + G(uR, d)) - 0.5 * c * (uR - uL)
                    out[:, z, y, x] -= dt / DX * phi
                    if own_right:
                        out[:, right[2], right[1], right[0]] += dt / DX * phi
                    # interface on the - side of a non-periodic low boundary
                    if idx[d] == 0 and bc[2 * d] != 0:
                        uG = uL.copy()
                        if bc[2 * d] == 2:
                            uG[1 + d] *= -1
                        phi = 0.5 * (G(uG, d) + G(uL, d)) - 0.5 * c * (uL - uG)
                        out[:, z, y, x] += dt / DX * phi
    return out[0][None], out[1:][None]


@pytest.mark.parametrize("bc", [(0,) * 6, (2, 1, 0, 0, 1, 1), (1, 2, 2, 1, 0, 0)])
def test_brute_force_tiny_grids(oracle_mod, bc):
    rng = np.random.default_rng(5)
    for n in [(2, 2, 2), (3, 2, 4), (4, 3, 3)]:
        if any(n[d] == 1 for d in range(3)):
            continue
        o = make(n, bc)
        st = random_state(n, 1, rng)
        dt = o.courant_dt()
        Nb, Fb = _brute_transport(n, bc, st["N"], st["F"], dt, C_R)
        o.transport(st, dt)
        assert np.allclose(st["N"], Nb, rtol=1e-12, atol=0)
        assert np.allclose(st["F"], Fb, rtol=1e-11, atol=1e-12 * C_R)


def test_hll_eigenvalues_interpolate_the_table(oracle_mod):
    # The HLL wave speeds come from the eigenvalue table of Sec. 3.2, read
    # bilinearly in (f, theta) on uniform nodes, theta the angle between F
    # and the +d axis.  A table of the form a + b f + e theta + g f theta is
    # reproduced exactly at any state; a random table gives back its node
    # values at the nodes and the mean of the four neighbours midway.
    nf, nth = 11, 13
    fs = np.linspace(0.0, 1.0, nf)
    ths = np.linspace(0.0, np.pi, nth)
    tab = np.empty((nf, nth, 2))
    tab[..., 0] = -(0.2 + 0.5 * fs[:, None] + 0.1 * ths[None, :] + 0.03 * fs[:, None] * ths[None, :])
    tab[..., 1] = 0.3 + 0.4 * fs[:, None] - 0.05 * ths[None, :]
    o = make((3, 3, 3), (0,) * 6, flux=1, hll=tab)
    rng = np.random.default_rng(8)
    for _ in range(300):
        N = rng.uniform(0.1, 2.0)
        f = rng.uniform(0.0, 1.0)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d = int(rng.integers(0, 3))
        lo, hi = o.hll_eig(d, np.r_[N, f * C_R * N * u])
        th = np.arccos(u[d])
        assert lo == pytest.approx(-(0.2 + 0.5 * f + 0.1 * th + 0.03 * f * th), rel=1e-12, abs=1e-14)
        assert hi == pytest.approx(0.3 + 0.4 * f - 0.05 * th, rel=1e-12, abs=1e-14)
    # f above 1 reads the f = 1 row; an empty cell with flux is a beam (f = 1)
    lo, hi = o.hll_eig(0, [1.0, 3.0 * C_R, 0.0, 0.0])
    assert (lo, hi) == pytest.approx((tab[-1, 0, 0], tab[-1, 0, 1]), rel=1e-12)
    lo, hi = o.hll_eig(1, [0.0, 0.0, -2.0, 0.0])
    assert (lo, hi) == pytest.approx((tab[-1, -1, 0], tab[-1, -1, 1]), rel=1e-12)
    # an empty cell without flux: f = 0, theta = 0
    assert o.hll_eig(2, [0.0, 0.0, 0.0, 0.0]) == pytest.approx((tab[0, 0, 0], tab[0, 0, 1]), rel=1e-12)
    tab2 = rng.uniform(-1.0, 1.0, (nf, nth, 2))
    o2 = make((3, 3, 3), (0,) * 6, flux=1, hll=tab2)

    def state(f, th, d):
        # unit vector at angle th from axis d, in the plane of axes d and d+1
        u = np.zeros(3)
        u[d] = np.cos(th)
        u[(d + 1) % 3] = np.sin(th)
        return np.r_[1.0, f * C_R * u]
    for i in (1, 4, nf - 1):  # at f = 0 there is no flux and theta reads 0
        for k in (0, 6, nth - 1):
            d = (i + k) % 3
            assert o2.hll_eig(d, state(fs[i], ths[k], d)) == pytest.approx(tuple(tab2[i, k]), rel=1e-9, abs=1e-9)
    for i in (0, 5, nf - 2):
        for k in (0, 7, nth - 2):
            d = (i + 2 * k) % 3
            mid = tab2[i:i + 2, k:k + 2].mean(axis=(0, 1))
            got = o2.hll_eig(d, state(0.5 * (fs[i] + fs[i + 1]), 0.5 * (ths[k] + ths[k + 1]), d))
            assert got == pytest.approx(tuple(mid), rel=1e-9, abs=1e-9)


def test_vanishing_density_carries_no_pressure(oracle_mod):
    # reading of Sec. 2 (f <= 1 must hold): N <= 0, and a density so small
    # that 1/(c_r N) overflows, carry no radiation pressure; the flux
    # component of G is F_d either way.  With UL = UR the GLF flux is G.
    o = make((2, 2, 2), (0,) * 6)
    for N in (0.0, 1e-320, -1e-10):
        U = np.array([N, 1e-300, -2e-300, 0.0])
        for d in range(3):
            G = o.face_flux(d, U, U)
            assert G[0] == U[1 + d] and G[1] == 0.0 and G[2] == 0.0 and G[3] == 0.0, (N, d, G)
    # a density just above that limit keeps its pressure: f = 1 along F
    N = 1e-300 / C_R
    U = np.array([N, 1e-300, 0.0, 0.0])
    G = o.face_flux(0, U, U)
    assert G[1] == pytest.approx(C_R * C_R * N, rel=1e-14) and G[2] == 0.0


def test_hll_speeds_contain_the_reduced_flux(oracle_mod):
    # The exact eigenvalues of the flux Jacobian bracket a cell's reduced
    # flux f cos(theta) (checked here by an eigen-solve); the HLL flux keeps
    # that bracket with the widened table speeds, so an empty cell upstream
    # of a beam gives nothing to it: Phi_N(empty | beam) <= 0.
    rng = np.random.default_rng(5)
    fs = np.concatenate([np.ones(200), rng.uniform(0.9, 1.0, 200), rng.uniform(0, 0.9, 100)])
    ths = rng.uniform(0, np.pi / 2, fs.size)
    o = make((2, 2, 2), (0,) * 6, flux=1, hll=physics.hll_table())
    empty = np.zeros(4)
    for f, th in zip(fs, ths):
        if f < 1:
            ev = np.linalg.eigvals(physics.m1_jacobian(f, np.array([th]))[0]).real
            assert ev.min() <= f * math.cos(th) <= ev.max()
        ph = rng.uniform(0, 2 * np.pi)
        n = np.array([math.cos(th), math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph)])
        R = np.array([1.0, *(f * C_R * n)])
        lo, hi = o.hll_eig(0, R)
        phi = o.face_flux(0, empty, R)
        assert phi[0] <= 1e-15 * C_R, (f, th, lo, hi, f * math.cos(th), phi[0])


def test_hll_beam_next_to_empty_cells_stays_positive_and_conservative(oracle_mod):
    # a beam at an angle between the table's nodes in an otherwise empty box:
    # no cell goes negative and no photon is created
    for th in (0.3, 1.0, 2.2):
        o = make((5, 5, 5), (1,) * 6, flux=1, hll=physics.hll_table())
        st = random_state((5, 5, 5), 1, np.random.default_rng(0))
        st["N"][:] = 0.0
        st["F"][:] = 0.0
        st["N"][0, 2, 2, 2] = 1.0
        st["F"][0, :, 2, 2, 2] = C_R * np.array([math.cos(th), math.sin(th), 0.0])
        o.transport(st, o.courant_dt())
        assert st["N"].min() >= 0.0
        assert abs(st["N"].sum() - 1.0) < 1e-14


@pytest.mark.parametrize("flux", [0, 1])
def test_transport_keeps_photon_density_nonnegative(oracle_mod, flux):
    # random states with empty cells and exact beams at random angles,
    # periodic, several steps: N >= 0 everywhere and the total conserved
    rng = np.random.default_rng(7)
    n = (7, 6, 5)
    o = make(n, (0,) * 6, flux=flux, hll=physics.hll_table(), M=1)
    st = random_state(n, 1, rng)
    st["N"][rng.uniform(size=st["N"].shape) < 0.5] = 0.0
    st["N"] *= 10.0 ** rng.uniform(-6, 0, st["N"].shape)
    d = st["F"] / np.maximum(np.linalg.norm(st["F"], axis=1, keepdims=True), 1e-300)
    st["F"] = np.ascontiguousarray(d * C_R * st["N"][:, None])  # every cell a beam
    tot = st["N"].sum()
    for _ in range(6):
        o.transport(st, o.courant_dt())
        assert st["N"].min() >= 0.0
    assert abs(st["N"].sum() / tot - 1) < 1e-13
