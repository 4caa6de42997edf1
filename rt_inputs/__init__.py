"""Seeded synthetic inputs for the explicit M1 RT step.

This module is shared by the HIP path's tests/benchmark and by the CPU oracle.
It holds no arithmetic of the method itself: only unit constants, the
workload descriptions (grid, gas, sources, spectra as *descriptions*), and
seeded random generators for density fields and source lists.  Everything
the method derives from these (time steps, group cross sections, photon
splits between groups, HLL eigenvalues) is computed separately on each side.

Workloads follow the tests of Iliev et al. (2006) as used in the paper's
Sec. 6 (tests 1 and 2: 6.6 kpc box, n_H = 1e-3 cm^-3, 5e48 photons/s,
c_r = c/100, Courant factor 0.8, three blackbody groups of a 1e5 K source);
the cosmological density field of Iliev test 4 is not available, so a
lognormal field with P(k) ~ k^-3 of the same mean density stands in for it.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

# ---- unit constants (cgs) -------------------------------------------------
C_LIGHT = 2.99792458e10          # cm/s
KPC = 3.0856775814913673e21      # cm
YR = 3.15576e7                   # s (Julian year)
MYR = 1e6 * YR
EV = 1.602176634e-12             # erg

# group edges of the paper's tests: ]13.6, 24.59], ]24.59, 54.42], ]54.42, inf[ eV
EDGES_3 = (13.6, 24.59, 54.42, np.inf)
EDGES_2 = (13.6, 24.59, np.inf)
EDGES_1 = (13.6, np.inf)

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_INFLOW = 0, 1, 2, 3
FLUX_GLF, FLUX_HLL = 0, 1


@dataclasses.dataclass
class Spectrum:
    """Source spectrum description.  kind='bb': blackbody at T_bb between
    group edges (eV).  kind='mono': monochromatic groups with given
    cross sections (cm^2, [group][HI,HeI,HeII]) and photon energies (eV)."""
    kind: str
    T_bb: float = 1e5
    edges_eV: Sequence[float] = EDGES_3
    mono_sigma: Optional[Sequence[Sequence[float]]] = None
    mono_energy_eV: Optional[Sequence[float]] = None

    @property
    def M(self) -> int:
        if self.kind == "mono":
            return len(self.mono_energy_eV)
        return len(self.edges_eV) - 1


# ionisation energies [eV] of the species whose recombinations to the ground
# state emit ionising photons: HII (-> HI), HeII (-> HeI), HeIII (-> HeII)
RECOMBINING_THRESHOLDS_EV = (13.60, 24.59, 54.42)


def recombination_groups(spec: "Spectrum") -> tuple:
    """For each of HII, HeII, HeIII the photon group its recombination
    photons go to (just above the threshold): the blackbody group whose
    energy interval holds the threshold, or the monochromatic group of the
    lowest energy at or above it; -1 where there is none."""
    out = []
    for e in RECOMBINING_THRESHOLDS_EV:
        g = -1
        if spec.kind == "mono":
            best = None
            for i, ei in enumerate(spec.mono_energy_eV):
                if ei >= e - 1e-9 and (best is None or ei < best):
                    best, g = ei, i
        else:
            ed = spec.edges_eV
            for i in range(len(ed) - 1):
                if ed[i] - 1e-9 <= e < ed[i + 1] - 1e-9:
                    g = i
        out.append(g)
    return tuple(out)


@dataclasses.dataclass
class Workload:
    name: str
    n: Sequence[int]               # (nx, ny, nz)
    L: float                       # box side along x [cm]
    bc: Sequence[int]              # -x,+x,-y,+y,-z,+z
    spectrum: Spectrum
    X: float
    Y: float
    T0: float
    xHII0: float
    xHeII0: float
    xHeIII0: float
    isothermal: bool
    flux: int
    steps: int
    c_r: float = C_LIGHT / 100.0
    courant: float = 0.8
    otsa: bool = True
    gamma: float = 5.0 / 3.0
    a_exp: float = 1.0
    x_min: float = 1e-6
    nH_mean: float = 1e-3
    sigma_ln: float = 0.0          # 0 -> uniform density
    n_sources: int = 1
    seed: int = 0
    # a uniform sphere of other gas: ((centre x, y, z) [cm], radius [cm], n_H, T, x_HII)
    clump: Optional[tuple] = None
    # photons s^-1 cm^-2 entering through each BC_INFLOW face, summed over groups
    inflow_total: Optional[Sequence[float]] = None

    @property
    def dx(self) -> float:
        return self.L / self.n[0]

    def inflow_flux(self, group_frac) -> np.ndarray:
        """(6, M) photon flux per face and group entering through the
        BC_INFLOW faces: the total split by the groups' photon fractions."""
        M = self.spectrum.M
        out = np.zeros((6, M))
        if self.inflow_total is not None:
            f = np.asarray(group_frac[:M], np.float64)
            f = f / f.sum()
            for face in range(6):
                if self.bc[face] == BC_INFLOW:
                    out[face] = self.inflow_total[face] * f
        return out

    @property
    def brec(self) -> tuple:
        return recombination_groups(self.spectrum)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))


def lognormal_nH(n: Sequence[int], sigma_ln: float, mean: float, seed: int) -> np.ndarray:
    """Lognormal density field of an isotropic Gaussian random field with
    P(k) ~ k^-3: white noise -> rFFT -> amplitude k^-3/2 (k = 0 mode
    removed) -> inverse FFT -> unit variance; n_H = mean exp(s d)/<exp(s d)>.
    Returns an array of shape (nz, ny, nx), float64, grid mean exactly `mean`
    up to rounding."""
    nx, ny, nz = (int(v) for v in n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    wk = np.fft.rfftn(w)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(k)
    nz_mask = k > 0
    amp[nz_mask] = k[nz_mask] ** -1.5
    d = np.fft.irfftn(wk * amp, s=(nz, ny, nx), axes=(0, 1, 2))
    d -= d.mean()
    sd = d.std()
    if sd > 0:
        d /= sd
    e = np.exp(sigma_ln * d)
    return np.ascontiguousarray(mean * e / e.mean())


def random_sources(n: Sequence[int], K: int, seed: int, log_lo: float = 47.0, log_hi: float = 49.0):
    """K point sources at uniform random cells with log10(Ndot) ~ U[log_lo, log_hi].
    Returns (ijk int32 (K,3) as (ix,iy,iz), Ndot float64 (K,)) in photons/s."""
    rng = np.random.default_rng(seed + 1000)
    nx, ny, nz = (int(v) for v in n)
    ijk = np.stack([rng.integers(0, nx, K), rng.integers(0, ny, K), rng.integers(0, nz, K)], axis=1)
    ndot = 10.0 ** rng.uniform(log_lo, log_hi, K)
    return np.ascontiguousarray(ijk.astype(np.int32)), np.ascontiguousarray(ndot.astype(np.float64))


def workload_sources(w: Workload):
    """Sources of a workload: the corner source of the Iliev tests (one
    octant of a 5e48 photons/s source in cell (0,0,0) of a reflecting corner)
    or K random sources."""
    if w.name.startswith("stromgren"):
        return np.zeros((1, 3), np.int32), np.array([5e48 / 8.0])
    return random_sources(w.n, w.n_sources, w.seed)


def initial_state(w: Workload):
    """Initial gas and radiation fields (float64 numpy, shape (nz,ny,nx)):
    dict with nH, xHII, xHeII, xHeIII, T, and N (M,...) / F (M,3,...) zeros."""
    nx, ny, nz = w.n
    shp = (nz, ny, nx)
    if w.sigma_ln > 0:
        nH = lognormal_nH(w.n, w.sigma_ln, w.nH_mean, w.seed)
    else:
        nH = np.full(shp, w.nH_mean)
    M = w.spectrum.M
    st = {
        "nH": nH,
        "xHII": np.full(shp, w.xHII0),
        "xHeII": np.full(shp, w.xHeII0),
        "xHeIII": np.full(shp, w.xHeIII0),
        "T": np.full(shp, w.T0),
        "N": np.zeros((M,) + shp),
        "F": np.zeros((M, 3) + shp),
    }
    if w.clump is not None:
        (xc, yc, zc), r, n_in, T_in, x_in = w.clump
        dx = w.dx
        z, y, x = np.meshgrid((np.arange(nz) + 0.5) * dx, (np.arange(ny) + 0.5) * dx, (np.arange(nx) + 0.5) * dx,
                              indexing="ij")
        inside = (x - xc) ** 2 + (y - yc) ** 2 + (z - zc) ** 2 <= r * r
        st["nH"][inside] = n_in
        st["T"][inside] = T_in
        st["xHII"][inside] = x_in
    return st


# ---- the paper-derived workloads -----------------------------------------
MONO_13p6 = Spectrum(kind="mono", mono_sigma=[[6.3e-18, 0.0, 0.0]], mono_energy_eV=[13.6])


def stromgren_32(steps: int = 100) -> Workload:
    """Isothermal H II region (Iliev test 1) on a uniform 32^3 grid: 6.6 kpc,
    n_H = 1e-3, x_HII = 1.2e-3, T = 1e4 K fixed, monochromatic 13.6 eV
    photons with sigma_HI = 6.3e-18 cm^2, corner source of 5e48 photons/s,
    GLF, reflecting faces through the source corner and outflow elsewhere."""
    return Workload(name="stromgren_32", n=(32, 32, 32), L=6.6 * KPC,
                    bc=(BC_REFLECT, BC_OUTFLOW) * 3, spectrum=MONO_13p6,
                    X=1.0, Y=0.0, T0=1e4, xHII0=1.2e-3, xHeII0=0.0, xHeIII0=0.0,
                    isothermal=True, flux=FLUX_GLF, steps=steps)


def shadow_clump(n: int = 128, steps: int = 100) -> Workload:
    """Iliev test 3 (Sec. 6) on a uniform n^3 grid: a 6.6 kpc box of hydrogen
    (n_H = 2e-4, T = 8000 K, x_HII at the floor 1e-6) with a sphere of radius
    0.8 kpc at (5, 3.3, 3.3) kpc of 200x denser gas (T = 40 K, x_HII = 1e-6);
    a constant flux of 1e6 photons s^-1 cm^-2 enters through the x = 0 face,
    the other faces let radiation out; three groups of a 1e5 K blackbody,
    HLL, OTSA, c_r = c/10, T evolving.  No point sources."""
    L = 6.6 * KPC
    return Workload(name=f"shadow_clump_{n}", n=(n, n, n), L=L,
                    bc=(BC_INFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW, BC_OUTFLOW),
                    spectrum=Spectrum(kind="bb", T_bb=1e5, edges_eV=EDGES_3),
                    X=1.0, Y=0.0, T0=8000.0, xHII0=1e-6, xHeII0=0.0, xHeIII0=0.0,
                    isothermal=False, flux=FLUX_HLL, steps=steps, c_r=C_LIGHT / 10.0,
                    nH_mean=2e-4, n_sources=0,
                    clump=((5.0 * KPC, 3.3 * KPC, 3.3 * KPC), 0.8 * KPC, 4e-2, 40.0, 1e-6),
                    inflow_total=(1e6, 0, 0, 0, 0, 0))


def lognormal_box(n: int, L_kpc: float, n_sources: int, steps: int, seed: int = 0,
                  flux: int = FLUX_HLL, spectrum: Optional[Spectrum] = None, sigma_ln: float = 1.0,
                  name: Optional[str] = None) -> Workload:
    """H+He gas (X=0.76, Y=0.24) with evolving temperature (T0 = 100 K,
    x_HII = 1e-6, He neutral), lognormal density of mean 1e-3 cm^-3, random
    sources with log-uniform rates in [1e47, 1e49] photons/s, three groups of a
    1e5 K blackbody, periodic box."""
    return Workload(name=name or f"lognormal_{n}", n=(n, n, n), L=L_kpc * KPC,
                    bc=(BC_PERIODIC,) * 6,
                    spectrum=spectrum or Spectrum(kind="bb", T_bb=1e5, edges_eV=EDGES_3),
                    X=0.76, Y=0.24, T0=100.0, xHII0=1e-6, xHeII0=0.0, xHeIII0=0.0,
                    isothermal=False, flux=flux, steps=steps, sigma_ln=sigma_ln,
                    n_sources=n_sources, seed=seed)


def lognormal_128(steps: int = 200, seed: int = 0) -> Workload:
    return lognormal_box(128, 6.6, 50, steps, seed)


def lognormal_256(steps: int = 100, seed: int = 0) -> Workload:
    return lognormal_box(256, 13.2, 200, steps, seed)


def subbox(w: Workload, n_sub: int):
    """The cells [0, n_sub)^3 of workload w's realisation (density field and
    the sources inside them) as a periodic box of its own, with the same cell
    size: (workload, initial state, source cells (K,3), source rates (K,))."""
    ws = dataclasses.replace(w, name=f"{w.name}_sub{n_sub}", n=(n_sub,) * 3, L=n_sub * w.dx,
                             bc=(BC_PERIODIC,) * 6)
    full = lognormal_nH(w.n, w.sigma_ln, w.nH_mean, w.seed) if w.sigma_ln > 0 else None
    st = initial_state(ws)
    if full is not None:
        st["nH"] = np.ascontiguousarray(full[:n_sub, :n_sub, :n_sub])
    ijk, nd = random_sources(w.n, w.n_sources, w.seed)
    keep = np.all(ijk < n_sub, axis=1)
    ws.n_sources = int(keep.sum())
    return ws, st, np.ascontiguousarray(ijk[keep]), np.ascontiguousarray(nd[keep])


def grey_box(n: int, L_kpc: float, n_sources: int, steps: int, seed: int = 0, isothermal: bool = False,
             sigma_ln: float = 0.8) -> Workload:
    """Periodic hydrogen-only box (X = 1, Y = 0) with one grey group
    [13.6 eV, inf) of a 1e5 K blackbody, lognormal density (mean 1e-3,
    sigma_ln), K random sources, GLF.  Isothermal: the gas of the Stromgren
    test (T = 1e4 K fixed, x_HII = 1.2e-3); otherwise T evolves from 100 K
    with x_HII = 1e-6."""
    w = lognormal_box(n, L_kpc, n_sources, steps, seed, flux=FLUX_GLF,
                      spectrum=Spectrum(kind="bb", T_bb=1e5, edges_eV=EDGES_1),
                      sigma_ln=sigma_ln, name=f"grey_{n}")
    w.X, w.Y = 1.0, 0.0
    if isothermal:
        w.isothermal, w.T0, w.xHII0 = True, 1e4, 1.2e-3
    return w


def grey_64(steps: int = 300, seed: int = 0, isothermal: bool = False) -> Workload:
    """The differentiation workload: 64^3, 3.3 kpc, 16 sources, sigma_ln = 0.8."""
    return grey_box(64, 3.3, 16, steps, seed, isothermal=isothermal)


def perturbed_log_rates(ndot: np.ndarray, seed: int, scale: float = 0.1) -> np.ndarray:
    """ln(Ndot) + scale * xi, xi ~ N(0, 1) per source (seed + 3000): the
    source rates of the run that makes the target of the gradient tests."""
    rng = np.random.default_rng(seed + 3000)
    return np.log(np.asarray(ndot, np.float64)) + scale * rng.standard_normal(len(ndot))


@dataclasses.dataclass
class BoxSpec:
    side: int
    M: int
    nH: float
    n_sources: int
    seed: int


def batch_boxes(nbox: int = 64, seed: int = 0) -> List[BoxSpec]:
    """Independent periodic boxes of uneven size: side ~ U{16,24,32,48,64,96},
    1-3 groups, uniform density with log10 n_H ~ U[-4,-1], 1-8 sources."""
    rng = np.random.default_rng(seed + 2000)
    sides = np.array([16, 24, 32, 48, 64, 96])
    out = []
    for b in range(nbox):
        out.append(BoxSpec(side=int(rng.choice(sides)), M=int(rng.integers(1, 4)),
                           nH=float(10.0 ** rng.uniform(-4, -1)),
                           n_sources=int(rng.integers(1, 9)), seed=int(seed * 1000 + b)))
    return out


def batch_box_workload(b: BoxSpec, dx: float, steps: int) -> Workload:
    edges = {1: EDGES_1, 2: EDGES_2, 3: EDGES_3}[b.M]
    w = Workload(name=f"box{b.seed}", n=(b.side,) * 3, L=b.side * dx, bc=(BC_PERIODIC,) * 6,
                 spectrum=Spectrum(kind="bb", T_bb=1e5, edges_eV=edges),
                 X=0.76, Y=0.24, T0=100.0, xHII0=1e-6, xHeII0=0.0, xHeIII0=0.0,
                 isothermal=False, flux=FLUX_GLF, steps=steps, nH_mean=b.nH, sigma_ln=0.0,
                 n_sources=b.n_sources, seed=b.seed)
    return w
