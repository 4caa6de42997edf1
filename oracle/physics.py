"""Host-side physics of the oracle: photoionisation cross sections, photon-group
attributes, the HLL eigenvalue table and the analytic laws the method is
pinned against.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain FP64 numpy/scipy;
shares nothing with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

EV = 1.602176634e-12
KB = 1.380649e-16
KB_EV = 8.617333262e-5  # Boltzmann constant in eV/K

# ionisation energies, App. E.4 threshold table [eV]
EPS_ION_EV = (13.60, 24.59, 54.42)

# Verner et al. (1996) fit parameters of App. E.4 (Table sigma.tbl):
# (eps0 [eV], sigma0 [cm^2], P, y_a, y_w, y0, y1).  The HeI eps0 is printed as
# 0.1361 eV; it is read as 13.61 eV (the printed value gives an HeI threshold
# cross section of ~1e-23 cm^2 instead of the known ~7.4e-18 cm^2).
VERNER = (
    (0.4298, 5.475e-14, 2.963, 32.88, 0.0, 0.0, 0.0),      # HI
    (13.61, 9.492e-16, 3.188, 1.469, 2.039, 0.4434, 2.136),  # HeI
    (1.720, 1.369e-14, 2.963, 32.88, 0.0, 0.0, 0.0),       # HeII
)


def sigma_verner(eps_eV, j: int):
    """Photoionisation cross section of species j (0 HI, 1 HeI, 2 HeII) at
    photon energy eps [eV], eq. (PhI); zero below the ionisation energy."""
    e0, s0, P, ya, yw, y0, y1 = VERNER[j]
    eps = np.asarray(eps_eV, dtype=np.float64)
    x = eps / e0 - y0
    y = np.sqrt(x * x + y1 * y1)
    s = s0 * ((x - 1.0) ** 2 + yw * yw) * y ** (0.5 * P - 5.5) * (1.0 + np.sqrt(y / ya)) ** (-P)
    return np.where(eps >= EPS_ION_EV[j], s, 0.0)


def planck_energy(eps_eV, T):
    """Blackbody spectral energy distribution J per unit photon energy,
    up to a constant: eps^3 / (exp(eps/kT) - 1)."""
    u = eps_eV / (KB_EV * T)
    if u > 700.0:
        return 0.0
    return eps_eV ** 3 / math.expm1(u)


def _quad(fun, a, b):
    """Integral of fun over [a, b], split at the ionisation thresholds inside."""
    pts = [a] + [e for e in EPS_ION_EV if a < e < b] + [b]
    tot = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        v, _ = integrate.quad(fun, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)
        tot += v
    return tot


def group_attributes(T_bb: float, edges_eV):
    """Group-averaged cross sections of eq. (csn_multi) [cm^2], energy-weighted
    cross sections of eq. (cse_multi) [cm^2], mean photon energies of
    eq. (egy_multi) [erg], and photon-number fractions of each group over the
    whole ionising range, for a blackbody source of temperature T_bb."""
    M = len(edges_eV) - 1
    sigN = np.zeros((3, 3))
    sigE = np.zeros((3, 3))
    ebar = np.zeros(3)
    frac = np.zeros(3)
    J = lambda e: planck_energy(e, T_bb)
    Jn = lambda e: planck_energy(e, T_bb) / e
    ntot = _quad(Jn, edges_eV[0], edges_eV[-1])
    for i in range(M):
        a, b = edges_eV[i], edges_eV[i + 1]
        n_i = _quad(Jn, a, b)
        e_i = _quad(J, a, b)
        ebar[i] = e_i / n_i * EV
        frac[i] = n_i / ntot
        for j in range(3):
            sigN[i, j] = _quad(lambda e: float(sigma_verner(e, j)) * Jn(e), a, b) / n_i
            sigE[i, j] = _quad(lambda e: float(sigma_verner(e, j)) * J(e), a, b) / e_i
    return sigN, sigE, ebar, frac


def mono_attributes(sigma, energy_eV):
    """Monochromatic groups set by hand (Sec. 2 allows attributes by hand)."""
    M = len(energy_eV)
    sigN = np.zeros((3, 3))
    sigE = np.zeros((3, 3))
    ebar = np.zeros(3)
    frac = np.zeros(3)
    for i in range(M):
        sigN[i, :] = sigma[i]
        sigE[i, :] = sigma[i]
        ebar[i] = energy_eV[i] * EV
        frac[i] = 1.0 / M
    return sigN, sigE, ebar, frac


def spectrum_attributes(spec):
    if spec.kind == "mono":
        return mono_attributes(spec.mono_sigma, spec.mono_energy_eV)
    return group_attributes(spec.T_bb, spec.edges_eV)


# ---------------------------------------------------------------------------
# HLL eigenvalues (Sec. 3.2): the extreme eigenvalues of the flux Jacobian
# dG_x/dU of the M1 system at c = 1, as functions of the reduced flux f and
# the angle theta between F and the interface normal.  The Jacobian is taken
# by complex-step differentiation of the closure as written in Sec. 2, and
# numpy's general eigen-solver gives the eigenvalues.
# ---------------------------------------------------------------------------
def _flux_x_complex(U):
    """G_x(U) for complex U (shape (..., 4)), c = 1, straight from eqs.
    (edd2)-(Udir): chi(f), n = F/|F|, D = (1-chi)/2 I + (3chi-1)/2 n n, P = N D."""
    N = U[..., 0]
    F = U[..., 1:]
    F2 = np.sum(F * F, axis=-1)
    s = F2 / (N * N)
    chi = (3.0 + 4.0 * s) / (5.0 + 2.0 * np.sqrt(4.0 - 3.0 * s))
    safe = np.where(F2 == 0, 1.0, F2)
    nn_x = F[..., 0:1] * F / safe[..., None]            # row x of n (x) n
    nn_x = np.where((F2 == 0)[..., None], 0.0, nn_x)
    Dx = 0.5 * (3.0 * chi[..., None] - 1.0) * nn_x
    Dx[..., 0] += 0.5 * (1.0 - chi)
    G = np.empty(U.shape, dtype=U.dtype)
    G[..., 0] = F[..., 0]
    G[..., 1:] = N[..., None] * Dx
    return G


def m1_jacobian(f, theta):
    """dG_x/dU (4x4) at N = 1, F = f (cos theta, sin theta, 0), c = 1."""
    f = np.asarray(f, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    shp = np.broadcast(f, theta).shape
    U = np.zeros(shp + (4,), dtype=np.complex128)
    U[..., 0] = 1.0
    U[..., 1] = f * np.cos(theta)
    U[..., 2] = f * np.sin(theta)
    h = 1e-30
    J = np.zeros(shp + (4, 4))
    for k in range(4):
        Uk = U.copy()
        Uk[..., k] += 1j * h
        J[..., :, k] = _flux_x_complex(Uk).imag / h
    return J


def hll_table(nf: int = 101, nth: int = 101):
    """Table of (lambda_min, lambda_max) on uniform nodes f in [0,1], theta in
    [0, pi]; shape (nf, nth, 2).  On the f = 1 row (a single beam) every
    eigenvalue equals cos(theta), the limit of the f < 1 rows."""
    fs = np.linspace(0.0, 1.0, nf)
    ths = np.linspace(0.0, np.pi, nth)
    F, TH = np.meshgrid(fs[:-1], ths, indexing="ij")
    J = m1_jacobian(F, TH)
    ev = np.linalg.eigvals(J).real
    tab = np.zeros((nf, nth, 2))
    tab[:-1, :, 0] = ev.min(axis=-1)
    tab[:-1, :, 1] = ev.max(axis=-1)
    tab[-1, :, 0] = np.cos(ths)
    tab[-1, :, 1] = np.cos(ths)
    return np.ascontiguousarray(tab)


# ---------------------------------------------------------------------------
# Analytic laws of Sec. 4.2 and the Iliev test 1 (Sec. 6)
# ---------------------------------------------------------------------------
def alpha_B_HII(T):
    """Case-B H recombination rate of App. E.2 (Hui & Gnedin fit)."""
    lam = 315614.0 / T
    return 2.753e-14 * lam ** 1.5 / (1.0 + (lam / 2.74) ** 0.407) ** 2.242


def stromgren_radius(ndot, nH, alphaB):
    """eq. (Stromgren_radius): (3 Ndot / (4 pi alpha_B n_H^2))^(1/3)."""
    return (3.0 * ndot / (4.0 * math.pi * alphaB * nH * nH)) ** (1.0 / 3.0)


def t_rec(nH, alphaB):
    """recombination time (n_H alpha_B)^-1."""
    return 1.0 / (nH * alphaB)


def ifront_radius(t, r_s, trec):
    """eq. (r_analyt): r_S (1 - exp(-t/t_rec))^(1/3)."""
    return r_s * (1.0 - math.exp(-t / trec)) ** (1.0 / 3.0)


def shapiro_y(w, q):
    """I-front radius y = r_I/r_S solving eq. (Stromgr_w_rel) w = q y - ln(1 - y^3)."""
    if w <= 0:
        return 0.0
    g = lambda y: q * y - math.log1p(-y ** 3) - w
    return optimize.brentq(g, 0.0, 1.0 - 1e-15, xtol=1e-15, rtol=1e-14)
