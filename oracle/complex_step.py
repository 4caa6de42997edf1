"""Complex-step reference derivatives of the RT step.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite may use
it.  It shares no code with the HIP library.

The differentiation setting is hydrogen-only gas (Y = 0), one photon group,
GLF transport and a periodic box, in FP64.  This module runs the same step
as the C oracle -- injection (Sec. 3.1), unsplit GLF transport with the M1
closure at the reduced light speed (Sec. 2, eqs. edd2, eddTens, Udir;
Sec. 3.2, eqs. dUdt_sol, glf), and the subcycled thermochemistry of App. A
with the case-B rates of App. E -- in complex128 numpy arithmetic.  Every
decision of the method (the 10% checks, the doubling and halving of the
substep, the clamps of x_HII) is taken on real parts, so that the real part
is the oracle's own result and, with parameters p + i e v (e = 1e-30), the
imaginary part is e times the derivative along v of the branch that the
real computation takes (complex-step differentiation: Squire & Trapp 1998;
Martins, Sturdza & Alonso 2003).  Holding the branch fixed is the
derivative the adjoint computes: the substep schedule is piecewise
constant in the state.

Functions written here are analytic continuations of the real formulas:
|F| = sqrt(Fx^2 + Fy^2 + Fz^2) without conjugation, comparisons and
absolute values on real parts only.  The chemistry is vectorised over cells
and advanced in lockstep: each pass makes one attempt in every cell that has
time left, exactly the per-cell loop of App. A.
"""
from __future__ import annotations

import numpy as np

KB = 1.380649e-16
EV = 1.602176634e-12
EPS_HI = 13.60 * EV          # App. E.4 threshold
TL_HI = 315614.0             # Hui & Gnedin threshold temperature of HI (App. E.2)


# ------------------------------------------------------------- App. E rates
def _cen(A, Tj, T):
    """A sqrt(T) / (1 + sqrt(T/1e5)) exp(-Tj/T) and d/dT (E.1, zeta of E.3)."""
    sq = np.sqrt(T)
    g = 1.0 / (1.0 + np.sqrt(T / 1e5))
    e = np.exp(-Tj / T)
    v = A * sq * g * e
    d = A * ((0.5 / sq) * g * e + sq * (-g * g * 0.5 / np.sqrt(T * 1e5)) * e + sq * g * e * Tj / (T * T))
    return v, d


def _hg(A, TL, p, l0, q, r, T):
    """Hui & Gnedin form A lam^p (1 + (lam/l0)^q)^-r, lam = TL/T, and d/dT (E.2)."""
    lam = TL / T
    u = (lam / l0) ** q
    v = A * lam ** p * (1.0 + u) ** (-r)
    dlam = A * (p * lam ** (p - 1.0) * (1.0 + u) ** (-r) - r * lam ** p * (1.0 + u) ** (-r - 1.0) * q * u / lam)
    return v, dlam * (-lam / T)


def beta_HI(T):
    return _cen(5.85e-11, 157809.1, T)


def alphaB_HII(T):
    return _hg(2.753e-14, TL_HI, 1.5, 2.74, 0.407, 2.242, T)


def cooling_H(T, ne, nHI, nHII, a_exp):
    """Primordial cooling of hydrogen-only gas, case B (eq. rate_cooling
    with the helium densities zero): collisional ionisation (zeta) and
    excitation (psi) of HI, recombination cooling of HII (eta_B),
    bremsstrahlung (theta), Compton (varpi).  Returns (L, dL/dT)."""
    zv, zd = _cen(1.27e-21, 157809.1, T)
    g = 1.0 / (1.0 + np.sqrt(T / 1e5))
    dg = -g * g * 0.5 / np.sqrt(T * 1e5)
    ep = np.exp(-118348.0 / T)
    pv = 7.5e-19 * g * ep
    pd = 7.5e-19 * (dg * ep + g * ep * 118348.0 / (T * T))
    hv, hd = _hg(1.0, TL_HI, 1.97, 2.25, 0.376, 3.72, T)
    ev = 3.435e-30 * T * hv
    ed = 3.435e-30 * hv + 3.435e-30 * T * hd
    tv = 1.42e-27 * np.sqrt(T)
    td = 1.42e-27 * 0.5 / np.sqrt(T)
    Tg = 2.727 / a_exp
    cv = 1.017e-37 * Tg ** 4 * (T - Tg)
    cd = 1.017e-37 * Tg ** 4
    L = (zv + pv) * ne * nHI + ev * ne * nHII + tv * ne * nHII + cv * ne
    dL = (zd + pd) * ne * nHI + ed * ne * nHII + td * ne * nHII + cd * ne
    return L, dL


# ----------------------------------------------------------------- settings
class CSParams:
    """Grid (n = (nx, ny, nz), dx), one group (c_r, sigma_N, sigma_E of HI,
    mean energy ebar [erg]) and gas parameters of the hydrogen-only step."""

    def __init__(self, n, dx, c_r, sigN, sigE, ebar, isothermal, X=1.0, gamma=5.0 / 3.0, a_exp=1.0,
                 x_min=1e-6, N_floor=0.0, max_attempts=100000):
        self.n = tuple(int(v) for v in n)
        self.dx = float(dx)
        self.c_r = float(c_r)
        self.sigN = float(sigN)
        self.sigE = float(sigE)
        self.ebar = float(ebar)
        self.isothermal = bool(isothermal)
        self.X = float(X)
        self.gamma = float(gamma)
        self.a_exp = float(a_exp)
        self.x_min = float(x_min)
        self.N_floor = float(N_floor)
        self.max_attempts = int(max_attempts)


# -------------------------------------------------------- transport (GLF)
def _pressure_row(N, F, c, d):
    """c^2 P_d. of the M1 closure for every cell: P = N D, D = (1-chi)/2 I
    + (3chi-1)/2 n n, chi = (3+4f^2)/(5+2 sqrt(4-3f^2)), f = |F|/(cN)
    capped at 1 (on the real part); zero for N <= 0."""
    Fn = np.sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2])
    has = (N.real > 0)
    safeN = np.where(has, N, 1.0)
    f = Fn / (c * safeN)
    f = np.where(f.real > 1.0, 1.0 + 0j, f)
    chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * np.sqrt(4.0 - 3.0 * f * f))
    nz = Fn.real > 0
    safeF = np.where(nz, Fn, 1.0)
    nvec = [np.where(nz, F[k] / safeF, 0.0) for k in range(3)]
    out = []
    for k in range(3):
        Dk = (0.5 * (1.0 - chi) if k == d else 0.0) + 0.5 * (3.0 * chi - 1.0) * nvec[d] * nvec[k]
        out.append(np.where(has, c * c * N * Dk, 0.0))
    return out


def transport(p, N, F, dt):
    """U' = U + dt/dx sum_d (Phi_{d,l-1/2} - Phi_{d,l+1/2}), GLF fluxes
    Phi = (G_L + G_R)/2 - c (U_R - U_L)/2, periodic neighbours, all from the
    source state.  Arrays (nz, ny, nx); F (3, nz, ny, nx)."""
    c = p.c_r
    k = dt / p.dx
    U = [N, F[0], F[1], F[2]]
    acc = [np.zeros_like(N) for _ in range(4)]
    for d in range(3):
        ax = 2 - d
        P = _pressure_row(N, F, c, d)
        G = [F[d], P[0], P[1], P[2]]
        for m in range(4):
            Gp = np.roll(G[m], -1, axis=ax)
            Up = np.roll(U[m], -1, axis=ax)
            phi_plus = 0.5 * (G[m] + Gp) - 0.5 * c * (Up - U[m])     # face l+1/2
            phi_minus = np.roll(phi_plus, 1, axis=ax)                 # face l-1/2
            acc[m] = acc[m] + (phi_minus - phi_plus)
    Nn = N + k * acc[0]
    Fn = np.stack([F[0] + k * acc[1], F[1] + k * acc[2], F[2] + k * acc[3]])
    return Nn, Fn


def inject(p, N, dt, ijk, ndot):
    """N += Ndot dt / dx^3 at the source cells (Sec. 3.1, f_esc = 1)."""
    N = N.copy()
    V = p.dx ** 3
    for s in range(len(ijk)):
        ix, iy, iz = (int(v) for v in ijk[s])
        N[iz, iy, ix] = N[iz, iy, ix] + ndot[s] * dt / V
    return N


# ------------------------------------------------------------ chemistry
def thermochem(p, N, F, x, T, nH, dt):
    """App. A for every cell over dt (hydrogen only, one group, case B).
    Arrays flattened to (ncell,) complex; F (3, ncell).  Returns the new
    (N, F, x, T) and the accepted-substep counts."""
    X = p.X
    iso = p.isothermal
    N = N.copy()
    F = F.copy()
    x = x.copy()
    nc = N.shape[0]
    Tiso = T.copy()
    mu = lambda xx: 1.0 / (X * (1.0 + xx))
    Tmu = T / mu(x)
    K = (p.gamma - 1.0) * X / (nH * KB)
    rem = np.full(nc, float(dt))
    h = np.full(nc, float(dt))
    att = np.zeros(nc, np.int64)
    acc = np.zeros(nc, np.int64)
    active = np.ones(nc, bool)
    sN, sE, eb, cr = p.sigN, p.sigE, p.ebar, p.c_r
    while active.any():
        idx = np.nonzero(active)[0]
        cap = att[idx] >= p.max_attempts
        if cap.any():
            active[idx[cap]] = False
            idx = idx[~cap]
            if idx.size == 0:
                break
        att[idx] += 1
        hi = h[idx]
        ri = rem[idx]
        hh = np.where(hi >= ri * (1.0 - 1e-10), ri, hi)
        xi, Ni, Fi, Tmi, nHi, Ki = x[idx], N[idx], F[:, idx], Tmu[idx], nH[idx], K[idx]
        # task 1: photons, semi-implicit absorption
        nHI = (1.0 - xi) * nHi
        nHII = xi * nHi
        D = cr * sN * nHI
        Nn = Ni / (1.0 + hh * D)
        Fn = Fi / (1.0 + hh * D)
        rN = np.where(Ni.real > p.N_floor, np.abs(Nn.real - Ni.real) / np.where(Ni.real > p.N_floor, Ni.real, 1.0),
                      0.0)
        fail = rN > 0.1
        maxrel = rN.copy()
        mu0 = mu(xi)
        ne0 = nHII
        # task 2: T_mu, semi-implicit
        if not iso:
            T0 = Tmi * mu0
            H = nHI * cr * Nn * (eb * sE - EPS_HI * sN)
            L, dL = cooling_H(T0, ne0, nHI, nHII, p.a_exp)
            Lam = H - L
            Lamp = -mu0 * dL
            den = 1.0 - Lamp * Ki * hh
            fail |= ~(den.real > 0.0)
            Tmun = Tmi + Lam * Ki * hh / den
            rT = np.abs(Tmun.real - Tmi.real) / Tmi.real
            fail |= (rT > 0.1) | (np.abs((Ki * Lam).real * hh) / Tmi.real > 0.1)
            maxrel = np.maximum(maxrel, rT)
            T1 = Tmun * mu0
        else:
            Tmun = Tmi
            T1 = Tiso[idx]
        # task 3: x_HII, semi-implicit with the Jacobian J
        bv, bd = beta_HI(T1)
        av, ad = alphaB_HII(T1)
        C = bv * ne0 + sN * cr * Nn
        Dd = av * ne0
        if iso:
            dC = nHi * bv
            dD = nHi * av
        else:
            fT = ne0 * Tmun * mu0 * mu0 * X
            dC = nHi * bv - fT * bd
            dD = nHi * av - fT * ad
        J = dC - (C + Dd) - xi * (dC + dD)
        denx = 1.0 - J * hh
        fail |= ~(denx.real > 0.0)
        rate = C - xi * (C + Dd)
        xn = xi + hh * rate / denx
        xn = np.where(xn.real < p.x_min, p.x_min + 0j, xn)
        xn = np.where(xn.real > 1.0, 1.0 + 0j, xn)
        rx = np.abs(xn.real - xi.real) / xi.real
        fail |= (rx > 0.1) | (np.abs(rate.real) * hh / xi.real > 0.1)
        maxrel = np.maximum(maxrel, rx)
        # electron density check
        nen = xn * nHi
        re = np.abs(nen.real - ne0.real) / ne0.real
        fail |= re > 0.1
        maxrel = np.maximum(maxrel, re)
        # accept, or halve and retry
        ok = ~fail
        io = idx[ok]
        N[io] = Nn[ok]
        F[:, io] = Fn[:, ok]
        x[io] = xn[ok]
        Tmu[io] = (Tiso[io] / mu(xn[ok])) if iso else Tmun[ok]
        rem[io] = rem[io] - hh[ok]
        acc[io] += 1
        h[io] = np.where(maxrel[ok] < 0.05, 2.0 * hh[ok], hh[ok])
        active[io] = rem[io] > 0.0
        h[idx[fail]] = 0.5 * hh[fail]
    Tout = Tiso if iso else Tmu * mu(x)
    return N, F, x, Tout, acc


# ----------------------------------------------------------------- runs
def run(p, state, dt, steps, ijk, lnNdot, lnnH):
    """steps RT steps from state (dict of real arrays N (nz,ny,nx), F
    (3,nz,ny,nx), xHII, T) with source rates exp(lnNdot) and densities
    exp(lnnH) (complex allowed).  Returns the final complex state and the
    per-step substep counts."""
    N = np.asarray(state["N"], np.complex128).copy()
    F = np.asarray(state["F"], np.complex128).copy()
    x = np.asarray(state["xHII"], np.complex128).ravel().copy()
    T = np.asarray(state["T"], np.complex128).ravel().copy()
    shp = N.shape
    nH = np.exp(np.asarray(lnnH, np.complex128)).ravel()
    ndot = np.exp(np.asarray(lnNdot, np.complex128))
    counts = []
    for _ in range(steps):
        N = inject(p, N, dt, ijk, ndot)
        N, F = transport(p, N, F, dt)
        Nf, Ff, x, T, acc = thermochem(p, N.ravel(), F.reshape(3, -1), x, T, nH, dt)
        N = Nf.reshape(shp)
        F = Ff.reshape((3,) + shp)
        counts.append(acc)
    return {"N": N, "F": F, "xHII": x.reshape(shp), "T": T.reshape(shp)}, counts


def loss(final, target):
    """L = sum over cells of (x_HII - target)^2."""
    d = final["xHII"] - target
    return np.sum(d * d)


def directional_derivative(p, state, dt, steps, ijk, lnNdot, lnnH, target, v_src=None, v_cell=None,
                           eps=1e-30):
    """dL/dtheta . v by one complex-step run, theta = (ln Ndot, ln n_H)."""
    a = np.asarray(lnNdot, np.complex128).copy()
    b = np.asarray(lnnH, np.complex128).copy()
    if v_src is not None:
        a = a + 1j * eps * np.asarray(v_src, np.float64)
    if v_cell is not None:
        b = b + 1j * eps * np.asarray(v_cell, np.float64)
    fin, _ = run(p, state, dt, steps, ijk, a, b)
    return float(loss(fin, target).imag / eps)
