// rt_cell.h -- per-cell device code of the RT step shared by the grid
// kernels (rt_kernels.hip) and the batched kernels (rt_batch.hip):
// the transport of one cell (Sec. 3.2) and one attempt of the subcycled
// thermochemistry (App. A), plus the queue of cells still subcycling.
#pragma once
#include <type_traits>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtm1 {

// --------------------------------------------------------------- transport
template <typename R>
struct U4 {
    R n, fx, fy, fz;
};

template <typename R>
__device__ __forceinline__ U4<R> load_u(const R *__restrict__ N, const R *__restrict__ F, size_t nc, uint32_t i)
{
    U4<R> u;
    u.n = N[i];
    u.fx = F[i];
    u.fy = F[nc + i];
    u.fz = F[2 * nc + i];
    return u;
}

template <typename R>
__device__ __forceinline__ R comp(const U4<R> &u, int d)
{
    return d == 0 ? u.fx : (d == 1 ? u.fy : u.fz);
}

// The six neighbours of a cell (-x,+x,-y,+y,-z,+z) with the ghost cells
// of the boundary conditions: periodic wraps, outflow repeats the cell,
// reflect repeats it with the normal flux component negated (bit d of refl),
// inflow holds a beam entering the grid.
struct Nbr {
    uint32_t idx[6];
    unsigned refl;    // bit f: face f's ghost mirrors the normal flux
    unsigned ghost;   // bit f: face f is a boundary face (outflow, reflect or inflow)
    unsigned inflow;  // bit f: face f's ghost is the entering beam
};

__device__ __forceinline__ void cell_coords(const KGrid &g, uint32_t i, int &ix, int &iy, int &iz)
{
    const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
    iz = (int)(i / nxy);
    const uint32_t r = i - (uint32_t)iz * nxy;
    iy = (int)(r / (uint32_t)g.nx);
    ix = (int)(r - (uint32_t)iy * (uint32_t)g.nx);
}

__device__ __forceinline__ Nbr neighbours(const KGrid &g, uint32_t i, int ix, int iy, int iz)
{
    Nbr nb;
    nb.refl = 0;
    nb.ghost = 0;
    nb.inflow = 0;
    const int c[3] = {ix, iy, iz};
    const int n[3] = {g.nx, g.ny, g.nz};
    const uint32_t stride[3] = {1u, (uint32_t)g.nx, (uint32_t)g.nx * (uint32_t)g.ny};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // low side
        if (c[d] > 0) {
            nb.idx[2 * d] = i - stride[d];
        } else if (g.bc[2 * d] == 0) {
            nb.idx[2 * d] = i + stride[d] * (uint32_t)(n[d] - 1);
        } else {
            nb.idx[2 * d] = i;
            nb.ghost |= 1u << (2 * d);
            if (g.bc[2 * d] == 2) nb.refl |= 1u << (2 * d);
            if (g.bc[2 * d] == 3) nb.inflow |= 1u << (2 * d);
        }
        // high side
        if (c[d] < n[d] - 1) {
            nb.idx[2 * d + 1] = i + stride[d];
        } else if (g.bc[2 * d + 1] == 0) {
            nb.idx[2 * d + 1] = i - stride[d] * (uint32_t)(n[d] - 1);
        } else {
            nb.idx[2 * d + 1] = i;
            nb.ghost |= 1u << (2 * d + 1);
            if (g.bc[2 * d + 1] == 2) nb.refl |= 1u << (2 * d + 1);
            if (g.bc[2 * d + 1] == 3) nb.inflow |= 1u << (2 * d + 1);
        }
    }
    return nb;
}

// physical flux G_d(U) from the pressure components
template <typename R>
__device__ __forceinline__ void flux_of(const U4<R> &u, const R P[6], int d, R G[4])
{
    R px, py, pz;
    prow(P, d, px, py, pz);
    G[0] = comp(u, d);
    G[1] = px;
    G[2] = py;
    G[3] = pz;
}

// intercell flux between L and R along axis d: eq. (glf) or eq. (hll);
// for HLL the wave-speed ranges (lLm, lLp), (lRm, lRp) are in units of c
template <typename R, int FLUX>
__device__ __forceinline__ void face_flux(const U4<R> &L, const R PL[6], R lLm, R lLp, const U4<R> &Rt,
                                          const R PR[6], R lRm, R lRp, int d, R c, R Phi[4])
{
    R GL[4], GR[4];
    flux_of(L, PL, d, GL);
    flux_of(Rt, PR, d, GR);
    const R uL[4] = {L.n, L.fx, L.fy, L.fz};
    const R uR[4] = {Rt.n, Rt.fx, Rt.fy, Rt.fz};
    if (FLUX == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) Phi[m] = R(0.5) * (GL[m] + GR[m]) - R(0.5) * c * (uR[m] - uL[m]);
        return;
    }
    R lp = lLp > lRp ? lLp : lRp;
    lp = (lp > R(0) ? lp : R(0)) * c;
    R lm = lLm < lRm ? lLm : lRm;
    lm = (lm < R(0) ? lm : R(0)) * c;
    const R den = lp - lm;
    if (den == R(0)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) Phi[m] = R(0.5) * (GL[m] + GR[m]);
        return;
    }
    const R iden = rcp(den);
#pragma unroll
    for (int m = 0; m < 4; ++m) Phi[m] = (lp * GL[m] - lm * GR[m] + lp * lm * (uR[m] - uL[m])) * iden;
}

// The ghost state of an inflow face: a beam of photon flux f along the
// inward normal (sgn = +1 on a low face, -1 on a high face), N = f / c.
template <typename R>
__device__ __forceinline__ U4<R> beam(double f, int d, double sgn, R c)
{
    U4<R> u;
    u.n = (R)(f / (double)c);
    const R fd = (R)(sgn * f);
    u.fx = d == 0 ? fd : R(0);
    u.fy = d == 1 ? fd : R(0);
    u.fz = d == 2 ? fd : R(0);
    return u;
}

// Transport of group grp of one cell: every face flux from the source
// arrays (N, F of this group),
//   U' = U + dt/dx * sum_d (Phi_{d,-1/2} - Phi_{d,+1/2})     (eq. dUdt_sol)
// bout receives the photon-density flux out of the grid through the cell's
// boundary faces (high faces count +Phi_N, low faces -Phi_N).
template <typename R, int FLUX>
__device__ __forceinline__ U4<R> transport_cell(const Nbr &nb, uint32_t i, size_t nc, const R *__restrict__ N,
                                                const R *__restrict__ F, R c, R kdx, const R *__restrict__ tab,
                                                int nf, int nth, double &bout, const KGrid &g, int grp)
{
    const U4<R> C = load_u(N, F, nc, i);
    R PC[6];
    m1_pressure(C.n, C.fx, C.fy, C.fz, c, PC);
    R acc[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        U4<R> L = load_u(N, F, nc, nb.idx[2 * d]);
        U4<R> Rt = load_u(N, F, nc, nb.idx[2 * d + 1]);
        if (nb.refl & (1u << (2 * d))) {
            if (d == 0) L.fx = -L.fx;
            else if (d == 1) L.fy = -L.fy;
            else L.fz = -L.fz;
        }
        if (nb.refl & (1u << (2 * d + 1))) {
            if (d == 0) Rt.fx = -Rt.fx;
            else if (d == 1) Rt.fy = -Rt.fy;
            else Rt.fz = -Rt.fz;
        }
        if (nb.inflow & (1u << (2 * d))) L = beam<R>(g.inflow[2 * d][grp], d, 1.0, c);
        if (nb.inflow & (1u << (2 * d + 1))) Rt = beam<R>(g.inflow[2 * d + 1][grp], d, -1.0, c);
        R PL[6], PR[6], Pm[4], Pp[4];
        m1_pressure(L.n, L.fx, L.fy, L.fz, c, PL);
        m1_pressure(Rt.n, Rt.fx, Rt.fy, Rt.fz, c, PR);
        R lLm = 0, lLp = 0, lCm = 0, lCp = 0, lRm = 0, lRp = 0;
        if (FLUX == 1) {
            hll_speeds(tab, nf, nth, L.n, L.fx, L.fy, L.fz, d, c, lLm, lLp);
            hll_speeds(tab, nf, nth, C.n, C.fx, C.fy, C.fz, d, c, lCm, lCp);
            hll_speeds(tab, nf, nth, Rt.n, Rt.fx, Rt.fy, Rt.fz, d, c, lRm, lRp);
        }
        face_flux<R, FLUX>(L, PL, lLm, lLp, C, PC, lCm, lCp, d, c, Pm);
        face_flux<R, FLUX>(C, PC, lCm, lCp, Rt, PR, lRm, lRp, d, c, Pp);
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] += Pm[m] - Pp[m];
        if (nb.ghost & (1u << (2 * d))) bout -= (double)Pm[0];
        if (nb.ghost & (1u << (2 * d + 1))) bout += (double)Pp[0];
    }
    U4<R> o;
    o.n = C.n + kdx * acc[0];
    o.fx = C.fx + kdx * acc[1];
    o.fy = C.fy + kdx * acc[2];
    o.fz = C.fz + kdx * acc[3];
    if (FLUX == 1) limit_flux(o.n, o.fx, o.fy, o.fz, c);
    return o;
}

// --------------------------------------------------------- thermochemistry
__device__ __forceinline__ double mu_of(const KChem &k, double x, double y2, double y3)
{
    return rcp_pos(k.X * (1.0 + x) + 0.25 * k.Y * (1.0 + y2 + 2.0 * y3));
}

// |a - b| > f b for b > 0: the relative-change test of App. A without a division
__device__ __forceinline__ bool rel_above(double a, double b, double f) { return fabs(a - b) > f * b; }

// Thermochemical state of one cell during its subcycling over dt_RT.  The
// flux of a group only scales with the absorption factor of each accepted
// substep, so the state carries that product (fs) and the flux itself stays
// in the destination arrays until the cell has finished.
struct CS {
    double N[3], fs[3];
    double x, y2, y3, Tmu;
    double rem, h;  // time left in dt_RT, length of the next substep
    int acc, att;   // accepted substeps, attempts
};

// Smoothed RT (Sec. 4.4): the cell starts from its photon density before
// injection and transport, and their change over dt_RT enters every substep
// as the constant rate Nr (eqs. thchem_N_smooth, smoothrate1).  The flux
// obeys the same linear update with the rate (F' - F^t)/dt_RT (eqs.
// thchem_F_smooth, smoothrate2), so after the accepted substeps h_k with
// absorption factors r_k = 1/(1 + h_k D_k) it is fs F^t + fb (F' - F^t)/dt_RT
// with fs = prod r_k and fb <- (fb + h_k) r_k; the state carries fb.
struct CSR : CS {
    double Nr[3], fb[3];
};

// Every chemistry kernel runs the attempt with three groups; groups a grid
// does not have carry zero photons and zero cross sections, which leaves
// every sum and check exactly as with fewer groups.  One instantiation for
// all kernels keeps their arithmetic identical, so that a cell's result does
// not depend on which kernel (first pass, queue, batch, tape) finishes it.
constexpr int CM = 3;

// Per-cell constants of the chemistry: n_H, n_He, the factor K of the
// T_mu equation (eq. ramsesrt_cool1_eq) and the fixed temperature of
// isothermal runs.
struct CC {
    double nH, nHe, K, Tiso;
};

__device__ __forceinline__ CC make_cc(const KChem &k, double nH, double T)
{
    CC c;
    c.nH = nH;
    c.nHe = nH * k.Y / (4.0 * k.X);
    c.K = k.Kfac / nH;
    c.Tiso = T;
    return c;
}

// Returns false (and leaves the cell untouched) when an input is not finite;
// fin says whether the cell's fluxes are finite.
// Method variant of the chemistry kernels: bit 0 smoothed RT (Sec. 4.4),
// bit 1 no on-the-spot approximation (Sec. 3.3.2: case A rates and the
// photons of recombinations to the ground state).
constexpr int V_SMOOTH = 1;
constexpr int V_CASE_A = 2;

template <int M, int V = 0, class St>
__device__ __forceinline__ bool chem_init(const KChem &k, double dt, double T, bool fin, St &s)
{
    constexpr bool SM = (V & V_SMOOTH) != 0;
    bool ok = fin && isfinite(T) && isfinite(s.x) && isfinite(s.y2) && isfinite(s.y3);
#pragma unroll
    for (int g = 0; g < M; ++g) {
        ok = ok && isfinite(s.N[g]);
        s.fs[g] = 1.0;
        if constexpr (SM) {
            ok = ok && isfinite(s.Nr[g]);
            s.fb[g] = 0.0;
        }
    }
    s.Tmu = T / mu_of(k, s.x, s.y2, s.y3);
    s.rem = ok ? dt : 0.0;
    s.h = dt;
    s.acc = 0;
    s.att = 0;
    return ok;
}

// One attempt of a substep of length h (App. A tasks 1-5).  On a failed
// 10% check the state is unchanged and h is halved; on success the state
// advances by h, and the next h doubles when every relative change was
// below 5%.  Returns true when the cell has filled dt_RT (or reached the
// attempt cap, flag bit 0).  With RETRY, attempts that fail the photon check
// (the first stage, which depends only on the state and h) are repeated
// with the halved h inside the call before the gas stages run: each still
// counts as an attempt, and the sequence of attempts is the same, but a
// lane that would sit out the rest of a failed attempt goes on at once.
template <int M, int V = 0, bool RETRY = true, class St>
__device__ __forceinline__ bool chem_attempt(const KChem &k, const CC &cc, St &s, unsigned &flags)
{
    constexpr bool SM = (V & V_SMOOTH) != 0;
    constexpr bool CA = (V & V_CASE_A) != 0;
    if (s.att >= k.max_att) {
        flags |= 1u;
        return true;
    }
    ++s.att;
    const bool iso = k.isothermal != 0;
    const double nH = cc.nH, nHe = cc.nHe, K = cc.K;
    double h = s.h;
    if (h >= s.rem * (1.0 - 1e-10)) h = s.rem;
    const double x = s.x, y2 = s.y2, y3 = s.y3, Tmu = s.Tmu;
    bool small = true;  // every relative change below 5%
    // ---- photons: semi-implicit absorption with backward abundances
    const double nHI = (1.0 - x) * nH;
    const double nHeI = (1.0 - y2 - y3) * nHe;
    const double nHeII = y2 * nHe;
    const double nHII = x * nH;
    const double nHeIII = y3 * nHe;
    double Nn[M], rd[M], D[M];
    // without OTSA: photons of recombinations straight to the ground state,
    // (alpha_A - alpha_B) n_j n_e with the state at the start of the
    // substep, into the group that holds species j's threshold (eq. cool_N_cr)
    double Crec[M];
    if constexpr (CA) {
        const Tq qc = make_Tq(iso ? cc.Tiso : Tmu * mu_of(k, x, y2, y3));
        const double ne = nHII + (y2 + 2.0 * y3) * nHe;
        const double em0 = (alphaA_HII(qc).v - alphaB_HII(qc).v) * nHII * ne;
        const double em1 = (alphaA_HeII(qc).v - alphaB_HeII(qc).v) * nHeII * ne;
        const double em2 = (alphaA_HeIII(qc).v - alphaB_HeIII(qc).v) * nHeIII * ne;
#pragma unroll
        for (int g = 0; g < M; ++g) Crec[g] = k.brec[g][0] * em0 + k.brec[g][1] * em1 + k.brec[g][2] * em2;
    }
#pragma unroll
    for (int g = 0; g < M; ++g) D[g] = k.csN[g][0] * nHI + k.csN[g][1] * nHeI + k.csN[g][2] * nHeII;
    for (;;) {
        bool fail = false;
        if constexpr (M == 3) {
            // the three absorption factors 1/(1 + h D_g) from one division
            const double a0 = 1.0 + h * D[0], a1 = 1.0 + h * D[1], a2 = 1.0 + h * D[2];
            const double a12 = a1 * a2;
            const double ia = 1.0 / (a0 * a12);
            rd[0] = ia * a12;
            rd[1] = ia * (a0 * a2);
            rd[2] = ia * (a0 * a1);
        } else {
#pragma unroll
            for (int g = 0; g < M; ++g) rd[g] = 1.0 / (1.0 + h * D[g]);
        }
#pragma unroll
        for (int g = 0; g < M; ++g) {
            if constexpr (SM) {
                // a negative rate may take the update below zero: it stops there
                const double src = CA ? Crec[g] + s.Nr[g] : s.Nr[g];
                const double nn = (s.N[g] + h * src) * rd[g];
                Nn[g] = nn < 0.0 ? 0.0 : nn;
            } else if constexpr (CA) {
                Nn[g] = (s.N[g] + h * Crec[g]) * rd[g];
            } else
                Nn[g] = s.N[g] * rd[g];
            if (s.N[g] > k.N_floor) {
                fail |= rel_above(Nn[g], s.N[g], 0.1);
                small &= fabs(Nn[g] - s.N[g]) < 0.05 * s.N[g];
            }
        }
        if (!fail) break;
        s.h = 0.5 * h;
        if (!RETRY) return false;
        // the next attempt, from its start
        if (s.att >= k.max_att) {
            flags |= 1u;
            return true;
        }
        ++s.att;
        h = s.h;
        if (h >= s.rem * (1.0 - 1e-10)) h = s.rem;
        small = true;
    }
    const double mu0 = mu_of(k, x, y2, y3);
    const double ne0 = nHII + (y2 + 2.0 * y3) * nHe;
    // ---- thermal update in T_mu = T/mu
    double Tmun = Tmu;
    if (!iso) {
        const Tq q0 = make_Tq(Tmu * mu0);
        double H = 0.0;
        {
            const double nj[3] = {nHI, nHeI, nHeII};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double sj = 0.0;
#pragma unroll
                for (int g = 0; g < M; ++g) sj += Nn[g] * k.hc[g][j];
                H += nj[j] * sj;
            }
        }
        double L, dL;
        cooling<CA>(q0, k.a_exp, ne0, nHI, nHII, nHeI, nHeII, nHeIII, L, dL);
        const double Lam = H - L;
        const double Lamp = -mu0 * dL;
        const double den = 1.0 - Lamp * K * h;
        if (!(den > 0.0)) {
            s.h = 0.5 * h;
            return false;
        }
        Tmun = Tmu + Lam * K * h / den;
        if (rel_above(Tmun, Tmu, 0.1) || fabs(K * Lam * h) > 0.1 * Tmu) {
            s.h = 0.5 * h;
            return false;
        }
        small &= fabs(Tmun - Tmu) < 0.05 * Tmu;
    }
    // ---- hydrogen: semi-implicit in x_HII
    double GHI = 0.0, GHeI = 0.0, GHeII = 0.0;
#pragma unroll
    for (int g = 0; g < M; ++g) {
        GHI += k.csN[g][0] * Nn[g];
        GHeI += k.csN[g][1] * Nn[g];
        GHeII += k.csN[g][2] * Nn[g];
    }
    const Tq q1 = make_Tq(iso ? cc.Tiso : Tmun * mu0);
    const vd bH = beta_HI(q1);
    const vd aH = alpha_HII<CA>(q1);
    const double Cr = bH.v * ne0 + GHI;
    const double Dr = aH.v * ne0;
    double dC, dD;
    if (iso) {
        dC = nH * bH.v;
        dD = nH * aH.v;
    } else {
        const double f = ne0 * Tmun * mu0 * mu0 * k.X;
        dC = nH * bH.v - f * bH.d;
        dD = nH * aH.v - f * aH.d;
    }
    const double J = dC - (Cr + Dr) - x * (dC + dD);
    const double denx = 1.0 - J * h;
    if (!(denx > 0.0)) {
        s.h = 0.5 * h;
        return false;
    }
    const double rate = Cr - x * (Cr + Dr);
    double xn = x + h * rate / denx;
    xn = xn < k.x_min ? k.x_min : (xn > 1.0 ? 1.0 : xn);
    if (rel_above(xn, x, 0.1) || fabs(rate) * h > 0.1 * x) {
        s.h = 0.5 * h;
        return false;
    }
    small &= fabs(xn - x) < 0.05 * x;
    // ---- helium: HeI, HeII, HeIII in order, then He conservation
    double y2n = y2, y3n = y3;
    if (nHe > 0.0) {
        const double ne1 = xn * nH + (y2 + 2.0 * y3) * nHe;
        const Tq q2 = make_Tq(iso ? cc.Tiso : Tmun * mu_of(k, xn, y2, y3));
        const vd bHe1 = beta_HeI(q2), aHe2 = alpha_HeII<CA>(q2), bHe2 = beta_HeII(q2), aHe3 = alpha_HeIII<CA>(q2);
        const double y1 = 1.0 - y2 - y3;
        const double y1n = div_pos(y1 + y2 * aHe2.v * ne1 * h, 1.0 + (bHe1.v * ne1 + GHeI) * h);
        y2n = div_pos(y2 + (y1n * (bHe1.v * ne1 + GHeI) + y3 * aHe3.v * ne1) * h,
                      1.0 + ((bHe2.v + aHe2.v) * ne1 + GHeII) * h);
        const double ne2 = xn * nH + (y2n + 2.0 * y3) * nHe;
        const Tq q3 = make_Tq(iso ? cc.Tiso : Tmun * mu_of(k, xn, y2n, y3));
        const vd bHe2b = beta_HeII(q3), aHe3b = alpha_HeIII<CA>(q3);
        y3n = div_pos(y3 + y2n * (bHe2b.v * ne2 + GHeII) * h, 1.0 + aHe3b.v * ne2 * h);
        const double S = y1n + y2n + y3n;
        if (!(y1n >= y2n && y1n >= y3n)) {
            if (y2n >= y3n) y2n -= (S - 1.0);
            else y3n -= (S - 1.0);
        }
    }
    // ---- electron density check
    const double nen = xn * nH + (y2n + 2.0 * y3n) * nHe;
    if (rel_above(nen, ne0, 0.1)) {
        s.h = 0.5 * h;
        return false;
    }
    small &= fabs(nen - ne0) < 0.05 * ne0;
    // ---- accept
#pragma unroll
    for (int g = 0; g < M; ++g) {
        s.N[g] = Nn[g];
        s.fs[g] *= rd[g];
        if constexpr (SM) s.fb[g] = (s.fb[g] + h) * rd[g];
    }
    s.x = xn;
    s.y2 = y2n;
    s.y3 = y3n;
    s.Tmu = iso ? cc.Tiso / mu_of(k, xn, y2n, y3n) : Tmun;
    s.rem -= h;
    ++s.acc;
    s.h = small ? 2.0 * h : h;
    return !(s.rem > 0.0);
}

template <int M, class S>
__device__ __forceinline__ double chem_finish(const KChem &k, const CC &cc, const S &s, unsigned &flags)
{
    const double T = k.isothermal ? cc.Tiso : s.Tmu * mu_of(k, s.x, s.y2, s.y3);
#pragma unroll
    for (int g = 0; g < M; ++g) {
        if (s.N[g] < 0.0) flags |= 8u;
        if (!isfinite(s.N[g])) flags |= 2u;
    }
    if (!isfinite(T) || !isfinite(s.x)) flags |= 2u;
    return T;
}

// Queue of cells still subcycling after the head pass (structure of arrays
// in caller scratch): the cell index, the attempt counters, and the partial
// state {N[3], fs[3], x_HII, x_HeII, x_HeIII, T_mu, rem, h}; the grid's queue
// adds the inputs of the cell constants {n_H, T at the start of the step}
// (so that a refill does not wait on a load that depends on the cell
// index), and with smoothed RT {Nr[3], fb[3]}.
constexpr int QV = 12;
constexpr int QV_CC = QV;
constexpr int QV_GRID = QV + 2;

// a queued cell that took at least this many attempts in the previous pass
// goes to the tail's first region
#ifndef RT_TAIL_LONG_ATTEMPTS
#define RT_TAIL_LONG_ATTEMPTS 48
#endif
constexpr int TAIL_LONG_ATTEMPTS = RT_TAIL_LONG_ATTEMPTS;
constexpr int QV_SMOOTH = QV_GRID + 6;

// queue positions a tail wave reserves at a time (at least the lanes that
// need a cell): most refills then take no atomic on the shared counter.  One
// wave's width: the first reservation gives every lane a cell, and a wave
// never holds a second of the long chains at the queue's front in reserve.
#ifndef RT_TAIL_CHUNK
#define RT_TAIL_CHUNK 64
#endif
constexpr unsigned TAIL_CHUNK = RT_TAIL_CHUNK;
// the most positions a wave of the one-pass chemistry reserves at a time
// once past the long chains (measured at 256^3 x 3: 64 -> 4.73 ms, 128 ->
// 4.30, 256 -> 4.27, 512 -> 4.29, 1024 -> 5.54 ms, the last from the
// imbalance at the end); smaller grids take less (chem_sweep_chunk)
#ifndef RT_CHEM_SWEEP_CHUNK
#define RT_CHEM_SWEEP_CHUNK 256
#endif
constexpr unsigned CHEM_SWEEP_CHUNK = RT_CHEM_SWEEP_CHUNK;

__device__ __forceinline__ void q_store_rates(const QueueView &q, uint32_t p, const CS &) {}
__device__ __forceinline__ void q_store_rates(const QueueView &q, uint32_t p, const CSR &s)
{
    double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        v[(size_t)(QV_GRID + g) * c] = s.Nr[g];
        v[(size_t)(QV_GRID + 3 + g) * c] = s.fb[g];
    }
}
__device__ __forceinline__ void q_load_rates(const QueueView &q, uint32_t p, CS &) {}
__device__ __forceinline__ void q_load_rates(const QueueView &q, uint32_t p, CSR &s)
{
    const double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        s.Nr[g] = v[(size_t)(QV_GRID + g) * c];
        s.fb[g] = v[(size_t)(QV_GRID + 3 + g) * c];
    }
}

template <class S>
__device__ __forceinline__ void q_store(const QueueView &q, uint32_t p, uint32_t cell, const S &s, const CC &cc)
{
    q.cell[p] = (int32_t)cell;
    q.acc[p] = s.acc;
    q.att[p] = s.att;
    double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        v[(size_t)g * c] = s.N[g];
        v[(size_t)(3 + g) * c] = s.fs[g];
    }
    v[6 * c] = s.x;
    v[7 * c] = s.y2;
    v[8 * c] = s.y3;
    v[9 * c] = s.Tmu;
    v[10 * c] = s.rem;
    v[11 * c] = s.h;
    v[(size_t)QV_CC * c] = cc.nH;
    v[(size_t)(QV_CC + 1) * c] = cc.Tiso;
    q_store_rates(q, p, s);
}

template <class S>
__device__ __forceinline__ uint32_t q_load(const KChem &k, const QueueView &q, uint32_t p, S &s, CC &cc)
{
    s.acc = q.acc[p];
    s.att = q.att[p];
    const double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        s.N[g] = v[(size_t)g * c];
        s.fs[g] = v[(size_t)(3 + g) * c];
    }
    s.x = v[6 * c];
    s.y2 = v[7 * c];
    s.y3 = v[8 * c];
    s.Tmu = v[9 * c];
    s.rem = v[10 * c];
    s.h = v[11 * c];
    cc = make_cc(k, v[(size_t)QV_CC * c], v[(size_t)(QV_CC + 1) * c]);
    q_load_rates(q, p, s);
    return (uint32_t)q.cell[p];
}

// Flux of group g of a finished cell from the transported flux fp in the
// destination (and, smoothed, the pre-step flux ft of the source set).
template <typename R>
__device__ __forceinline__ R finish_flux(const ChemIO<R> &io, const CS &s, int g, R fp, R ft)
{
    return (R)((double)fp * s.fs[g]);
}
template <typename R>
__device__ __forceinline__ R finish_flux(const ChemIO<R> &io, const CSR &s, int g, R fp, R ftr)
{
    // a cell that accepted no substep keeps its pre-step state
    const double ft = (double)ftr;
    if (s.acc == 0) return (R)ft;
    return (R)(s.fs[g] * ft + s.fb[g] * (((double)fp - ft) / io.sm.dt));
}

// The previous-pass attempt count kept per cell: the count, capped at 127,
// in bits 0-6; bit 7 marks a cell the chemistry pass takes from its list of
// long chains (it is then passed over in the sweep over all cells).
constexpr uint8_t ATT_MASK = 0x7F, ATT_LISTED = 0x80;

// Write a finished cell: N, the flux in the destination scaled by fs (with
// smoothed RT: fs F^t + fb (F' - F^t)/dt_RT), the gas state and the counters.
// The destination fluxes (fp) are in hand before anything is written, given
// by the caller (LOADED) or loaded first: a load issued after a store waits
// for that store (one counter tracks both), so loads placed between the
// stores would each wait out the stores before them.
template <typename R, int M, bool LOADED, class S>
__device__ __forceinline__ void store_cell_impl(const ChemIO<R> &io, uint32_t i, const S &s, double T,
                                                const R *fpin, uint8_t mark)
{
    constexpr bool SM = std::is_same<S, CSR>::value;
    const size_t nc = io.ncell;
    R fp[3 * M], ft[3 * M];
#pragma unroll
    for (int j = 0; j < 3 * M; ++j) {
        if constexpr (LOADED) fp[j] = fpin[j];
        else fp[j] = io.F[(size_t)j * nc + i];
        if constexpr (SM) ft[j] = io.sm.F[(size_t)j * nc + i];
        else ft[j] = fp[j];
    }
#pragma unroll
    for (int g = 0; g < M; ++g) io.N[(size_t)g * nc + i] = (R)(s.N[g] * io.a3);
    io.xHII[i] = s.x;
    io.xHeII[i] = s.y2;
    io.xHeIII[i] = s.y3;
    io.T[i] = T;
    if (io.nacc) io.nacc[i] = s.acc;
    if (io.natt) io.natt[i] = s.att;
    if (io.prev_att) io.prev_att[i] = (uint8_t)(mark | (s.att < (int)ATT_MASK ? s.att : (int)ATT_MASK));
#pragma unroll
    for (int g = 0; g < M; ++g)
#pragma unroll
        for (int d = 0; d < 3; ++d) io.F[(size_t)(3 * g + d) * nc + i] = finish_flux(io, s, g, fp[3 * g + d], ft[3 * g + d]);
}

template <typename R, int M, class S>
__device__ __forceinline__ void store_cell(const ChemIO<R> &io, uint32_t i, const S &s, double T, uint8_t mark = 0)
{
    store_cell_impl<R, M, false>(io, i, s, T, nullptr, mark);
}

// the same with the destination fluxes loaded by the caller
template <typename R, int M, class S>
__device__ __forceinline__ void store_cell_with(const ChemIO<R> &io, uint32_t i, const S &s, double T, const R *fp,
                                                uint8_t mark = 0)
{
    store_cell_impl<R, M, true>(io, i, s, T, fp, mark);
}

}  // namespace rtm1
