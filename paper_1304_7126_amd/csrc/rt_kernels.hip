// rt_kernels.hip -- gfx950 kernels of the explicit M1 RT step.
//
//   k_inject     point-source injection (Sec. 3.1)
//   k_transport  unsplit GLF/HLL update of (N, F), all groups (Sec. 3.2)
//   k_head       per-cell thermochemistry in FP64 (App. A), up to K attempts
//                per cell; with FUSE the cell is transported first, so one
//                pass reads the source set and writes the destination set
//   k_tail       the cells still subcycling after the head pass, compacted
//                into a queue and worked off by lanes that refill themselves
//   k_reduce_*   photon budget and diagnostics (fixed-order tree sums)
//
// Radiation arrays are structure-of-arrays, x fastest, one plane of ncell
// values per group and component, so a wavefront reads 64 consecutive cells
// of one component with one coalesced access.
#include "rt_device.h"
#include "rt_internal.h"

namespace rtm1 {

// ------------------------------------------------------------------ inject
template <typename R>
__global__ void k_inject(R *__restrict__ N, size_t ncell, int M, int nsrc, const int32_t *__restrict__ cell,
                         const double *__restrict__ rate, double dtV)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    const size_t i = (size_t)cell[s];
    for (int g = 0; g < M; ++g) {
        R *p = N + (size_t)g * ncell + i;
        *p = R((double)*p + rate[(size_t)s * M + g] * dtV);
    }
}

hipError_t launch_inject(bool fp32, void *N, size_t ncell, int M, int nsrc, const int32_t *cell,
                         const double *rate, double dt_over_V, hipStream_t s)
{
    if (nsrc <= 0) return hipSuccess;
    dim3 b(64), gr((nsrc + 63) / 64);
    if (fp32)
        hipLaunchKernelGGL(k_inject<float>, gr, b, 0, s, (float *)N, ncell, M, nsrc, cell, rate, dt_over_V);
    else
        hipLaunchKernelGGL(k_inject<double>, gr, b, 0, s, (double *)N, ncell, M, nsrc, cell, rate, dt_over_V);
    return hipGetLastError();
}

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
// reflect repeats it with the normal flux component negated (bit d of refl).
struct Nbr {
    uint32_t idx[6];
    unsigned refl;
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
            if (g.bc[2 * d] == 2) nb.refl |= 1u << (2 * d);
        }
        // high side
        if (c[d] < n[d] - 1) {
            nb.idx[2 * d + 1] = i + stride[d];
        } else if (g.bc[2 * d + 1] == 0) {
            nb.idx[2 * d + 1] = i - stride[d] * (uint32_t)(n[d] - 1);
        } else {
            nb.idx[2 * d + 1] = i;
            if (g.bc[2 * d + 1] == 2) nb.refl |= 1u << (2 * d + 1);
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

// Transport of one group of one cell: every face flux from the source
// arrays (N, F of this group),
//   U' = U + dt/dx * sum_d (Phi_{d,-1/2} - Phi_{d,+1/2})     (eq. dUdt_sol)
template <typename R, int FLUX>
__device__ __forceinline__ U4<R> transport_cell(const Nbr &nb, uint32_t i, size_t nc, const R *__restrict__ N,
                                                const R *__restrict__ F, R c, R kdx, const R *__restrict__ tab,
                                                int nf, int nth)
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
        R PL[6], PR[6], Pm[4], Pp[4];
        m1_pressure(L.n, L.fx, L.fy, L.fz, c, PL);
        m1_pressure(Rt.n, Rt.fx, Rt.fy, Rt.fz, c, PR);
        R lLm = 0, lLp = 0, lCm = 0, lCp = 0, lRm = 0, lRp = 0;
        if (FLUX == 1) {
            hll_speeds(tab, nf, nth, L.n, L.fx, L.fy, L.fz, comp(L, d), c, lLm, lLp);
            hll_speeds(tab, nf, nth, C.n, C.fx, C.fy, C.fz, comp(C, d), c, lCm, lCp);
            hll_speeds(tab, nf, nth, Rt.n, Rt.fx, Rt.fy, Rt.fz, comp(Rt, d), c, lRm, lRp);
        }
        face_flux<R, FLUX>(L, PL, lLm, lLp, C, PC, lCm, lCp, d, c, Pm);
        face_flux<R, FLUX>(C, PC, lCm, lCp, Rt, PR, lRm, lRp, d, c, Pp);
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] += Pm[m] - Pp[m];
    }
    U4<R> o;
    o.n = C.n + kdx * acc[0];
    o.fx = C.fx + kdx * acc[1];
    o.fy = C.fy + kdx * acc[2];
    o.fz = C.fz + kdx * acc[3];
    return o;
}

template <typename R, int FLUX>
__global__ __launch_bounds__(256) void k_transport(KGrid g, int M, R c, R kdx, const R *__restrict__ Nin,
                                                   const R *__restrict__ Fin, R *__restrict__ Nout,
                                                   R *__restrict__ Fout, const R *__restrict__ tab, int nf,
                                                   int nth)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)g.ncell) return;
    const size_t nc = g.ncell;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    const Nbr nb = neighbours(g, i, ix, iy, iz);
    for (int grp = 0; grp < M; ++grp) {
        const U4<R> o = transport_cell<R, FLUX>(nb, i, nc, Nin + (size_t)grp * nc, Fin + (size_t)3 * grp * nc, c,
                                                kdx, tab, nf, nth);
        Nout[(size_t)grp * nc + i] = o.n;
        R *Fo = Fout + (size_t)3 * grp * nc;
        Fo[i] = o.fx;
        Fo[nc + i] = o.fy;
        Fo[2 * nc + i] = o.fz;
    }
}

hipError_t launch_transport(bool fp32, int flux, const KGrid &g, int M, double c, double dt, const void *Nin,
                            const void *Fin, void *Nout, void *Fout, const void *hll, int nf, int nth,
                            hipStream_t s)
{
    dim3 b(256), gr((unsigned)((g.ncell + 255) / 256));
    const double k = dt / g.dx;
    if (fp32) {
        auto kern = flux ? k_transport<float, 1> : k_transport<float, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, M, (float)c, (float)k, (const float *)Nin, (const float *)Fin,
                           (float *)Nout, (float *)Fout, (const float *)hll, nf, nth);
    } else {
        auto kern = flux ? k_transport<double, 1> : k_transport<double, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, M, c, k, (const double *)Nin, (const double *)Fin,
                           (double *)Nout, (double *)Fout, (const double *)hll, nf, nth);
    }
    return hipGetLastError();
}

// --------------------------------------------------------- thermochemistry
__device__ __forceinline__ double mu_of(const KChem &k, double x, double y2, double y3)
{
    return 1.0 / (k.X * (1.0 + x) + 0.25 * k.Y * (1.0 + y2 + 2.0 * y3));
}

__device__ __forceinline__ double rel_change(double a, double b) { return fabs(a - b) / b; }

// Thermochemical state of one cell during its subcycling over dt_RT.
struct CS {
    double N[3], F[3][3];
    double x, y2, y3, Tmu;
    double rem, h;  // time left in dt_RT, length of the next substep
    int acc, att;   // accepted substeps, attempts
};

// Returns false (and leaves the cell untouched) when an input is not finite.
template <int M>
__device__ __forceinline__ bool chem_init(const KChem &k, double dt, double T, CS &s)
{
    bool ok = isfinite(T) && isfinite(s.x) && isfinite(s.y2) && isfinite(s.y3);
#pragma unroll
    for (int g = 0; g < M; ++g)
        ok = ok && isfinite(s.N[g]) && isfinite(s.F[g][0]) && isfinite(s.F[g][1]) && isfinite(s.F[g][2]);
    s.Tmu = T / mu_of(k, s.x, s.y2, s.y3);
    s.rem = ok ? dt : 0.0;
    s.h = dt;
    s.acc = 0;
    s.att = 0;
    return ok;
}

// One attempt of a substep of length h (App. A tasks 1-5).  On a failed
// 10% check the state is unchanged and h is halved; on success the state
// advances by h, and the next h doubles when the largest relative change
// was below 5%.  Returns true when the cell has filled dt_RT (or reached
// the attempt cap, flag bit 0).
template <int M>
__device__ __forceinline__ bool chem_attempt(const KChem &k, double nH, double Tiso, CS &s, unsigned &flags)
{
    if (s.att >= k.max_att) {
        flags |= 1u;
        return true;
    }
    ++s.att;
    const bool iso = k.isothermal != 0;
    const double nHe = nH * k.Y / (4.0 * k.X);
    const double K = k.Kfac / nH;
    double h = s.h;
    if (h >= s.rem * (1.0 - 1e-10)) h = s.rem;
    const double x = s.x, y2 = s.y2, y3 = s.y3, Tmu = s.Tmu;
    double maxrel = 0.0, r;
    // ---- photons: semi-implicit absorption with backward abundances
    const double nHI = (1.0 - x) * nH;
    const double nHeI = (1.0 - y2 - y3) * nHe;
    const double nHeII = y2 * nHe;
    const double nHII = x * nH;
    const double nHeIII = y3 * nHe;
    double Nn[M], Fn[M][3];
    bool fail = false;
#pragma unroll
    for (int g = 0; g < M; ++g) {
        const double D = k.cr * (k.sN[g][0] * nHI + k.sN[g][1] * nHeI + k.sN[g][2] * nHeII);
        const double rden = 1.0 / (1.0 + h * D);
        Nn[g] = s.N[g] * rden;
        Fn[g][0] = s.F[g][0] * rden;
        Fn[g][1] = s.F[g][1] * rden;
        Fn[g][2] = s.F[g][2] * rden;
        r = s.N[g] > k.N_floor ? rel_change(Nn[g], s.N[g]) : 0.0;
        fail |= r > 0.1;
        maxrel = r > maxrel ? r : maxrel;
    }
    if (fail) {
        s.h = 0.5 * h;
        return false;
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
            const double ej[3] = {EPS_HI, EPS_HEI, EPS_HEII};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double sj = 0.0;
#pragma unroll
                for (int g = 0; g < M; ++g) sj += k.cr * Nn[g] * (k.eb[g] * k.sE[g][j] - ej[j] * k.sN[g][j]);
                H += nj[j] * sj;
            }
        }
        double L, dL;
        cooling_B(q0, k.a_exp, ne0, nHI, nHII, nHeI, nHeII, nHeIII, L, dL);
        const double Lam = H - L;
        const double Lamp = -mu0 * dL;
        const double den = 1.0 - Lamp * K * h;
        if (!(den > 0.0)) {
            s.h = 0.5 * h;
            return false;
        }
        Tmun = Tmu + Lam * K * h / den;
        r = rel_change(Tmun, Tmu);
        if (r > 0.1 || fabs(K * Lam * h) / Tmu > 0.1) {
            s.h = 0.5 * h;
            return false;
        }
        maxrel = r > maxrel ? r : maxrel;
    }
    // ---- hydrogen: semi-implicit in x_HII
    double GHI = 0.0, GHeI = 0.0, GHeII = 0.0;
#pragma unroll
    for (int g = 0; g < M; ++g) {
        GHI += k.sN[g][0] * k.cr * Nn[g];
        GHeI += k.sN[g][1] * k.cr * Nn[g];
        GHeII += k.sN[g][2] * k.cr * Nn[g];
    }
    const Tq q1 = make_Tq(iso ? Tiso : Tmun * mu0);
    const vd bH = beta_HI(q1);
    const vd aH = alphaB_HII(q1);
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
    r = rel_change(xn, x);
    if (r > 0.1 || fabs(rate) * h / x > 0.1) {
        s.h = 0.5 * h;
        return false;
    }
    maxrel = r > maxrel ? r : maxrel;
    // ---- helium: HeI, HeII, HeIII in order, then He conservation
    double y2n = y2, y3n = y3;
    if (nHe > 0.0) {
        const double ne1 = xn * nH + (y2 + 2.0 * y3) * nHe;
        const Tq q2 = make_Tq(iso ? Tiso : Tmun * mu_of(k, xn, y2, y3));
        const vd bHe1 = beta_HeI(q2), aHe2 = alphaB_HeII(q2), bHe2 = beta_HeII(q2), aHe3 = alphaB_HeIII(q2);
        const double y1 = 1.0 - y2 - y3;
        const double y1n = (y1 + y2 * aHe2.v * ne1 * h) / (1.0 + (bHe1.v * ne1 + GHeI) * h);
        y2n = (y2 + (y1n * (bHe1.v * ne1 + GHeI) + y3 * aHe3.v * ne1) * h) /
              (1.0 + ((bHe2.v + aHe2.v) * ne1 + GHeII) * h);
        const double ne2 = xn * nH + (y2n + 2.0 * y3) * nHe;
        const Tq q3 = make_Tq(iso ? Tiso : Tmun * mu_of(k, xn, y2n, y3));
        const vd bHe2b = beta_HeII(q3), aHe3b = alphaB_HeIII(q3);
        y3n = (y3 + y2n * (bHe2b.v * ne2 + GHeII) * h) / (1.0 + aHe3b.v * ne2 * h);
        const double S = y1n + y2n + y3n;
        if (!(y1n >= y2n && y1n >= y3n)) {
            if (y2n >= y3n) y2n -= (S - 1.0);
            else y3n -= (S - 1.0);
        }
    }
    // ---- electron density check
    const double nen = xn * nH + (y2n + 2.0 * y3n) * nHe;
    r = rel_change(nen, ne0);
    if (r > 0.1) {
        s.h = 0.5 * h;
        return false;
    }
    maxrel = r > maxrel ? r : maxrel;
    // ---- accept
#pragma unroll
    for (int g = 0; g < M; ++g) {
        s.N[g] = Nn[g];
        s.F[g][0] = Fn[g][0];
        s.F[g][1] = Fn[g][1];
        s.F[g][2] = Fn[g][2];
    }
    s.x = xn;
    s.y2 = y2n;
    s.y3 = y3n;
    s.Tmu = iso ? Tiso / mu_of(k, xn, y2n, y3n) : Tmun;
    s.rem -= h;
    ++s.acc;
    s.h = maxrel < 0.05 ? 2.0 * h : h;
    return !(s.rem > 0.0);
}

template <int M>
__device__ __forceinline__ double chem_finish(const KChem &k, double Tiso, const CS &s, unsigned &flags)
{
    const double T = k.isothermal ? Tiso : s.Tmu * mu_of(k, s.x, s.y2, s.y3);
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
// state {N[3], F[3][3], x_HII, x_HeII, x_HeIII, T_mu, rem, h}.
constexpr int QV = 18;

__device__ __forceinline__ void q_store(const QueueView &q, uint32_t p, uint32_t cell, const CS &s)
{
    q.cell[p] = (int32_t)cell;
    q.acc[p] = s.acc;
    q.att[p] = s.att;
    double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        v[(size_t)g * c] = s.N[g];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[(size_t)(3 + 3 * g + d) * c] = s.F[g][d];
    }
    v[12 * c] = s.x;
    v[13 * c] = s.y2;
    v[14 * c] = s.y3;
    v[15 * c] = s.Tmu;
    v[16 * c] = s.rem;
    v[17 * c] = s.h;
}

__device__ __forceinline__ uint32_t q_load(const QueueView &q, uint32_t p, CS &s)
{
    s.acc = q.acc[p];
    s.att = q.att[p];
    const double *v = q.v + p;
    const size_t c = q.stride;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        s.N[g] = v[(size_t)g * c];
#pragma unroll
        for (int d = 0; d < 3; ++d) s.F[g][d] = v[(size_t)(3 + 3 * g + d) * c];
    }
    s.x = v[12 * c];
    s.y2 = v[13 * c];
    s.y3 = v[14 * c];
    s.Tmu = v[15 * c];
    s.rem = v[16 * c];
    s.h = v[17 * c];
    return (uint32_t)q.cell[p];
}

template <typename R, int M>
__device__ __forceinline__ void store_cell(const ChemIO<R> &io, uint32_t i, const CS &s, double T)
{
    const size_t nc = io.ncell;
#pragma unroll
    for (int g = 0; g < M; ++g) {
        io.N[(size_t)g * nc + i] = (R)s.N[g];
#pragma unroll
        for (int d = 0; d < 3; ++d) io.F[(size_t)(3 * g + d) * nc + i] = (R)s.F[g][d];
    }
    io.xHII[i] = s.x;
    io.xHeII[i] = s.y2;
    io.xHeIII[i] = s.y3;
    io.T[i] = T;
    if (io.nacc) io.nacc[i] = s.acc;
    if (io.natt) io.natt[i] = s.att;
}

// Per-block reduction of the chemistry counters; one atomic per block.
__device__ __forceinline__ void block_stats(DevStats *st, unsigned long long acc, unsigned long long att,
                                            unsigned long long mx, unsigned fl)
{
    __shared__ unsigned long long s_acc[256], s_att[256], s_max[256];
    __shared__ unsigned s_fl[256];
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    s_acc[t] = acc;
    s_att[t] = att;
    s_max[t] = mx;
    s_fl[t] = fl;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_acc[t] += s_acc[t + o];
            s_att[t] += s_att[t + o];
            s_max[t] = s_max[t] > s_max[t + o] ? s_max[t] : s_max[t + o];
            s_fl[t] |= s_fl[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (s_att[0]) {
            atomicAdd(&st->acc_total, s_acc[0]);
            atomicAdd(&st->att_total, s_att[0]);
            atomicMax(&st->att_max, s_max[0]);
        }
        if (s_fl[0]) atomicOr(&st->flags, s_fl[0]);
    }
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Head pass: one thread per cell.  With FUSE the cell is first transported
// (all groups, source set -> registers); then up to K chemistry attempts.
// Cells that finish are written to the destination arrays; the rest go to
// the queue (or, when it is full, finish in place).
// Waves per SIMD the chemistry kernels are compiled for (caps their VGPRs).
#ifndef RT_CHEM_WAVES
#define RT_CHEM_WAVES 1
#endif

template <typename R, int M, int FUSE, int FLUX>
__global__ __launch_bounds__(256, RT_CHEM_WAVES) void k_head(KGrid g, const KChem *__restrict__ kp, double dt, R c, R kdx, const R *__restrict__ Nin,
                                              const R *__restrict__ Fin, ChemIO<R> io, const R *__restrict__ tab,
                                              int nf, int nth, QueueView q, int K, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < (uint32_t)g.ncell;
    const size_t nc = g.ncell;
    CS s;
    double nH = 1.0, Tiso = 0.0;
    bool done = true;
    unsigned fl = 0;
    if (valid) {
        if (FUSE) {
            int ix, iy, iz;
            cell_coords(g, i, ix, iy, iz);
            const Nbr nb = neighbours(g, i, ix, iy, iz);
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                const U4<R> o = transport_cell<R, FLUX>(nb, i, nc, Nin + (size_t)grp * nc,
                                                        Fin + (size_t)3 * grp * nc, c, kdx, tab, nf, nth);
                s.N[grp] = (double)o.n;
                s.F[grp][0] = (double)o.fx;
                s.F[grp][1] = (double)o.fy;
                s.F[grp][2] = (double)o.fz;
            }
        } else {
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                s.N[grp] = (double)io.N[(size_t)grp * nc + i];
#pragma unroll
                for (int d = 0; d < 3; ++d) s.F[grp][d] = (double)io.F[(size_t)(3 * grp + d) * nc + i];
            }
        }
        s.x = io.xHII[i];
        s.y2 = io.xHeII[i];
        s.y3 = io.xHeIII[i];
        Tiso = io.T[i];
        nH = io.nH[i];
        if (chem_init<M>(k, dt, Tiso, s)) {
            done = false;
            for (int a = 0; a < K && !done; ++a) done = chem_attempt<M>(k, nH, Tiso, s, fl);
        } else {
            fl |= 2u;
        }
    }
    // wave-aggregated enqueue of the unfinished cells
    const bool want = !done;
    const unsigned long long m = __ballot(want);
    bool queued = false;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned base = 0;
        if (lane_id() == leader) base = atomicAdd(q.count, (unsigned)__popcll(m));
        base = __shfl(base, leader);
        if (want) {
            const unsigned p = base + (unsigned)__popcll(m & ((1ull << lane_id()) - 1ull));
            if (p < q.cap) {
                q_store(q, p, i, s);
                queued = true;
            }
        }
    }
    if (want && !queued) {
        while (!done) done = chem_attempt<M>(k, nH, Tiso, s, fl);
    }
    unsigned long long a_acc = 0, a_att = 0;
    if (valid && !queued) {
        const double T = chem_finish<M>(k, Tiso, s, fl);
        store_cell<R, M>(io, i, s, T);
        a_acc = (unsigned long long)s.acc;
        a_att = (unsigned long long)s.att;
    }
    block_stats(st, a_acc, a_att, a_att, fl);
}

// Tail pass over the queue: persistent waves whose lanes each take a queued
// cell, run one attempt per loop trip, and refill from the queue as soon as
// their cell has filled dt_RT, so that a few slow cells do not hold whole
// waves of finished lanes.
template <typename R, int M>
__global__ __launch_bounds__(256, RT_CHEM_WAVES) void k_tail(const KChem *__restrict__ kp, ChemIO<R> io, QueueView q, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    const unsigned n = min(*q.count, q.cap);
    CS s;
    uint32_t cell = 0;
    double nH = 1.0, Tiso = 0.0;
    bool active = false, exhausted = false;
    unsigned fl = 0;
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    while (true) {
        if (!exhausted) {
            const bool need = !active;
            const unsigned long long m = __ballot(need);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                unsigned base = 0;
                if (lane_id() == leader) base = atomicAdd(q.head, (unsigned)__popcll(m));
                base = __shfl(base, leader);
                if (base >= n) exhausted = true;
                if (need) {
                    const unsigned p = base + (unsigned)__popcll(m & ((1ull << lane_id()) - 1ull));
                    if (p < n) {
                        cell = q_load(q, p, s);
                        nH = io.nH[cell];
                        Tiso = io.T[cell];
                        active = true;
                    }
                }
            }
        }
        if (!__any(active)) break;
        if (active) {
            if (chem_attempt<M>(k, nH, Tiso, s, fl)) {
                const double T = chem_finish<M>(k, Tiso, s, fl);
                store_cell<R, M>(io, cell, s, T);
                a_acc += (unsigned long long)s.acc;
                a_att += (unsigned long long)s.att;
                a_max = a_max > (unsigned long long)s.att ? a_max : (unsigned long long)s.att;
                active = false;
            }
        }
    }
    block_stats(st, a_acc, a_att, a_max, fl);
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    if (threadIdx.x < (unsigned)n) p[threadIdx.x] = 0u;
}

// part 1: reset the queue counters and run the head pass; part 2: the tail
template <typename R, int M, int FUSE, int FLUX>
static void launch_head_tail(int part, const KGrid &g, const KChem &kc, const KChem *dk, double dt, R c, R kdx, const void *Nin,
                             const void *Fin, const ChemIO<R> &io, const void *tab, int nf, int nth,
                             const QueueView &q, int K, DevStats *st, hipStream_t s)
{
    if (part == 1) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, q.count, 2);
        hipLaunchKernelGGL((k_head<R, M, FUSE, FLUX>), dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, s, g,
                           dk, dt, c, kdx, (const R *)Nin, (const R *)Fin, io, (const R *)tab, nf, nth, q, K, st);
    } else {
        hipLaunchKernelGGL((k_tail<R, M>), dim3(TAIL_BLOCKS), dim3(256), 0, s, dk, io, q, st);
    }
}

template <typename R, int FUSE, int FLUX>
static void dispatch_M(int part, const KGrid &g, const KChem &kc, const KChem *dk, double dt, R c, R kdx, const void *Nin, const void *Fin,
                       const ChemIO<R> &io, const void *tab, int nf, int nth, const QueueView &q, int K,
                       DevStats *st, hipStream_t s)
{
    if (kc.M == 1) launch_head_tail<R, 1, FUSE, FLUX>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else if (kc.M == 2) launch_head_tail<R, 2, FUSE, FLUX>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else launch_head_tail<R, 3, FUSE, FLUX>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
}

template <typename R>
static ChemIO<R> make_io(size_t ncell, void *N, void *F, double *xHII, double *xHeII, double *xHeIII, double *T,
                         const double *nH, int32_t *nacc, int32_t *natt)
{
    ChemIO<R> io;
    io.ncell = ncell;
    io.N = (R *)N;
    io.F = (R *)F;
    io.xHII = xHII;
    io.xHeII = xHeII;
    io.xHeIII = xHeIII;
    io.T = T;
    io.nH = nH;
    io.nacc = nacc;
    io.natt = natt;
    return io;
}

hipError_t launch_chem(int part, bool fp32, const KGrid &g, const KChem &kc, const KChem *dk, double dt, void *N, void *F, double *xHII,
                       double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc, int32_t *natt,
                       const QueueView &q, int K, DevStats *stats, hipStream_t s)
{
    if (fp32) {
        ChemIO<float> io = make_io<float>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt);
        dispatch_M<float, 0, 0>(part, g, kc, dk, dt, 0.f, 0.f, nullptr, nullptr, io, nullptr, 0, 0, q, K, stats, s);
    } else {
        ChemIO<double> io = make_io<double>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt);
        dispatch_M<double, 0, 0>(part, g, kc, dk, dt, 0.0, 0.0, nullptr, nullptr, io, nullptr, 0, 0, q, K, stats, s);
    }
    return hipGetLastError();
}

hipError_t launch_step_fused(int part, bool fp32, int flux, const KGrid &g, const KChem &kc, const KChem *dk, double dt, const void *Nin,
                             const void *Fin, void *Nout, void *Fout, double *xHII, double *xHeII, double *xHeIII,
                             double *T, const double *nH, int32_t *nacc, int32_t *natt, const void *hll, int nf,
                             int nth, const QueueView &q, int K, DevStats *stats, hipStream_t s)
{
    const double kdx = dt / g.dx;
    if (fp32) {
        ChemIO<float> io = make_io<float>(g.ncell, Nout, Fout, xHII, xHeII, xHeIII, T, nH, nacc, natt);
        if (flux)
            dispatch_M<float, 1, 1>(part, g, kc, dk, dt, (float)kc.cr, (float)kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
        else
            dispatch_M<float, 1, 0>(part, g, kc, dk, dt, (float)kc.cr, (float)kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
    } else {
        ChemIO<double> io = make_io<double>(g.ncell, Nout, Fout, xHII, xHeII, xHeIII, T, nH, nacc, natt);
        if (flux)
            dispatch_M<double, 1, 1>(part, g, kc, dk, dt, kc.cr, kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
        else
            dispatch_M<double, 1, 0>(part, g, kc, dk, dt, kc.cr, kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- reductions
size_t reduction_scratch_bytes() { return (size_t)RED_BLOCKS * sizeof(RedOut); }

// scratch layout: [reduction partials][2 counters, padded to 256 B]
//                 [cell, acc, att: 3 x cap int32][18 x cap doubles]
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t queue_bytes(unsigned cap)
{
    return 256 + align256((size_t)cap * 3 * sizeof(int32_t)) + (size_t)QV * cap * sizeof(double);
}

QueueView queue_view(void *scratch, unsigned cap, unsigned layout_cap)
{
    char *b = (char *)scratch + align256(reduction_scratch_bytes());
    QueueView q;
    q.count = (unsigned *)b;
    q.head = q.count + 1;
    b += 256;
    q.cell = (int32_t *)b;
    q.acc = q.cell + layout_cap;
    q.att = q.acc + layout_cap;
    b += align256((size_t)layout_cap * 3 * sizeof(int32_t));
    q.v = (double *)b;
    q.cap = cap;
    q.stride = layout_cap;
    return q;
}

template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_partial(size_t nc, int M, double c, double V,
                                                                const R *__restrict__ N, const R *__restrict__ F,
                                                                const double *__restrict__ xHII,
                                                                const double *__restrict__ nH,
                                                                RedOut *__restrict__ part)
{
    double ph[3] = {0, 0, 0}, ion = 0, mf = 0, mn = 1e300;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (size_t)gridDim.x * blockDim.x) {
        for (int g = 0; g < M; ++g) {
            const double n = (double)N[(size_t)g * nc + i];
            const double fx = (double)F[(size_t)(3 * g) * nc + i];
            const double fy = (double)F[(size_t)(3 * g + 1) * nc + i];
            const double fz = (double)F[(size_t)(3 * g + 2) * nc + i];
            ph[g] += n;
            mn = n < mn ? n : mn;
            if (n > 0) {
                const double f = sqrt(fx * fx + fy * fy + fz * fz) / (c * n);
                mf = f > mf ? f : mf;
            }
        }
        ion += xHII[i] * nH[i];
    }
    __shared__ double s[6][RED_THREADS];
    const int t = threadIdx.x;
    s[0][t] = ph[0];
    s[1][t] = ph[1];
    s[2][t] = ph[2];
    s[3][t] = ion;
    s[4][t] = mf;
    s[5][t] = mn;
    __syncthreads();
    for (int o = RED_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) {
            for (int q = 0; q < 4; ++q) s[q][t] += s[q][t + o];
            s[4][t] = s[4][t] > s[4][t + o] ? s[4][t] : s[4][t + o];
            s[5][t] = s[5][t] < s[5][t + o] ? s[5][t] : s[5][t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        RedOut r;
        for (int g = 0; g < 3; ++g) r.photons[g] = s[g][0] * V;
        r.ionised = s[3][0] * V;
        r.maxf = s[4][0];
        r.minN = s[5][0];
        part[blockIdx.x] = r;
    }
}

__global__ void k_reduce_final(const RedOut *__restrict__ part, int np, RedOut *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RedOut r = part[0];
    for (int b = 1; b < np; ++b) {
        for (int g = 0; g < 3; ++g) r.photons[g] += part[b].photons[g];
        r.ionised += part[b].ionised;
        r.maxf = part[b].maxf > r.maxf ? part[b].maxf : r.maxf;
        r.minN = part[b].minN < r.minN ? part[b].minN : r.minN;
    }
    *out = r;
}

hipError_t launch_reduce(bool fp32, size_t ncell, int M, double c, double V, const void *N, const void *F,
                         const double *xHII, const double *nH, void *scratch, RedOut *dev_out, hipStream_t s)
{
    RedOut *part = (RedOut *)scratch;
    if (fp32)
        hipLaunchKernelGGL(k_reduce_partial<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, ncell, M, c, V,
                           (const float *)N, (const float *)F, xHII, nH, part);
    else
        hipLaunchKernelGGL(k_reduce_partial<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, ncell, M, c, V,
                           (const double *)N, (const double *)F, xHII, nH, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, s, part, RED_BLOCKS, dev_out);
    return hipGetLastError();
}

}  // namespace rtm1
