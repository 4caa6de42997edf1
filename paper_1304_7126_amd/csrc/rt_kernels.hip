// rt_kernels.hip -- gfx950 kernels of the explicit M1 RT step.
//
//   k_inject     point-source injection (Sec. 3.1)
//   k_transport  unsplit GLF/HLL update of (N, F) per group (Sec. 3.2)
//   k_chem       per-cell subcycled thermochemistry in FP64 (App. A)
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
__device__ __forceinline__ U4<R> load_u(const R *__restrict__ N, const R *__restrict__ F, size_t nc, size_t i)
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

// neighbour of cell c along axis d at offset s (+-1), with ghost cells per bc
template <typename R>
__device__ __forceinline__ U4<R> neighbour(const KGrid &g, const R *N, const R *F, int ix, int iy, int iz, int d,
                                           int s)
{
    int c[3] = {ix, iy, iz};
    const int n[3] = {g.nx, g.ny, g.nz};
    int j = c[d] + s;
    bool refl = false;
    if (j < 0 || j >= n[d]) {
        const int bc = g.bc[2 * d + (s > 0 ? 1 : 0)];
        if (bc == 0) {
            j = j < 0 ? j + n[d] : j - n[d];
        } else {
            j = c[d];
            refl = (bc == 2);
        }
    }
    c[d] = j;
    const size_t i = (size_t)c[0] + (size_t)g.nx * ((size_t)c[1] + (size_t)g.ny * (size_t)c[2]);
    U4<R> u = load_u(N, F, g.ncell, i);
    if (refl) {
        if (d == 0) u.fx = -u.fx;
        else if (d == 1) u.fy = -u.fy;
        else u.fz = -u.fz;
    }
    return u;
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

// intercell flux between L and R along axis d: eq. (glf) or eq. (hll)
template <typename R, int FLUX>
__device__ __forceinline__ void face_flux(const U4<R> &L, const R PL[6], const U4<R> &Rt, const R PR[6], int d,
                                          R c, const R *tab, int nf, int nth, R Phi[4])
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
    R l0m, l0p, l1m, l1p;
    hll_speeds(tab, nf, nth, L.n, L.fx, L.fy, L.fz, comp(L, d), c, l0m, l0p);
    hll_speeds(tab, nf, nth, Rt.n, Rt.fx, Rt.fy, Rt.fz, comp(Rt, d), c, l1m, l1p);
    R lp = l0p > l1p ? l0p : l1p;
    lp = (lp > R(0) ? lp : R(0)) * c;
    R lm = l0m < l1m ? l0m : l1m;
    lm = (lm < R(0) ? lm : R(0)) * c;
    const R den = lp - lm;
    if (den == R(0)) {
#pragma unroll
        for (int m = 0; m < 4; ++m) Phi[m] = R(0.5) * (GL[m] + GR[m]);
        return;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) Phi[m] = (lp * GL[m] - lm * GR[m] + lp * lm * (uR[m] - uL[m])) / den;
}

// One thread per cell of one group (blockIdx.y).  Every face flux comes from
// the source arrays; the destination arrays receive
//   U' = U + dt/dx * sum_d (Phi_{d,-1/2} - Phi_{d,+1/2})     (eq. dUdt_sol)
template <typename R, int FLUX>
__global__ __launch_bounds__(256) void k_transport(KGrid g, R c, R kdx, const R *__restrict__ Nin,
                                                   const R *__restrict__ Fin, R *__restrict__ Nout,
                                                   R *__restrict__ Fout, const R *__restrict__ tab, int nf,
                                                   int nth)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.ncell) return;
    const int grp = blockIdx.y;
    const size_t nc = g.ncell;
    const R *N = Nin + (size_t)grp * nc;
    const R *F = Fin + (size_t)3 * grp * nc;
    const int ix = (int)(i % (size_t)g.nx);
    const int iy = (int)((i / (size_t)g.nx) % (size_t)g.ny);
    const int iz = (int)(i / ((size_t)g.nx * (size_t)g.ny));
    const U4<R> C = load_u(N, F, nc, i);
    R PC[6];
    m1_pressure(C.n, C.fx, C.fy, C.fz, c, PC);
    R acc[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const U4<R> L = neighbour(g, N, F, ix, iy, iz, d, -1);
        const U4<R> Rt = neighbour(g, N, F, ix, iy, iz, d, +1);
        R PL[6], PR[6], Pm[4], Pp[4];
        m1_pressure(L.n, L.fx, L.fy, L.fz, c, PL);
        m1_pressure(Rt.n, Rt.fx, Rt.fy, Rt.fz, c, PR);
        face_flux<R, FLUX>(L, PL, C, PC, d, c, tab, nf, nth, Pm);
        face_flux<R, FLUX>(C, PC, Rt, PR, d, c, tab, nf, nth, Pp);
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] += Pm[m] - Pp[m];
    }
    Nout[(size_t)grp * nc + i] = C.n + kdx * acc[0];
    R *Fo = Fout + (size_t)3 * grp * nc;
    Fo[i] = C.fx + kdx * acc[1];
    Fo[nc + i] = C.fy + kdx * acc[2];
    Fo[2 * nc + i] = C.fz + kdx * acc[3];
}

hipError_t launch_transport(bool fp32, int flux, const KGrid &g, int M, double c, double dt, const void *Nin,
                            const void *Fin, void *Nout, void *Fout, const void *hll, int nf, int nth,
                            hipStream_t s)
{
    dim3 b(256), gr((unsigned)((g.ncell + 255) / 256), (unsigned)M);
    const double k = dt / g.dx;
    if (fp32) {
        auto kern = flux ? k_transport<float, 1> : k_transport<float, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, (float)c, (float)k, (const float *)Nin, (const float *)Fin,
                           (float *)Nout, (float *)Fout, (const float *)hll, nf, nth);
    } else {
        auto kern = flux ? k_transport<double, 1> : k_transport<double, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, c, k, (const double *)Nin, (const double *)Fin,
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

// One cell over dt_RT (App. A).  The substep length h starts at dt_RT; a
// substep is restarted with h/2 when any checked quantity changes by more
// than 10% (photon densities, T_mu and its first-order estimate, x_HII and
// its first-order estimate, n_e); after an accepted substep the next h is
// doubled when the largest change was below 5%.
template <int M>
__device__ unsigned chem_cell(const KChem &k, double dt, double nH, double (&N)[3], double (&F)[3][3], double &x,
                              double &y2, double &y3, double &T, int &nacc, int &natt)
{
    const double nHe = nH * k.Y / (4.0 * k.X);
    const double K = k.Kfac / nH;
    const bool iso = k.isothermal != 0;
    const double Tiso = T;
    double Tmu = T / mu_of(k, x, y2, y3);
    // isothermal: every rate is fixed for the whole step
    vd bH_i = {0, 0}, aH_i = {0, 0}, bHe1_i = {0, 0}, aHe2_i = {0, 0}, bHe2_i = {0, 0}, aHe3_i = {0, 0};
    if (iso) {
        const Tq q = make_Tq(Tiso);
        bH_i = beta_HI(q);
        aH_i = alphaB_HII(q);
        if (nHe > 0.0) {
            bHe1_i = beta_HeI(q);
            aHe2_i = alphaB_HeII(q);
            bHe2_i = beta_HeII(q);
            aHe3_i = alphaB_HeIII(q);
        }
    }
    double rem = dt, h = dt;
    int acc = 0, att = 0;
    unsigned flags = 0;
    while (rem > 0.0) {
        if (att >= k.max_att) {
            flags |= 1u;
            break;
        }
        ++att;
        if (h >= rem * (1.0 - 1e-10)) h = rem;
        double maxrel = 0.0, r;
        // ---- photons: semi-implicit absorption from backward abundances
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
            const double den = 1.0 + h * D;
            Nn[g] = N[g] / den;
            Fn[g][0] = F[g][0] / den;
            Fn[g][1] = F[g][1] / den;
            Fn[g][2] = F[g][2] / den;
            r = N[g] > k.N_floor ? rel_change(Nn[g], N[g]) : 0.0;
            fail |= r > 0.1;
            maxrel = r > maxrel ? r : maxrel;
        }
        if (fail) {
            h *= 0.5;
            continue;
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
                h *= 0.5;
                continue;
            }
            Tmun = Tmu + Lam * K * h / den;
            r = rel_change(Tmun, Tmu);
            if (r > 0.1 || fabs(K * Lam * h) / Tmu > 0.1) {
                h *= 0.5;
                continue;
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
        vd bH, aH;
        if (iso) {
            bH = bH_i;
            aH = aH_i;
        } else {
            const Tq q1 = make_Tq(Tmun * mu0);
            bH = beta_HI(q1);
            aH = alphaB_HII(q1);
        }
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
            h *= 0.5;
            continue;
        }
        const double rate = Cr - x * (Cr + Dr);
        double xn = x + h * rate / denx;
        xn = xn < k.x_min ? k.x_min : (xn > 1.0 ? 1.0 : xn);
        r = rel_change(xn, x);
        if (r > 0.1 || fabs(rate) * h / x > 0.1) {
            h *= 0.5;
            continue;
        }
        maxrel = r > maxrel ? r : maxrel;
        // ---- helium: HeI, HeII, HeIII in order, then He conservation
        double y2n = y2, y3n = y3;
        if (nHe > 0.0) {
            const double ne1 = xn * nH + (y2 + 2.0 * y3) * nHe;
            vd bHe1, aHe2, bHe2, aHe3;
            if (iso) {
                bHe1 = bHe1_i;
                aHe2 = aHe2_i;
                bHe2 = bHe2_i;
                aHe3 = aHe3_i;
            } else {
                const Tq q2 = make_Tq(Tmun * mu_of(k, xn, y2, y3));
                bHe1 = beta_HeI(q2);
                aHe2 = alphaB_HeII(q2);
                bHe2 = beta_HeII(q2);
                aHe3 = alphaB_HeIII(q2);
            }
            const double y1 = 1.0 - y2 - y3;
            const double y1n = (y1 + y2 * aHe2.v * ne1 * h) / (1.0 + (bHe1.v * ne1 + GHeI) * h);
            y2n = (y2 + (y1n * (bHe1.v * ne1 + GHeI) + y3 * aHe3.v * ne1) * h) /
                  (1.0 + ((bHe2.v + aHe2.v) * ne1 + GHeII) * h);
            const double ne2 = xn * nH + (y2n + 2.0 * y3) * nHe;
            vd bHe2b, aHe3b;
            if (iso) {
                bHe2b = bHe2_i;
                aHe3b = aHe3_i;
            } else {
                const Tq q3 = make_Tq(Tmun * mu_of(k, xn, y2n, y3));
                bHe2b = beta_HeII(q3);
                aHe3b = alphaB_HeIII(q3);
            }
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
            h *= 0.5;
            continue;
        }
        maxrel = r > maxrel ? r : maxrel;
        // ---- accept
#pragma unroll
        for (int g = 0; g < M; ++g) {
            N[g] = Nn[g];
            F[g][0] = Fn[g][0];
            F[g][1] = Fn[g][1];
            F[g][2] = Fn[g][2];
        }
        x = xn;
        y2 = y2n;
        y3 = y3n;
        Tmu = iso ? Tiso / mu_of(k, x, y2, y3) : Tmun;
        rem -= h;
        ++acc;
        if (maxrel < 0.05) h *= 2.0;
    }
    T = iso ? Tiso : Tmu * mu_of(k, x, y2, y3);
#pragma unroll
    for (int g = 0; g < M; ++g) {
        if (N[g] < 0.0) flags |= 8u;
        if (!isfinite(N[g])) flags |= 2u;
    }
    if (!isfinite(T) || !isfinite(x)) flags |= 2u;
    nacc = acc;
    natt = att;
    return flags;
}

template <typename R, int M>
__global__ __launch_bounds__(256) void k_chem(KChem k, size_t nc, double dt, R *__restrict__ Nr, R *__restrict__ Fr,
                                              double *__restrict__ xHII, double *__restrict__ xHeII,
                                              double *__restrict__ xHeIII, double *__restrict__ Tg,
                                              const double *__restrict__ nH, int32_t *__restrict__ nacc,
                                              int32_t *__restrict__ natt, DevStats *__restrict__ st)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    unsigned fl = 0;
    if (i < nc) {
        double N[3], F[3][3];
#pragma unroll
        for (int g = 0; g < M; ++g) {
            N[g] = (double)Nr[(size_t)g * nc + i];
#pragma unroll
            for (int d = 0; d < 3; ++d) F[g][d] = (double)Fr[(size_t)(3 * g + d) * nc + i];
        }
        double x = xHII[i], y2 = xHeII[i], y3 = xHeIII[i], T = Tg[i];
        int na, nt;
        fl = chem_cell<M>(k, dt, nH[i], N, F, x, y2, y3, T, na, nt);
#pragma unroll
        for (int g = 0; g < M; ++g) {
            Nr[(size_t)g * nc + i] = (R)N[g];
#pragma unroll
            for (int d = 0; d < 3; ++d) Fr[(size_t)(3 * g + d) * nc + i] = (R)F[g][d];
        }
        xHII[i] = x;
        xHeII[i] = y2;
        xHeIII[i] = y3;
        Tg[i] = T;
        if (nacc) nacc[i] = na;
        if (natt) natt[i] = nt;
        a_acc = (unsigned long long)na;
        a_att = (unsigned long long)nt;
        a_max = a_att;
    }
    // block reduction of the counters, one atomic per block
    __shared__ unsigned long long s_acc[256], s_att[256], s_max[256];
    __shared__ unsigned s_fl[256];
    const int t = threadIdx.x;
    s_acc[t] = a_acc;
    s_att[t] = a_att;
    s_max[t] = a_max;
    s_fl[t] = fl;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_acc[t] += s_acc[t + o];
            s_att[t] += s_att[t + o];
            s_max[t] = s_max[t] > s_max[t + o] ? s_max[t] : s_max[t + o];
            s_fl[t] |= s_fl[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        atomicAdd(&st->acc_total, s_acc[0]);
        atomicAdd(&st->att_total, s_att[0]);
        atomicMax(&st->att_max, s_max[0]);
        if (s_fl[0]) atomicOr(&st->flags, s_fl[0]);
    }
}

hipError_t launch_chem(bool fp32, const KChem &kc, size_t ncell, double dt, void *N, void *F, double *xHII,
                       double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc, int32_t *natt,
                       DevStats *stats, hipStream_t s)
{
    dim3 b(256), gr((unsigned)((ncell + 255) / 256));
#define RT_CHEM_LAUNCH(R, MM)                                                                                 \
    hipLaunchKernelGGL((k_chem<R, MM>), gr, b, 0, s, kc, ncell, dt, (R *)N, (R *)F, xHII, xHeII, xHeIII, T, \
                       nH, nacc, natt, stats)
    if (fp32) {
        if (kc.M == 1) RT_CHEM_LAUNCH(float, 1);
        else if (kc.M == 2) RT_CHEM_LAUNCH(float, 2);
        else RT_CHEM_LAUNCH(float, 3);
    } else {
        if (kc.M == 1) RT_CHEM_LAUNCH(double, 1);
        else if (kc.M == 2) RT_CHEM_LAUNCH(double, 2);
        else RT_CHEM_LAUNCH(double, 3);
    }
#undef RT_CHEM_LAUNCH
    return hipGetLastError();
}

// -------------------------------------------------------------- reductions
size_t reduction_scratch_bytes() { return (size_t)RED_BLOCKS * sizeof(RedOut); }

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
