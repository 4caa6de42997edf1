// rt_adjoint.hip -- kernels of the differentiation form: the reverse
// (adjoint) pass of the RT step for hydrogen-only gas, one photon group,
// GLF transport and periodic boundaries.  The forward state is FP64 or the
// mixed form's (FP32 N and F, FP64 gas); tapes and adjoint variables are
// FP64 in both, so the mixed form's gradient is that of its own forward map,
// evaluated at its FP32 radiation states.
//
// Forward step:  U_k --inject--> U_a --transport--> U_b --chemistry--> U_k+1
// with parameters ln Ndot_s (sources) and ln n_H (cells).
//
//  * injection (Sec. 3.1) adds Ndot_s dt / V to N at the source cells, so
//      lambda_k = lambda_a,   dL/dln Ndot_s += lambda_a,N(c_s) Ndot_s dt / V;
//  * GLF transport (eq. dUdt_sol with eq. glf) is, per axis d,
//      U_b(l) = U_a(l) + k [ (G_d(U_l-d) - G_d(U_l+d)) / 2
//                            + c (U_l+d + U_l-d - 2 U_l) / 2 ],   k = dt/dx,
//    whose transpose gives
//      lambda_a(m) = (1 - 3kc) lambda_b(m)
//                  + k/2 sum_d [ J_d(U_a(m))^T (lambda_b(m+d) - lambda_b(m-d))
//                                + c (lambda_b(m+d) + lambda_b(m-d)) ]
//    with J_d = dG_d/dU the Jacobian of the M1 flux;
//  * the chemistry of a cell (App. A) is the chain of its accepted
//    substeps; their lengths are piecewise constant in the state and are
//    held fixed.  The record pass stores each cell's state before every
//    accepted substep and the substep length; the reverse pass rebuilds
//    each substep's Jacobian in forward-mode dual numbers over
//    (N, x_HII, T_mu, ln n_H) -- F only scales by the absorption factor --
//    and applies its transpose, last substep first.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_cell.h"

namespace rtm1 {

// ------------------------------------------------------------ dual numbers
constexpr int ND = 4;  // d/dN, d/dx_HII, d/dT_mu (T when isothermal), d/dln n_H
enum { VN = 0, VX = 1, VT = 2, VL = 3 };

struct Dual {
    double v;
    double d[ND];
};

__device__ __forceinline__ Dual dconst(double v)
{
    Dual r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = 0.0;
    return r;
}
__device__ __forceinline__ Dual dvar(double v, int i)
{
    Dual r = dconst(v);
    r.d[i] = 1.0;
    return r;
}
// f(a) for a scalar function with value fv and derivative fd at a.v
__device__ __forceinline__ Dual dchain(const Dual &a, double fv, double fd)
{
    Dual r;
    r.v = fv;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = fd * a.d[i];
    return r;
}
__device__ __forceinline__ Dual operator+(const Dual &a, const Dual &b)
{
    Dual r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
__device__ __forceinline__ Dual operator-(const Dual &a, const Dual &b)
{
    Dual r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
__device__ __forceinline__ Dual operator-(const Dual &a) { return dchain(a, -a.v, -1.0); }
__device__ __forceinline__ Dual operator*(const Dual &a, const Dual &b)
{
    Dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
__device__ __forceinline__ Dual operator/(const Dual &a, const Dual &b)
{
    Dual r;
    const double ib = 1.0 / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
__device__ __forceinline__ Dual operator+(const Dual &a, double b)
{
    Dual r = a;
    r.v += b;
    return r;
}
__device__ __forceinline__ Dual operator+(double b, const Dual &a) { return a + b; }
__device__ __forceinline__ Dual operator-(const Dual &a, double b) { return a + (-b); }
__device__ __forceinline__ Dual operator-(double b, const Dual &a) { return (-a) + b; }
__device__ __forceinline__ Dual operator*(const Dual &a, double b) { return dchain(a, a.v * b, b); }
__device__ __forceinline__ Dual operator*(double b, const Dual &a) { return dchain(a, a.v * b, b); }
__device__ __forceinline__ Dual operator/(double a, const Dual &b)
{
    const double ib = 1.0 / b.v;
    return dchain(b, a * ib, -a * ib * ib);
}
__device__ __forceinline__ Dual dexp(const Dual &a)
{
    const double e = exp(a.v);
    return dchain(a, e, e);
}
__device__ __forceinline__ Dual dlog(const Dual &a) { return dchain(a, rt_log(a.v), 1.0 / a.v); }
__device__ __forceinline__ Dual dlog1p(const Dual &a) { return dchain(a, rt_log1p(a.v), 1.0 / (1.0 + a.v)); }
__device__ __forceinline__ Dual dsqrt(const Dual &a)
{
    const double s = sqrt(a.v);
    return dchain(a, s, 0.5 / s);
}

// plain doubles through the same code (the frozen-schedule replay)
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(const Dual &a) { return a.v; }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ double dlog(double a) { return rt_log(a); }
__device__ __forceinline__ double dlog1p(double a) { return rt_log1p(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
template <class D>
__device__ __forceinline__ D cst(double v);
template <>
__device__ __forceinline__ double cst<double>(double v) { return v; }
template <>
__device__ __forceinline__ Dual cst<Dual>(double v) { return dconst(v); }

// ---------------------------------------------- App. E rates, dual numbers
// The hydrogen terms of the case-B rate set with their d/dT, as functions
// of a dual temperature (so that d/dT itself is differentiated too).
template <class D>
struct DTq {
    D T, lnT, invT, sqT, s5, g;
};
template <class D>
__device__ __forceinline__ DTq<D> dmake_Tq(const D &T)
{
    DTq<D> q;
    q.T = T;
    q.lnT = dlog(T);
    q.invT = 1.0 / T;
    q.sqT = dsqrt(T);
    q.s5 = q.sqT * 3.1622776601683795e-3;  // sqrt(T / 1e5)
    q.g = 1.0 / (1.0 + q.s5);
    return q;
}
template <class D>
struct DV {
    D v, d;  // value and d/dT
};
// A sqrt(T) (1+sqrt(T/1e5))^-1 exp(-Tj/T)
template <class D>
__device__ __forceinline__ DV<D> d_cen(const DTq<D> &q, double A, double Tj)
{
    DV<D> o;
    o.v = A * q.sqT * q.g * dexp(-Tj * q.invT);
    o.d = o.v * (0.5 - 0.5 * q.s5 * q.g + Tj * q.invT) * q.invT;
    return o;
}
// A lam^p / (1+(lam/l0)^q)^r, lam = TL/T
template <class D>
__device__ __forceinline__ DV<D> d_hg(const DTq<D> &q, double A, double lnTL, double p, double lnl0, double qq, double r)
{
    const D lnlam = lnTL - q.lnT;
    const D u = dexp(qq * (lnlam - lnl0));
    DV<D> o;
    o.v = A * dexp(p * lnlam - r * dlog1p(u));
    o.d = -(o.v * (p - r * qq * u / (1.0 + u)) * q.invT);
    return o;
}
// B T lam^p / (1+(lam/l0)^q)^r
template <class D>
__device__ __forceinline__ DV<D> d_hgc(const DTq<D> &q, double B, double lnTL, double p, double lnl0, double qq, double r)
{
    const D lnlam = lnTL - q.lnT;
    const D u = dexp(qq * (lnlam - lnl0));
    DV<D> o;
    o.v = B * q.T * dexp(p * lnlam - r * dlog1p(u));
    o.d = o.v * (1.0 - (p - r * qq * u / (1.0 + u))) * q.invT;
    return o;
}

// Primordial cooling of hydrogen-only gas (eq. rate_cooling without the
// helium terms) and dL/dT: collisional ionisation and excitation of HI,
// case-B recombination cooling of HII, bremsstrahlung, Compton.
template <class D>
__device__ __forceinline__ void dcooling_H(const DTq<D> &q, double a_exp, const D &ne, const D &nHI, const D &nHII,
                                           D &L, D &dL)
{
    const D zHI = 1.27e-21 * q.sqT * q.g * dexp(-157809.1 * q.invT);
    const D zHIl = 0.5 - 0.5 * q.s5 * q.g + 157809.1 * q.invT;  // dln/dlnT
    const D psHI = 7.5e-19 * q.g * dexp(-118348.0 * q.invT);
    const D psHIl = -0.5 * q.s5 * q.g + 118348.0 * q.invT;
    const DV<D> eHII = d_hgc(q, 3.435e-30, LN_TL_HI, 1.97, LN_2p25, 0.376, 3.72);
    const D th = 1.42e-27 * q.sqT;
    const double Tg = 2.727 / a_exp;
    const double cpk = 1.017e-37 * Tg * Tg * Tg * Tg;
    const D cHI = ne * nHI, cHII = ne * nHII;
    L = (zHI + psHI) * cHI + eHII.v * cHII + th * cHII + cpk * (q.T - Tg) * ne;
    dL = ((zHI * zHIl + psHI * psHIl) * cHI + 0.5 * th * cHII) * q.invT + eHII.d * cHII + cpk * ne;
}

// One accepted substep of length h (App. A tasks 1-3 and the accept step
// for hydrogen-only gas and one group).  In: N, x_HII, T_mu (T when
// isothermal) and ln n_H as duals; out: the new N, x_HII, T_mu and the
// absorption factor 1/(1 + h D) that also scales F.  The 10% checks do
// not enter: the substep was accepted.
template <class D>
__device__ __forceinline__ void dsubstep(const KChem &k, double h, const D &N, const D &x, const D &Tm, const D &lnnH,
                                         D &Nn, D &xn, D &Tmn, D &rden)
{
    const bool iso = k.isothermal != 0;
    const D nH = dexp(lnnH);
    const D nHI = (1.0 - x) * nH;
    const D nHII = x * nH;
    rden = 1.0 / (1.0 + h * (k.cr * k.sN[0][0]) * nHI);
    Nn = N * rden;
    const D mu0 = 1.0 / (k.X * (1.0 + x));
    const D &ne0 = nHII;
    D T1;
    if (!iso) {
        const D K = k.Kfac / nH;
        const DTq<D> q0 = dmake_Tq(Tm * mu0);
        const D H = nHI * (k.cr * (k.eb[0] * k.sE[0][0] - EPS_HI * k.sN[0][0])) * Nn;
        D L, dL;
        dcooling_H(q0, k.a_exp, ne0, nHI, nHII, L, dL);
        const D Kh = K * h;
        Tmn = Tm + (H - L) * Kh / (1.0 + mu0 * dL * Kh);
        T1 = Tmn * mu0;
    } else {
        Tmn = Tm;
        T1 = Tm;
    }
    const DTq<D> q1 = dmake_Tq(T1);
    const DV<D> bH = d_cen(q1, 5.85e-11, 157809.1);
    const DV<D> aH = d_hg(q1, 2.753e-14, LN_TL_HI, 1.5, LN_2p74, 0.407, 2.242);
    const D Cr = bH.v * ne0 + (k.sN[0][0] * k.cr) * Nn;
    const D Dr = aH.v * ne0;
    D dC, dD;
    if (iso) {
        dC = nH * bH.v;
        dD = nH * aH.v;
    } else {
        const D f = ne0 * Tmn * mu0 * mu0 * k.X;
        dC = nH * bH.v - f * bH.d;
        dD = nH * aH.v - f * aH.d;
    }
    const D J = dC - (Cr + Dr) - x * (dC + dD);
    xn = x + h * (Cr - x * (Cr + Dr)) / (1.0 - J * h);
    if (val(xn) < k.x_min) xn = cst<D>(k.x_min);
    else if (val(xn) > 1.0) xn = cst<D>(1.0);
}

// ------------------------------------------------------------ trace layout
// Cell i owns trace entries off[i] .. off[i] + counts[i] (counts[i] + 1 of
// them, 7 doubles each): entry j < counts[i] is the state before accepted
// substep j {N, Fx, Fy, Fz, x_HII, T_mu (T when isothermal), h}; the last
// is the state after the chemistry with slot 6 = number of substeps taken.
constexpr int TV = 7;

// Thermochemistry of every cell as in rt_thermochem (one group, hydrogen
// only, FP64 arithmetic on N and F stored as R), in place, writing the
// trace.  A cell that takes more
// substeps than counts[i], or whose entries would pass cap, sets flag bit
// RT_TRACE_FLAG and records what fits.
constexpr unsigned RT_TRACE_FLAG = 16u;

template <typename R>
__global__ __launch_bounds__(256) void k_chem_record(const KChem *__restrict__ kp, size_t nc, double dt,
                                                     R *__restrict__ N, R *__restrict__ F,
                                                     double *__restrict__ xHII, double *__restrict__ T,
                                                     const double *__restrict__ nH, const int32_t *__restrict__ counts,
                                                     const int64_t *__restrict__ off, long long cap,
                                                     double *__restrict__ trace, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int cnt = counts[i];
    const int64_t o = off[i];
    const bool fits = cnt >= 0 && o + cnt < (int64_t)cap;
    double *tr = trace + (size_t)TV * (size_t)o;
    CS s;
    s.N[0] = (double)N[i];
    s.N[1] = s.N[2] = 0.0;
    s.fs[1] = s.fs[2] = 1.0;
    const double F0[3] = {(double)F[i], (double)F[nc + i], (double)F[2 * nc + i]};
    s.x = xHII[i];
    s.y2 = 0.0;
    s.y3 = 0.0;
    const CC cc = make_cc(k, nH[i], T[i]);
    unsigned fl = 0;
    const bool ok =
        chem_init<CM>(k, dt, cc.Tiso, isfinite(F0[0]) && isfinite(F0[1]) && isfinite(F0[2]), s);
    bool done = !ok;
    int n = 0;
    while (!done) {
        const double e0 = s.N[0], e4 = s.x, fs = s.fs[0];
        const double e5 = k.isothermal ? cc.Tiso : s.Tmu;
        const double h = s.h >= s.rem * (1.0 - 1e-10) ? s.rem : s.h;  // the length chem_attempt takes
        const int acc0 = s.acc;
        done = chem_attempt<CM, 0, false>(k, cc, s, fl);  // one attempt per call: h above is its length
        if (s.acc != acc0) {
            if (fits && n < cnt) {
                double *e = tr + TV * n;
                e[0] = e0;
                e[1] = F0[0] * fs;
                e[2] = F0[1] * fs;
                e[3] = F0[2] * fs;
                e[4] = e4;
                e[5] = e5;
                e[6] = h;
            }
            ++n;
        }
    }
    if (n != cnt || !fits) fl |= RT_TRACE_FLAG;
    if (fits) {
        double *e = tr + TV * cnt;
        e[0] = s.N[0];
        e[1] = F0[0] * s.fs[0];
        e[2] = F0[1] * s.fs[0];
        e[3] = F0[2] * s.fs[0];
        e[4] = s.x;
        e[5] = k.isothermal ? cc.Tiso : s.Tmu;
        e[6] = (double)(n < cnt ? n : cnt);
    }
    if (ok) {
        const double Tout = chem_finish<CM>(k, cc, s, fl);
        N[i] = (R)s.N[0];
        F[i] = (R)(F0[0] * s.fs[0]);
        F[nc + i] = (R)(F0[1] * s.fs[0]);
        F[2 * nc + i] = (R)(F0[2] * s.fs[0]);
        xHII[i] = s.x;
        T[i] = Tout;
    } else {
        fl |= 2u;
    }
    if (fl) atomicOr(&st->flags, fl);
}

// Chemistry with a recorded substep schedule: every cell takes the number
// of substeps and the lengths of its trace, from its current state and
// without the 10% checks.  The result is a smooth function of the inputs
// whose derivative is the one the adjoint computes; with the recorded
// inputs it reproduces the recorded step up to rounding.
template <typename R>
__global__ __launch_bounds__(256) void k_chem_replay(const KChem *__restrict__ kp, size_t nc, R *__restrict__ N,
                                                     R *__restrict__ F, double *__restrict__ xHII,
                                                     double *__restrict__ T, const double *__restrict__ nH,
                                                     const int32_t *__restrict__ counts,
                                                     const int64_t *__restrict__ off, long long cap,
                                                     const double *__restrict__ trace)
{
    const KChem &k = *kp;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int cnt = counts[i];
    const int64_t o = off[i];
    if (!(cnt >= 0 && o + cnt < (int64_t)cap)) return;
    const double *tr = trace + (size_t)TV * (size_t)o;
    const double nf = tr[TV * cnt + 6];
    const int n = (nf >= 0.0 && nf <= (double)cnt) ? (int)nf : 0;
    const bool iso = k.isothermal != 0;
    double Nc = (double)N[i], Fx = (double)F[i], Fy = (double)F[nc + i], Fz = (double)F[2 * nc + i], x = xHII[i];
    const double T0 = T[i];
    double Tm = iso ? T0 : T0 * (k.X * (1.0 + x));  // T_mu = T / mu
    const double lnnH = log(nH[i]);
    for (int j = 0; j < n; ++j) {
        double Nn, xn, Tmn, rden;
        dsubstep(k, tr[TV * j + 6], Nc, x, Tm, lnnH, Nn, xn, Tmn, rden);
        Nc = Nn;
        Fx *= rden;
        Fy *= rden;
        Fz *= rden;
        x = xn;
        Tm = Tmn;
    }
    N[i] = (R)Nc;
    F[i] = (R)Fx;
    F[nc + i] = (R)Fy;
    F[2 * nc + i] = (R)Fz;
    xHII[i] = x;
    T[i] = iso ? T0 : Tm / (k.X * (1.0 + x));
}

// --------------------------------------------------------------- chem adjoint
// (lambda_N, lambda_F) after the chemistry -> (wN, wF) before it;
// lambda_x, lambda_T in place; g_lnnH += the step's d/dln n_H.
__global__ __launch_bounds__(256) void k_chem_adj(const KChem *__restrict__ kp, size_t nc,
                                                  const double *__restrict__ nH, const int32_t *__restrict__ counts,
                                                  const int64_t *__restrict__ off, long long cap,
                                                  const double *__restrict__ trace, const double *__restrict__ lN,
                                                  const double *__restrict__ lF, double *__restrict__ lx,
                                                  double *__restrict__ lT, double *__restrict__ wN,
                                                  double *__restrict__ wF, double *__restrict__ glnnH)
{
    const KChem &k = *kp;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const bool iso = k.isothermal != 0;
    const int cnt = counts[i];
    const int64_t o = off[i];
    double aN = lN[i], aFx = lF[i], aFy = lF[nc + i], aFz = lF[2 * nc + i], ax = lx[i], aT = lT[i];
    double g = 0.0;
    if (cnt >= 0 && o + cnt < (int64_t)cap) {
        const double *tr = trace + (size_t)TV * (size_t)o;
        const double *fin = tr + TV * cnt;
        const double nf = fin[6];  // substeps recorded, at most cnt
        const int n = (nf >= 0.0 && nf <= (double)cnt) ? (int)nf : 0;
        if (!iso) {
            // T_out = T_mu mu(x), mu = 1/(X (1 + x))
            const double mu = 1.0 / (k.X * (1.0 + fin[4]));
            ax += aT * fin[5] * (-k.X * mu * mu);
            aT *= mu;
        }
        const double lnnH = log(nH[i]);
        for (int j = n - 1; j >= 0; --j) {
            const double *e = tr + TV * j;
            Dual Nn, xn, Tmn, rden;
            dsubstep(k, e[6], dvar(e[0], VN), dvar(e[4], VX), dvar(e[5], VT), dvar(lnnH, VL), Nn, xn, Tmn, rden);
            // F_out = F_in rden: the F adjoint scales, and (lambda_F . F_in) weighs d rden
            const double wr = aFx * e[1] + aFy * e[2] + aFz * e[3];
            double a[ND];
#pragma unroll
            for (int q = 0; q < ND; ++q)
                a[q] = aN * Nn.d[q] + ax * xn.d[q] + (iso ? 0.0 : aT * Tmn.d[q]) + wr * rden.d[q];
            aFx *= rden.v;
            aFy *= rden.v;
            aFz *= rden.v;
            aN = a[VN];
            ax = a[VX];
            if (!iso) aT = a[VT];
            g += a[VL];
        }
        if (!iso) {
            // T_mu = T / mu(x) at the start of the chemistry
            const double x0 = tr[4];
            const double T0 = tr[5] / (k.X * (1.0 + x0));
            const double aTm = aT;
            aT = aTm * k.X * (1.0 + x0);
            ax += aTm * T0 * k.X;
        }
    }
    wN[i] = aN;
    wF[i] = aFx;
    wF[nc + i] = aFy;
    wF[2 * nc + i] = aFz;
    lx[i] = ax;
    lT[i] = aT;
    glnnH[i] += g;
}

// ---------------------------------------------------------- transport adjoint
// out = J_d^T v for the M1 flux G_d = (F_d, c^2 P_.d) at state (N, F),
// c = c_r.  With phi = F/(c N), s = |phi|^2 and, for s <= 1,
//   c^2 P = c^2 N [ a(s) I + b(s) phi (x) phi ],
//   a = (1 - chi)/2,  b = (3 chi - 1)/(2 s) = 3/(2 + r),  r = sqrt(4 - 3 s):
//   dG_j/dN   = c^2 [ (a - 2 s a') delta_jd - phi_j phi_d (b + 2 s b') ]
//   dG_j/dF_k = c [ 2 a' phi_k delta_jd + b (delta_jk phi_d + phi_j delta_dk)
//                   + 2 b' phi_j phi_d phi_k ]
// (row j of the F part); for s > 1 (chi = 1) c^2 P = c^2 N n (x) n.
__device__ __forceinline__ void m1_jt(double N, double Fx, double Fy, double Fz, double c, int d, const double v[4],
                                      double out[4])
{
    const double vf[3] = {v[1], v[2], v[3]};
    out[0] = 0.0;
    out[1] = out[2] = out[3] = 0.0;
    out[1 + d] = v[0];  // dG_N/dF_d = 1
    const double icN = 1.0 / (c * N);
    if (!(N > 0.0) || isinf(icN)) return;  // empty cells carry no pressure
    const double ph[3] = {Fx * icN, Fy * icN, Fz * icN};
    const double s = ph[0] * ph[0] + ph[1] * ph[1] + ph[2] * ph[2];
    const double pv = ph[0] * vf[0] + ph[1] * vf[1] + ph[2] * vf[2];
    if (s > 1.0) {
        // c^2 P_jd = c^2 N n_j n_d, n = phi/|phi|; d(n_j n_d)/dF_k =
        // [(delta_jk - n_j n_k) n_d + n_j (delta_dk - n_d n_k)] / |F|
        const double ir = 1.0 / sqrt(s);
        const double n[3] = {ph[0] * ir, ph[1] * ir, ph[2] * ir};
        const double nv = n[0] * vf[0] + n[1] * vf[1] + n[2] * vf[2];
        out[0] = c * c * n[d] * nv;
        const double w = c * ir;  // c^2 N / |F|
        for (int kk = 0; kk < 3; ++kk)
            out[1 + kk] += w * (vf[kk] * n[d] - 2.0 * n[kk] * n[d] * nv + (kk == d ? nv : 0.0));
        return;
    }
    const double r = sqrt(4.0 - 3.0 * s);
    const double q = 5.0 + 2.0 * r;
    const double chi = (3.0 + 4.0 * s) / q;
    const double chis = (4.0 * q + (3.0 + 4.0 * s) * 3.0 / r) / (q * q);  // dchi/ds
    const double a = 0.5 * (1.0 - chi), ap = -0.5 * chis;
    const double b = 3.0 / (2.0 + r), bp = 4.5 / (r * (2.0 + r) * (2.0 + r));
    out[0] = c * c * ((a - 2.0 * s * ap) * vf[d] - ph[d] * (b + 2.0 * s * bp) * pv);
    for (int kk = 0; kk < 3; ++kk)
        out[1 + kk] += c * (2.0 * ap * ph[kk] * vf[d] + (kk == d ? b * pv : 0.0) + b * ph[d] * vf[kk] +
                            2.0 * bp * ph[d] * ph[kk] * pv);
}

__global__ __launch_bounds__(256) void k_transport_adj(KGrid g, double c, double kdx, const double *__restrict__ Na,
                                                       const double *__restrict__ Fa, const double *__restrict__ lNb,
                                                       const double *__restrict__ lFb, double *__restrict__ lNa,
                                                       double *__restrict__ lFa)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)g.ncell) return;
    const size_t nc = g.ncell;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    const Nbr nb = neighbours(g, i, ix, iy, iz);
    const double N = Na[i], Fx = Fa[i], Fy = Fa[nc + i], Fz = Fa[2 * nc + i];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t im = nb.idx[2 * d], ip = nb.idx[2 * d + 1];
        const double lm[4] = {lNb[im], lFb[im], lFb[nc + im], lFb[2 * nc + im]};
        const double lp[4] = {lNb[ip], lFb[ip], lFb[nc + ip], lFb[2 * nc + ip]};
        double dv[4], jt[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dv[q] = lp[q] - lm[q];
        m1_jt(N, Fx, Fy, Fz, c, d, dv, jt);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += 0.5 * (jt[q] + c * (lp[q] + lm[q]));
    }
    const double dg = 1.0 - 3.0 * kdx * c;
    lNa[i] = dg * lNb[i] + kdx * acc[0];
    lFa[i] = dg * lFb[i] + kdx * acc[1];
    lFa[nc + i] = dg * lFb[nc + i] + kdx * acc[2];
    lFa[2 * nc + i] = dg * lFb[2 * nc + i] + kdx * acc[3];
}

// injection adjoint over the sources as given by the caller
__global__ void k_inject_adj(const double *__restrict__ lN, int nsrc, const int32_t *__restrict__ cell,
                             const double *__restrict__ ndot, double dtV, double *__restrict__ g)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    g[s] += lN[cell[s]] * ndot[s] * dtV;
}

// ------------------------------------------------------------ offsets scan
// off[i] = sum_{j<i} (counts[j] + 1), off[nc] = total; off[nc+1 ...] holds
// one partial sum per 1024 cells.
constexpr int SCAN_T = 256, SCAN_PER = 4, SCAN_BLK = SCAN_T * SCAN_PER;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        const int64_t a = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[SCAN_T - 1];
    const int64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_part(const int32_t *__restrict__ counts, size_t nc,
                                                      int64_t *__restrict__ part)
{
    __shared__ int64_t sh[SCAN_T];
    const size_t base = (size_t)blockIdx.x * SCAN_BLK + (size_t)threadIdx.x * SCAN_PER;
    int64_t v = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j)
        if (base + j < nc) v += (int64_t)counts[base + j] + 1;
    int64_t tot;
    block_excl_scan(v, sh, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_top(int64_t *__restrict__ part, size_t nblk,
                                                     int64_t *__restrict__ total_out)
{
    __shared__ int64_t sh[SCAN_T];
    int64_t carry = 0;
    for (size_t b0 = 0; b0 < nblk; b0 += SCAN_T) {
        const size_t b = b0 + threadIdx.x;
        const int64_t v = b < nblk ? part[b] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, sh, tot);
        if (b < nblk) part[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int32_t *__restrict__ counts, size_t nc,
                                                       const int64_t *__restrict__ part, int64_t *__restrict__ off)
{
    __shared__ int64_t sh[SCAN_T];
    const size_t base = (size_t)blockIdx.x * SCAN_BLK + (size_t)threadIdx.x * SCAN_PER;
    int64_t v[SCAN_PER], s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        v[j] = base + j < nc ? (int64_t)counts[base + j] + 1 : 0;
        s += v[j];
    }
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_excl_scan(s, sh, tot);
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        if (base + j < nc) off[base + j] = run;
        run += v[j];
    }
}

size_t adj_scan_parts(size_t nc) { return (nc + SCAN_BLK - 1) / SCAN_BLK; }

hipError_t launch_offsets(const int32_t *counts, size_t nc, int64_t *off, hipStream_t s)
{
    const size_t nblk = adj_scan_parts(nc);
    int64_t *part = off + nc + 1;
    hipLaunchKernelGGL(k_scan_part, dim3((unsigned)nblk), dim3(SCAN_T), 0, s, counts, nc, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, part, nblk, off + nc);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(SCAN_T), 0, s, counts, nc, part, off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_chem_record(const KChem *dk, size_t nc, double dt, R *N, R *F, double *xHII, double *T,
                              const double *nH, const int32_t *counts, const int64_t *off, long long cap,
                              double *trace, DevStats *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_chem_record<R>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, dk, nc, dt, N, F, xHII,
                       T, nH, counts, off, cap, trace, st);
    return hipGetLastError();
}
template hipError_t launch_chem_record<double>(const KChem *, size_t, double, double *, double *, double *, double *,
                                               const double *, const int32_t *, const int64_t *, long long, double *,
                                               DevStats *, hipStream_t);
template hipError_t launch_chem_record<float>(const KChem *, size_t, double, float *, float *, double *, double *,
                                              const double *, const int32_t *, const int64_t *, long long, double *,
                                              DevStats *, hipStream_t);

template <typename R>
hipError_t launch_chem_replay(const KChem *dk, size_t nc, R *N, R *F, double *xHII, double *T, const double *nH,
                              const int32_t *counts, const int64_t *off, long long cap, const double *trace,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_chem_replay<R>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, dk, nc, N, F, xHII, T,
                       nH, counts, off, cap, trace);
    return hipGetLastError();
}
template hipError_t launch_chem_replay<double>(const KChem *, size_t, double *, double *, double *, double *,
                                               const double *, const int32_t *, const int64_t *, long long,
                                               const double *, hipStream_t);
template hipError_t launch_chem_replay<float>(const KChem *, size_t, float *, float *, double *, double *,
                                              const double *, const int32_t *, const int64_t *, long long,
                                              const double *, hipStream_t);

// the pre-transport radiation of a step, widened to the tape's FP64
__global__ void k_widen(const float *__restrict__ a, double *__restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

hipError_t launch_widen(const float *a, double *b, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_chem_adj(const KChem *dk, size_t nc, const double *nH, const int32_t *counts, const int64_t *off,
                           long long cap, const double *trace, const double *lN, const double *lF, double *lx,
                           double *lT, double *wN, double *wF, double *g, hipStream_t s)
{
    hipLaunchKernelGGL(k_chem_adj, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, dk, nc, nH, counts, off, cap,
                       trace, lN, lF, lx, lT, wN, wF, g);
    return hipGetLastError();
}

hipError_t launch_transport_adj(const KGrid &g, double c, double kdx, const double *Na, const double *Fa,
                                const double *lNb, const double *lFb, double *lNa, double *lFa, hipStream_t s)
{
    hipLaunchKernelGGL(k_transport_adj, dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, s, g, c, kdx, Na, Fa,
                       lNb, lFb, lNa, lFa);
    return hipGetLastError();
}

hipError_t launch_inject_adj(const double *lN, int nsrc, const int32_t *cell, const double *ndot, double dtV,
                             double *g, hipStream_t s)
{
    if (nsrc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inject_adj, dim3((unsigned)((nsrc + 63) / 64)), dim3(64), 0, s, lN, nsrc, cell, ndot, dtV, g);
    return hipGetLastError();
}

}  // namespace rtm1
