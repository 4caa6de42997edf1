/*
 * rt_oracle.c -- plain, slow, FP64 CPU reference of the explicit M1
 * radiative-transfer step of Rosdahl et al. (2013), "RAMSES-RT: radiation
 * hydrodynamics in the cosmological context".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library; the two are compared element by element.
 *
 * Every routine follows the paper's own order of operations and notation:
 *   - injection           : Sec. 3.1, eq. (injnum) with f_esc = 1 and point
 *                           sources of constant rate
 *   - M1 closure          : Sec. 2, eqs. (edd2), (eddTens), (Udir), with the
 *                           reduced light speed c_r of Sec. 4.1
 *   - transport           : Sec. 3.2, eqs. (dUdt_sol), (hll), (glf); unsplit
 *                           in 3D, all six face fluxes from the source state
 *                           (App. D source/destination copies)
 *   - thermochemistry     : App. A tasks 1-5 (photon SIE update, T_mu update,
 *                           x_HII, He fractions, electron check, 10%/5% rule)
 *   - rate coefficients   : App. E.1-E.3
 * Floating point: IEEE FP64, built with -ffp-contract=off, libm transcendentals.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Physical constants, cgs (CODATA 2018).  Ionisation energies from the
 * photoionisation-threshold table of App. E.4. */
#define OR_KB      1.380649e-16
#define OR_EV      1.602176634e-12
#define OR_EPS_HI   (13.60 * OR_EV)
#define OR_EPS_HEI  (24.59 * OR_EV)
#define OR_EPS_HEII (54.42 * OR_EV)

/* flag bits reported by the chemistry */
#define OR_FLAG_CAP   1u   /* attempt cap reached before dt_RT was filled */
#define OR_FLAG_NAN   2u   /* non-finite value in the result             */
#define OR_FLAG_NNEG  8u   /* negative photon density after the update   */

enum { OR_BC_PERIODIC = 0, OR_BC_OUTFLOW = 1, OR_BC_REFLECT = 2, OR_BC_INFLOW = 3 };
enum { OR_FLUX_GLF = 0, OR_FLUX_HLL = 1 };

typedef struct {
    int nx, ny, nz;
    double dx;
    int bc[6];                 /* -x,+x,-y,+y,-z,+z */
    int M;                     /* photon groups, 1..3 */
    double c_r;                /* reduced light speed [cm/s] */
    double sigN[3][3];         /* [group][HI,HeI,HeII], eq. (csn_multi) */
    double sigE[3][3];         /* eq. (cse_multi) */
    double ebar[3];            /* eq. (egy_multi), erg */
    int flux;                  /* OR_FLUX_* */
    int otsa;                  /* on-the-spot approximation (Sec. 3.3.2) */
    int isothermal;            /* hold T fixed (Iliev test 1) */
    double X, Y;               /* H and He mass fractions */
    double gamma;              /* ratio of specific heats */
    double a_exp;              /* expansion factor in the Compton term */
    double x_min;              /* floor on x_HII */
    double N_floor;            /* densities at or below it skip the 10% check */
    long long max_attempts;    /* cap on chemistry attempts per cell per RT step */
    const double *hll;         /* [nf][nth][2] (lambda_min, lambda_max), c = 1 */
    int hll_nf, hll_nth;
    int brec[3];               /* without OTSA: the group receiving the recombination
                                * photons of HII, HeII, HeIII (b^rec of eq. cool_N_cr),
                                * -1: none */
    double inflow[6][3];       /* OR_BC_INFLOW faces: photon flux [s^-1 cm^-2] per group
                                * entering the box through the face (the Iliev test 3 source) */
} or_params;

/* ======================================================================
 * App. E rate coefficients.  Each returns the value and d/dT.
 * ====================================================================== */
typedef struct { double v, d; } vd;

/* Common form of App. E.1 (collisional ionisation) and the collisional
 * ionisation cooling of E.3:  A sqrt(T) (1 + sqrt(T/1e5))^-1 exp(-Tj/T). */
static vd cen_form(double A, double Tj, double T)
{
    double sq = sqrt(T);
    double g = 1.0 / (1.0 + sqrt(T / 1e5));
    double e = exp(-Tj / T);
    vd r;
    r.v = A * sq * g * e;
    double dsq = 0.5 / sq;
    double dg = -g * g * 0.5 / sqrt(T * 1e5);
    double de = e * Tj / (T * T);
    r.d = A * (dsq * g * e + sq * dg * e + sq * g * de);
    return r;
}

/* Hui & Gnedin form of App. E.2: A lam^p / (1 + (lam/l0)^q)^r, lam = TL/T. */
static vd hg_form(double A, double TL, double p, double l0, double q, double r, double T)
{
    double lam = TL / T;
    double u = pow(lam / l0, q);
    double den = pow(1.0 + u, -r);
    vd o;
    o.v = A * pow(lam, p) * den;
    /* d/dlam then chain with dlam/dT = -lam/T */
    double dl = A * (p * pow(lam, p - 1.0) * den
                     + pow(lam, p) * (-r) * pow(1.0 + u, -r - 1.0) * q * u / lam);
    o.d = dl * (-lam / T);
    return o;
}

/* Recombination-cooling form of App. E.3: B T lam^p / (1 + (lam/l0)^q)^r. */
static vd hg_cool_form(double B, double TL, double p, double l0, double q, double r, double T)
{
    vd h = hg_form(1.0, TL, p, l0, q, r, T);
    vd o;
    o.v = B * T * h.v;
    o.d = B * h.v + B * T * h.d;
    return o;
}

/* power form A lam^p, lam = TL/T */
static vd pw_form(double A, double TL, double p, double T)
{
    double lam = TL / T;
    vd o;
    o.v = A * pow(lam, p);
    o.d = A * p * pow(lam, p - 1.0) * (-lam / T);
    return o;
}

#define TL_HI   315614.0
#define TL_HEI  570670.0
#define TL_HEII 1263030.0

/* E.1 collisional ionisation rates [cm^3 s^-1] */
vd or_beta_HI(double T)   { return cen_form(5.85e-11, 157809.1, T); }
vd or_beta_HeI(double T)  { return cen_form(2.38e-11, 285335.4, T); }
vd or_beta_HeII(double T) { return cen_form(5.68e-12, 631515.0, T); }

/* E.2 recombination rates [cm^3 s^-1] */
vd or_alphaA_HII(double T)   { return hg_form(1.269e-13, TL_HI, 1.503, 0.522, 0.47, 1.923, T); }
vd or_alphaA_HeII(double T)  { return pw_form(3e-14, TL_HEI, 0.654, T); }
vd or_alphaA_HeIII(double T) { return hg_form(2.538e-13, TL_HEII, 1.503, 0.522, 0.47, 1.923, T); }
vd or_alphaB_HII(double T)   { return hg_form(2.753e-14, TL_HI, 1.5, 2.74, 0.407, 2.242, T); }
vd or_alphaB_HeII(double T)  { return pw_form(1.26e-14, TL_HEI, 0.75, T); }
vd or_alphaB_HeIII(double T) { return hg_form(5.506e-14, TL_HEII, 1.5, 2.74, 0.407, 2.242, T); }

/* E.3 cooling rate coefficients [erg cm^3 s^-1] */
vd or_zeta_HI(double T)   { return cen_form(1.27e-21, 157809.1, T); }
vd or_zeta_HeI(double T)  { return cen_form(9.38e-22, 285335.4, T); }
vd or_zeta_HeII(double T) { return cen_form(4.95e-22, 631515.0, T); }

vd or_etaA_HII(double T)   { return hg_cool_form(1.778e-29, TL_HI, 1.965, 0.541, 0.502, 2.697, T); }
vd or_etaA_HeIII(double T) { return hg_cool_form(8.0 * 1.778e-29, TL_HEII, 1.965, 0.541, 0.502, 2.697, T); }
vd or_etaB_HII(double T)   { return hg_cool_form(3.435e-30, TL_HI, 1.97, 2.25, 0.376, 3.72, T); }
vd or_etaB_HeIII(double T) { return hg_cool_form(8.0 * 3.435e-30, TL_HEII, 1.97, 2.25, 0.376, 3.72, T); }
/* eta_HeII = k_B T alpha_HeII (the paper states it this way) */
vd or_etaA_HeII(double T)
{
    vd a = or_alphaA_HeII(T), o;
    o.v = OR_KB * T * a.v;
    o.d = OR_KB * a.v + OR_KB * T * a.d;
    return o;
}
vd or_etaB_HeII(double T)
{
    vd a = or_alphaB_HeII(T), o;
    o.v = OR_KB * T * a.v;
    o.d = OR_KB * a.v + OR_KB * T * a.d;
    return o;
}

/* collisional excitation */
vd or_psi_HI(double T)
{
    double g = 1.0 / (1.0 + sqrt(T / 1e5));
    double e = exp(-118348.0 / T);
    vd o;
    o.v = 7.5e-19 * g * e;
    double dg = -g * g * 0.5 / sqrt(T * 1e5);
    o.d = 7.5e-19 * (dg * e + g * e * 118348.0 / (T * T));
    return o;
}
vd or_psi_HeII(double T)
{
    double tp = pow(T, -0.397);
    double g = 1.0 / (1.0 + sqrt(T / 1e5));
    double e = exp(-473638.0 / T);
    vd o;
    o.v = 5.54e-17 * tp * g * e;
    double dtp = -0.397 * pow(T, -1.397);
    double dg = -g * g * 0.5 / sqrt(T * 1e5);
    double de = e * 473638.0 / (T * T);
    o.d = 5.54e-17 * (dtp * g * e + tp * dg * e + tp * g * de);
    return o;
}

/* bremsstrahlung, per unit of n_e (n_HII + n_HeII + 4 n_HeIII) */
vd or_theta(double T)
{
    vd o;
    o.v = 1.42e-27 * sqrt(T);
    o.d = 1.42e-27 * 0.5 / sqrt(T);
    return o;
}

/* Compton cooling/heating [erg s^-1], per electron */
vd or_varpi(double T, double a)
{
    double Tg = 2.727 / a;
    vd o;
    o.v = 1.017e-37 * pow(Tg, 4.0) * (T - Tg);
    o.d = 1.017e-37 * pow(Tg, 4.0);
    return o;
}

/* dielectronic recombination cooling */
vd or_omega_HeII(double T)
{
    double t15 = pow(T, -1.5);
    double e1 = exp(-470000.0 / T);
    double e2 = exp(-94000.0 / T);
    vd o;
    o.v = 1.24e-13 * t15 * e1 * (1.0 + 0.3 * e2);
    double dt15 = -1.5 * pow(T, -2.5);
    double de1 = e1 * 470000.0 / (T * T);
    double de2 = e2 * 94000.0 / (T * T);
    o.d = 1.24e-13 * (dt15 * e1 * (1.0 + 0.3 * e2) + t15 * de1 * (1.0 + 0.3 * e2)
                      + t15 * e1 * 0.3 * de2);
    return o;
}

/* Rate lookup by id, for the unit tests. */
int or_rate(int id, double T, double a_exp, double *v, double *d)
{
    vd r;
    switch (id) {
    case 0: r = or_beta_HI(T); break;
    case 1: r = or_beta_HeI(T); break;
    case 2: r = or_beta_HeII(T); break;
    case 3: r = or_alphaA_HII(T); break;
    case 4: r = or_alphaA_HeII(T); break;
    case 5: r = or_alphaA_HeIII(T); break;
    case 6: r = or_alphaB_HII(T); break;
    case 7: r = or_alphaB_HeII(T); break;
    case 8: r = or_alphaB_HeIII(T); break;
    case 9: r = or_zeta_HI(T); break;
    case 10: r = or_zeta_HeI(T); break;
    case 11: r = or_zeta_HeII(T); break;
    case 12: r = or_etaA_HII(T); break;
    case 13: r = or_etaA_HeII(T); break;
    case 14: r = or_etaA_HeIII(T); break;
    case 15: r = or_etaB_HII(T); break;
    case 16: r = or_etaB_HeII(T); break;
    case 17: r = or_etaB_HeIII(T); break;
    case 18: r = or_psi_HI(T); break;
    case 19: r = or_psi_HeII(T); break;
    case 20: r = or_theta(T); break;
    case 21: r = or_varpi(T, a_exp); break;
    case 22: r = or_omega_HeII(T); break;
    default: return -1;
    }
    *v = r.v;
    *d = r.d;
    return 0;
}

/* ======================================================================
 * Sec. 2 M1 closure and Sec. 3.2 intercell fluxes.
 * ====================================================================== */

/* Eddington tensor D (row-major 3x3) of eqs. (eddTens), (Udir) at light
 * speed c.  f is capped at 1; for F = 0 the n (x) n term vanishes. */
/* |F| without overflow or underflow of the squares */
static double norm3(const double F[3])
{
    return hypot(hypot(F[0], F[1]), F[2]);
}

void or_eddington(double N, const double F[3], double c, double D[9])
{
    double Fn = norm3(F);
    double f = 0.0;
    if (N > 0.0)
        f = Fn / (c * N);
    else if (Fn > 0.0)
        f = 1.0;
    if (f > 1.0) f = 1.0;
    double chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
    double n[3] = {0.0, 0.0, 0.0};
    if (Fn > 0.0) {
        n[0] = F[0] / Fn;
        n[1] = F[1] / Fn;
        n[2] = F[2] / Fn;
    }
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++)
            D[3 * i + k] = (i == k ? 0.5 * (1.0 - chi) : 0.0) + 0.5 * (3.0 * chi - 1.0) * n[i] * n[k];
}

/* Physical flux along axis d of eq. (dUdt): G = [F_d, c^2 P_d.], P = D N.
 * A cell with N <= 0 carries no pressure, and so does a density so small
 * that 1/(c_r N) overflows: its reduced flux is not representable. */
static void flux_G(int d, const double U[4], double c, double G[4])
{
    G[0] = U[1 + d];
    if (U[0] <= 0.0 || isinf(1.0 / (c * U[0]))) {
        G[1] = G[2] = G[3] = 0.0;
        return;
    }
    double D[9];
    or_eddington(U[0], U + 1, c, D);
    for (int k = 0; k < 3; k++)
        G[1 + k] = c * c * U[0] * D[3 * d + k];
}

/* Jacobian eigenvalue range (c = 1 units) of a cell along axis d, by
 * bilinear interpolation in the (f, theta) table of Sec. 3.2; theta is the
 * angle between F and the +d axis, f in [0,1] and theta in [0,pi] are
 * mapped onto uniform nodes. */
static void hll_eig(const or_params *p, int d, const double U[4], double *lmin, double *lmax)
{
    double Fn = norm3(U + 1);
    double f;
    if (U[0] > 0.0)
        f = Fn / (p->c_r * U[0]);
    else
        f = (Fn > 0.0) ? 1.0 : 0.0;
    if (f > 1.0) f = 1.0;
    double ct = (Fn > 0.0) ? U[1 + d] / Fn : 1.0;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    double th = acos(ct);
    double uf = f * (p->hll_nf - 1);
    double ut = th / M_PI * (p->hll_nth - 1);
    int i = (int)floor(uf), k = (int)floor(ut);
    if (i > p->hll_nf - 2) i = p->hll_nf - 2;
    if (k > p->hll_nth - 2) k = p->hll_nth - 2;
    if (i < 0) i = 0;
    if (k < 0) k = 0;
    double wf = uf - i, wt = ut - k;
    const double *t = p->hll;
    int nt = p->hll_nth;
#define TAB(ii, kk, m) t[(((size_t)(ii) * nt) + (kk)) * 2 + (m)]
    for (int m = 0; m < 2; m++) {
        double v = (1.0 - wf) * (1.0 - wt) * TAB(i, k, m) + wf * (1.0 - wt) * TAB(i + 1, k, m)
                 + (1.0 - wf) * wt * TAB(i, k + 1, m) + wf * wt * TAB(i + 1, k + 1, m);
        if (m == 0) *lmin = v; else *lmax = v;
    }
#undef TAB
}

/* Reduced flux component f cos(theta) of a cell along axis d, with f and
 * theta as the table lookup takes them (f capped at 1; an empty cell with
 * flux is a beam, f = 1). */
static double reduced_flux(const or_params *p, int d, const double U[4])
{
    double Fn = norm3(U + 1);
    if (!(Fn > 0.0)) return 0.0;
    double f;
    if (U[0] > 0.0)
        f = Fn / (p->c_r * U[0]);
    else
        f = 1.0;
    if (f > 1.0) f = 1.0;
    double ct = U[1 + d] / Fn;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    return f * ct;
}

/* The table lookup above, exported for the tests that pin it. */
void or_hll_eig(const or_params *p, int d, const double U[4], double *lmin, double *lmax)
{
    hll_eig(p, d, U, lmin, lmax);
}

/* Intercell flux at the interface between UL (left) and UR (right) along
 * axis d: eq. (glf) or eq. (hll). */
void or_face_flux(const or_params *p, int d, const double UL[4], const double UR[4], double Phi[4])
{
    double GL[4], GR[4];
    double c = p->c_r;
    flux_G(d, UL, c, GL);
    flux_G(d, UR, c, GR);
    if (p->flux == OR_FLUX_GLF) {
        for (int m = 0; m < 4; m++)
            Phi[m] = 0.5 * (GL[m] + GR[m]) - 0.5 * c * (UR[m] - UL[m]);
        return;
    }
    double l0m, l0p, l1m, l1p;
    hll_eig(p, d, UL, &l0m, &l0p);
    hll_eig(p, d, UR, &l1m, &l1p);
    /* The exact eigenvalues of a cell always bracket its reduced flux
     * f cos(theta) = F_d/(c N) (f capped at 1); the bilinear table does not
     * (at f = 1 the chord of cos(theta) between nodes misses it by up to
     * ~1e-4), and a speed range that excludes it lets this flux draw
     * photons out of an empty cell upstream of a beam.  Each cell's range
     * is widened to contain it. */
    double aL = reduced_flux(p, d, UL), aR = reduced_flux(p, d, UR);
    l0m = fmin(l0m, aL);
    l0p = fmax(l0p, aL);
    l1m = fmin(l1m, aR);
    l1p = fmax(l1p, aR);
    double lp = fmax(0.0, fmax(l0p, l1p)) * c;
    double lm = fmin(0.0, fmin(l0m, l1m)) * c;
    if (lp - lm == 0.0) {
        for (int m = 0; m < 4; m++) Phi[m] = 0.5 * (GL[m] + GR[m]);
        return;
    }
    for (int m = 0; m < 4; m++)
        Phi[m] = (lp * GL[m] - lm * GR[m] + lp * lm * (UR[m] - UL[m])) / (lp - lm);
}

/* ======================================================================
 * Transport step (Sec. 3.2), one group at a time.
 * State layout (structure of arrays, x fastest):
 *   N[g*nc + i], F[(3*g + d)*nc + i], i = x + nx*(y + ny*z).
 * ====================================================================== */
static void load_U(const double *N, const double *F, size_t nc, int g, size_t i, double U[4])
{
    U[0] = N[(size_t)g * nc + i];
    for (int d = 0; d < 3; d++) U[1 + d] = F[(size_t)(3 * g + d) * nc + i];
}

/* Neighbour state of cell (ix,iy,iz) at offset s (-1/+1) along axis d,
 * with the boundary conditions of the grid (ghost cells). */
static void neighbour_U(const or_params *p, const double *N, const double *F, int g,
                        int ix, int iy, int iz, int d, int s, double U[4])
{
    int n[3] = {p->nx, p->ny, p->nz};
    int c[3] = {ix, iy, iz};
    int j = c[d] + s;
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    int reflect = 0;
    if (j < 0 || j >= n[d]) {
        int face = 2 * d + (s > 0 ? 1 : 0);
        int bc = p->bc[face];
        if (bc == OR_BC_INFLOW) {
            /* the ghost cell holds a beam entering the box: N = F / c_r
             * (reduced flux 1) with F along the inward normal */
            double f = p->inflow[face][g];
            U[0] = f / p->c_r;
            U[1] = U[2] = U[3] = 0.0;
            U[1 + d] = s < 0 ? f : -f;
            return;
        }
        if (bc == OR_BC_PERIODIC) {
            j = (j + n[d]) % n[d];
        } else {
            j = c[d];
            reflect = (bc == OR_BC_REFLECT);
        }
    }
    c[d] = j;
    size_t i = (size_t)c[0] + (size_t)p->nx * ((size_t)c[1] + (size_t)p->ny * c[2]);
    load_U(N, F, nc, g, i, U);
    if (reflect) U[1 + d] = -U[1 + d];
}

/* After an HLL update a flux above c_r N (reduced flux f > 1, reachable by
 * rounding next to an exact beam) is scaled back to c_r N.  The paper does
 * not say how unrealisable states are treated; left alone, an exact beam
 * entering through a face grows an instability under HLL, whose wave speeds
 * at f = 1 are both +c while the closure capped at f = 1 propagates a
 * backward wave.  A negative photon density (with the widened speeds of
 * or_face_flux only rounding leaves one, next to a beam) empties the cell. */
static void limit_flux(double U[4], double c)
{
    if (U[0] < 0.0) {
        U[0] = U[1] = U[2] = U[3] = 0.0;
        return;
    }
    /* as in the closure, a density so small that 1/(c_r N) overflows counts as empty */
    double icn = 1.0 / (c * U[0]);
    if (!(U[0] > 0.0) || isinf(icn)) return;
    double a[3], a2 = 0.0;
    for (int d = 0; d < 3; d++) {
        a[d] = U[1 + d] * icn;
        a2 += a[d] * a[d];
    }
    if (a2 > 1.0) {
        double s = 1.0 / sqrt(a2);
        for (int d = 0; d < 3; d++) U[1 + d] *= s;
    }
}

/* U' = U + dt/dx * sum_d (Phi_{d,l-1/2} - Phi_{d,l+1/2})   (eq. dUdt_sol),
 * every face flux evaluated from the source state (N, F); the result goes
 * to the destination arrays (Nout, Fout). */
void or_transport(const or_params *p, double dt, const double *N, const double *F,
                  double *Nout, double *Fout)
{
    int nx = p->nx, ny = p->ny, nz = p->nz;
    size_t nc = (size_t)nx * ny * nz;
    double k = dt / p->dx;
    for (int g = 0; g < p->M; g++) {
#pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)nc; i++) {
            int ix = (int)(i % nx);
            int iy = (int)((i / nx) % ny);
            int iz = (int)(i / ((long long)nx * ny));
            double UC[4], UL[4], UR[4], Pm[4], Pp[4], acc[4] = {0, 0, 0, 0};
            load_U(N, F, nc, g, (size_t)i, UC);
            for (int d = 0; d < 3; d++) {
                neighbour_U(p, N, F, g, ix, iy, iz, d, -1, UL);
                neighbour_U(p, N, F, g, ix, iy, iz, d, +1, UR);
                or_face_flux(p, d, UL, UC, Pm);
                or_face_flux(p, d, UC, UR, Pp);
                for (int m = 0; m < 4; m++) acc[m] += Pm[m] - Pp[m];
            }
            double Un[4];
            for (int m = 0; m < 4; m++) Un[m] = UC[m] + k * acc[m];
            if (p->flux == OR_FLUX_HLL) limit_flux(Un, p->c_r);
            Nout[(size_t)g * nc + i] = Un[0];
            for (int d = 0; d < 3; d++) Fout[(size_t)(3 * g + d) * nc + i] = Un[1 + d];
        }
    }
}

/* ======================================================================
 * Injection step (Sec. 3.1, eq. injnum): point sources of constant rate
 * ndot[s*M + g] photons/s, f_esc = 1.  N += ndot dt / V.
 * ====================================================================== */
void or_inject(const or_params *p, double dt, int nsrc, const int *ijk, const double *ndot, double *N)
{
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    double V = p->dx * p->dx * p->dx;
    for (int s = 0; s < nsrc; s++) {
        size_t i = (size_t)ijk[3 * s] + (size_t)p->nx * ((size_t)ijk[3 * s + 1] + (size_t)p->ny * ijk[3 * s + 2]);
        for (int g = 0; g < p->M; g++)
            N[(size_t)g * nc + i] += ndot[(size_t)s * p->M + g] * dt / V;
    }
}

/* ======================================================================
 * Thermochemistry (App. A): one cell over dt_RT, subcycled by the 10% rule.
 * ====================================================================== */

/* mean mass per particle in units of m_H, eq. (mu) */
static double mu_of(const or_params *p, double x, double y2, double y3)
{
    return 1.0 / (p->X * (1.0 + x) + 0.25 * p->Y * (1.0 + y2 + 2.0 * y3));
}

/* primordial cooling rate L of eq. (rate_cooling) [erg cm^-3 s^-1] and dL/dT.
 * Case-B recombination cooling under the OTSA. */
static void cooling(const or_params *p, double T, double ne, double nHI, double nHII,
                    double nHeI, double nHeII, double nHeIII, double *L, double *dL)
{
    vd zHI = or_zeta_HI(T), zHeI = or_zeta_HeI(T), zHeII = or_zeta_HeII(T);
    vd psHI = or_psi_HI(T), psHeII = or_psi_HeII(T);
    vd eHII = p->otsa ? or_etaB_HII(T) : or_etaA_HII(T);
    vd eHeII = p->otsa ? or_etaB_HeII(T) : or_etaA_HeII(T);
    vd eHeIII = p->otsa ? or_etaB_HeIII(T) : or_etaA_HeIII(T);
    vd om = or_omega_HeII(T), th = or_theta(T), cp = or_varpi(T, p->a_exp);
    double brem_n = nHII + nHeII + 4.0 * nHeIII;
    *L = (zHI.v + psHI.v) * ne * nHI
       + zHeI.v * ne * nHeI
       + (zHeII.v + psHeII.v + eHeII.v + om.v) * ne * nHeII
       + eHII.v * ne * nHII
       + eHeIII.v * ne * nHeIII
       + th.v * ne * brem_n
       + cp.v * ne;
    *dL = (zHI.d + psHI.d) * ne * nHI
        + zHeI.d * ne * nHeI
        + (zHeII.d + psHeII.d + eHeII.d + om.d) * ne * nHeII
        + eHII.d * ne * nHII
        + eHeIII.d * ne * nHeIII
        + th.d * ne * brem_n
        + cp.d * ne;
}

/* photoheating rate H of eq. (PHeat2) from the updated photon densities
 * and the backward abundances */
static double heating(const or_params *p, const double *Nn, double nHI, double nHeI, double nHeII)
{
    const double nj[3] = {nHI, nHeI, nHeII};
    const double epsj[3] = {OR_EPS_HI, OR_EPS_HEI, OR_EPS_HEII};
    double H = 0.0;
    for (int j = 0; j < 3; j++) {
        double s = 0.0;
        for (int g = 0; g < p->M; g++)
            s += p->c_r * Nn[g] * (p->ebar[g] * p->sigE[g][j] - epsj[j] * p->sigN[g][j]);
        H += nj[j] * s;
    }
    return H;
}

static double relchg(double a, double b, double floor)
{
    return (b > floor) ? fabs(a - b) / b : 0.0;
}

/* One cell over dt_RT.  N[g], F[g][3] in/out; xs = {x_HII, x_HeII, x_HeIII}
 * in/out; T in/out; nacc/natt: accepted substeps / attempts.  Returns flags. */
unsigned or_thermo_cell_rates(const or_params *p, double dtRT, double nH, double *N, double *F,
                              const double *Nr, const double *Fr, double *xs, double *T, int *nacc, int *natt);

unsigned or_thermo_cell(const or_params *p, double dtRT, double nH, double *N, double *F,
                        double *xs, double *T, int *nacc, int *natt)
{
    return or_thermo_cell_rates(p, dtRT, nH, N, F, NULL, NULL, xs, T, nacc, natt);
}

/* As or_thermo_cell, with the photon-density and flux rates of smoothed RT
 * (Sec. 4.4, eqs. thchem_N_smooth, thchem_F_smooth): Nr[g], Fr[3g+d] are
 * added to the photon equations of App. A task 1 (NULL: none). */
unsigned or_thermo_cell_rates(const or_params *p, double dtRT, double nH, double *N, double *F,
                              const double *Nr, const double *Fr, double *xs, double *T, int *nacc, int *natt)
{
    const int M = p->M;
    const double cr = p->c_r;
    const double nHe = nH * p->Y / (4.0 * p->X);
    /* K converts the thermal-energy rate to a T_mu rate, eq. (ramsesrt_cool1_eq):
     * K = (gamma-1) m_H / (rho k_B) with rho = n_H m_H / X */
    const double K = (p->gamma - 1.0) * p->X / (nH * OR_KB);
    double x = xs[0], y2 = xs[1], y3 = xs[2];
    const double Tiso = *T;
    double Tmu = *T / mu_of(p, x, y2, y3);
    double rem = dtRT, h = dtRT;
    int acc = 0, att = 0;
    unsigned flags = 0;
    /* a cell with a non-finite input is reported and left as it is */
    int finite_in = isfinite(*T) && isfinite(x) && isfinite(y2) && isfinite(y3);
    for (int g = 0; g < M; g++) {
        finite_in = finite_in && isfinite(N[g]) && (!Nr || isfinite(Nr[g]));
        for (int d = 0; d < 3; d++)
            finite_in = finite_in && isfinite(F[3 * g + d]) && (!Fr || isfinite(Fr[3 * g + d]));
    }
    if (!finite_in) {
        *nacc = 0;
        *natt = 0;
        return OR_FLAG_NAN;
    }

    while (rem > 0.0) {
        if (att >= p->max_attempts) { flags |= OR_FLAG_CAP; break; }
        att++;
        /* h <- min(h, time left); a substep that would leave less than
         * 1e-10 of itself undone finishes the RT step instead, so that
         * rounding in the running remainder never adds a sliver substep */
        if (h >= rem * (1.0 - 1e-10)) h = rem;
        double maxrel = 0.0, r;
        int fail = 0;

        /* ---- task 1: photon density and flux, eq. (SIE photons) ---- */
        const double nHI = (1.0 - x) * nH;
        const double nHeI = (1.0 - y2 - y3) * nHe;
        const double nHeII = y2 * nHe;
        const double nHII = x * nH;
        const double nHeIII = y3 * nHe;
        double Nn[3], Fn[3][3];
        /* photons from recombinations straight to the ground state, eq.
         * cool_N_cr, without OTSA (Sec. 3.3.2): (alpha_A - alpha_B) n_j n_e
         * with the state at the start of the substep */
        double Crec[3] = {0.0, 0.0, 0.0};
        if (!p->otsa) {
            const double Tc = p->isothermal ? Tiso : Tmu * mu_of(p, x, y2, y3);
            const double ne = nHII + (y2 + 2.0 * y3) * nHe;
            const double em[3] = {(or_alphaA_HII(Tc).v - or_alphaB_HII(Tc).v) * nHII * ne,
                                  (or_alphaA_HeII(Tc).v - or_alphaB_HeII(Tc).v) * nHeII * ne,
                                  (or_alphaA_HeIII(Tc).v - or_alphaB_HeIII(Tc).v) * nHeIII * ne};
            for (int j = 0; j < 3; j++)
                if (p->brec[j] >= 0 && p->brec[j] < M) Crec[p->brec[j]] += em[j];
        }
        for (int g = 0; g < M; g++) {
            double D = cr * (p->sigN[g][0] * nHI + p->sigN[g][1] * nHeI + p->sigN[g][2] * nHeII);
            /* eq. SIE photons: creation by recombinations and, with
             * smoothing, the transport rate */
            Nn[g] = (N[g] + h * (Crec[g] + (Nr ? Nr[g] : 0.0))) / (1.0 + h * D);
            /* a negative rate can take the smoothed update below zero (its
             * steady state Nr/D is then negative): no photon density is
             * negative, so it stops at zero.  Above N_floor the 10% check
             * below refuses such a substep anyway. */
            if (Nr && Nn[g] < 0.0) Nn[g] = 0.0;
            for (int d = 0; d < 3; d++)
                Fn[g][d] = (Fr ? F[3 * g + d] + h * Fr[3 * g + d] : F[3 * g + d]) / (1.0 + h * D);
            r = relchg(Nn[g], N[g], p->N_floor);
            if (r > 0.1) fail = 1;
            if (r > maxrel) maxrel = r;
        }
        if (fail) { h *= 0.5; continue; }

        /* ---- task 2: thermal update, eq. (T integration num eq 2) ---- */
        const double mu0 = mu_of(p, x, y2, y3);
        const double ne0 = nHII + (y2 + 2.0 * y3) * nHe;
        double Tmun = Tmu;
        if (!p->isothermal) {
            double T0 = Tmu * mu0;
            double H = heating(p, Nn, nHI, nHeI, nHeII);
            double L, dL;
            cooling(p, T0, ne0, nHI, nHII, nHeI, nHeII, nHeIII, &L, &dL);
            double Lam = H - L;           /* Lambda > 0 heats */
            double Lamp = -mu0 * dL;      /* dLambda/dT_mu; heating has no T dependence */
            double den = 1.0 - Lamp * K * h;
            if (den <= 0.0) { h *= 0.5; continue; }
            Tmun = Tmu + Lam * K * h / den;
            r = fabs(Tmun - Tmu) / Tmu;
            if (r > 0.1 || fabs(K * Lam * h) / Tmu > 0.1) { h *= 0.5; continue; }
            if (r > maxrel) maxrel = r;
        }

        /* ---- task 3: hydrogen ionised fraction, eq. (xhii_update_2) ---- */
        double T1 = p->isothermal ? Tiso : Tmun * mu0;
        vd bH = or_beta_HI(T1);
        vd aH = p->otsa ? or_alphaB_HII(T1) : or_alphaA_HII(T1);
        double GamHI = 0.0, GamHeI = 0.0, GamHeII = 0.0;
        for (int g = 0; g < M; g++) {
            GamHI += p->sigN[g][0] * cr * Nn[g];
            GamHeI += p->sigN[g][1] * cr * Nn[g];
            GamHeII += p->sigN[g][2] * cr * Nn[g];
        }
        double C = bH.v * ne0 + GamHI;
        double Dd = aH.v * ne0;
        double dC, dD;
        if (p->isothermal) {
            dC = nH * bH.v;
            dD = nH * aH.v;
        } else {
            dC = nH * bH.v - ne0 * Tmun * mu0 * mu0 * p->X * bH.d;
            dD = nH * aH.v - ne0 * Tmun * mu0 * mu0 * p->X * aH.d;
        }
        double J = dC - (C + Dd) - x * (dC + dD);
        double denx = 1.0 - J * h;
        if (denx <= 0.0) { h *= 0.5; continue; }
        double rate = C - x * (C + Dd);
        double xn = x + h * rate / denx;
        if (xn < p->x_min) xn = p->x_min;
        if (xn > 1.0) xn = 1.0;
        r = fabs(xn - x) / x;
        if (r > 0.1 || fabs(rate) * h / x > 0.1) { h *= 0.5; continue; }
        if (r > maxrel) maxrel = r;

        /* ---- task 4: helium fractions, eqs. (xhei_update), (xheii_update),
         * (xheiii_update) and the He conservation fix ---- */
        double y2n = y2, y3n = y3;
        if (nHe > 0.0) {
            double mu1 = mu_of(p, xn, y2, y3);
            double ne1 = xn * nH + (y2 + 2.0 * y3) * nHe;
            double T2 = p->isothermal ? Tiso : Tmun * mu1;
            vd aHe2 = p->otsa ? or_alphaB_HeII(T2) : or_alphaA_HeII(T2);
            vd aHe3 = p->otsa ? or_alphaB_HeIII(T2) : or_alphaA_HeIII(T2);
            vd bHe1 = or_beta_HeI(T2), bHe2 = or_beta_HeII(T2);
            double y1 = 1.0 - y2 - y3;
            /* HeI: created by HeII recombination, destroyed by collisional
             * and photo-ionisation */
            double Ch = y2 * aHe2.v * ne1;
            double Dh = bHe1.v * ne1 + GamHeI;
            double y1n = (y1 + Ch * h) / (1.0 + Dh * h);
            /* HeII */
            Ch = y1n * (bHe1.v * ne1 + GamHeI) + y3 * aHe3.v * ne1;
            Dh = (bHe2.v + aHe2.v) * ne1 + GamHeII;
            y2n = (y2 + Ch * h) / (1.0 + Dh * h);
            /* HeIII, with n_e and mu refreshed for the new HeII */
            double mu2 = mu_of(p, xn, y2n, y3);
            double ne2 = xn * nH + (y2n + 2.0 * y3) * nHe;
            double T3 = p->isothermal ? Tiso : Tmun * mu2;
            vd bHe2b = or_beta_HeII(T3);
            vd aHe3b = p->otsa ? or_alphaB_HeIII(T3) : or_alphaA_HeIII(T3);
            Ch = y2n * (bHe2b.v * ne2 + GamHeII);
            Dh = aHe3b.v * ne2;
            y3n = (y3 + Ch * h) / (1.0 + Dh * h);
            /* x_HeI + x_HeII + x_HeIII = 1 by lowering the largest; no
             * change when HeI is the largest (ties: HeI, then HeII) */
            double S = y1n + y2n + y3n;
            if (y1n >= y2n && y1n >= y3n) {
                /* no update */
            } else if (y2n >= y3n) {
                y2n -= (S - 1.0);
            } else {
                y3n -= (S - 1.0);
            }
        }

        /* ---- electron-density check ---- */
        double nen = xn * nH + (y2n + 2.0 * y3n) * nHe;
        r = fabs(nen - ne0) / ne0;
        if (r > 0.1) { h *= 0.5; continue; }
        if (r > maxrel) maxrel = r;

        /* ---- accept; task 5: double the next substep below 5% ---- */
        for (int g = 0; g < M; g++) {
            N[g] = Nn[g];
            for (int d = 0; d < 3; d++) F[3 * g + d] = Fn[g][d];
        }
        x = xn;
        y2 = y2n;
        y3 = y3n;
        if (p->isothermal)
            Tmu = Tiso / mu_of(p, x, y2, y3);
        else
            Tmu = Tmun;
        rem -= h;
        acc++;
        if (maxrel < 0.05) h *= 2.0;
    }
    xs[0] = x;
    xs[1] = y2;
    xs[2] = y3;
    *T = p->isothermal ? Tiso : Tmu * mu_of(p, x, y2, y3);
    for (int g = 0; g < M; g++) {
        if (N[g] < 0.0) flags |= OR_FLAG_NNEG;
        if (!isfinite(N[g])) flags |= OR_FLAG_NAN;
    }
    if (!isfinite(*T) || !isfinite(x)) flags |= OR_FLAG_NAN;
    *nacc = acc;
    *natt = att;
    return flags;
}

/* Thermochemistry over the whole grid.  nacc/natt may be NULL. */
/* Thermochemistry over the whole grid, with the smoothed-RT rates
 * Nr[g*nc + i], Fr[(3g+d)*nc + i] when they are not NULL.  nacc/natt may be NULL. */
unsigned or_thermochem_rates(const or_params *p, double dt, double *N, double *F, const double *Nr,
                             const double *Fr, double *xHII, double *xHeII, double *xHeIII, double *T,
                             const double *nH, int *nacc, int *natt)
{
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    unsigned flags = 0;
    const int M = p->M;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : flags)
    for (long long i = 0; i < (long long)nc; i++) {
        double Nc[3], Fc[9], Nrc[3], Frc[9], xs[3], Tc;
        for (int g = 0; g < M; g++) {
            Nc[g] = N[(size_t)g * nc + i];
            for (int d = 0; d < 3; d++) Fc[3 * g + d] = F[(size_t)(3 * g + d) * nc + i];
            if (Nr) Nrc[g] = Nr[(size_t)g * nc + i];
            if (Fr)
                for (int d = 0; d < 3; d++) Frc[3 * g + d] = Fr[(size_t)(3 * g + d) * nc + i];
        }
        xs[0] = xHII[i];
        xs[1] = xHeII[i];
        xs[2] = xHeIII[i];
        Tc = T[i];
        int a, t;
        flags |= or_thermo_cell_rates(p, dt, nH[i], Nc, Fc, Nr ? Nrc : NULL, Fr ? Frc : NULL, xs, &Tc, &a, &t);
        for (int g = 0; g < M; g++) {
            N[(size_t)g * nc + i] = Nc[g];
            for (int d = 0; d < 3; d++) F[(size_t)(3 * g + d) * nc + i] = Fc[3 * g + d];
        }
        xHII[i] = xs[0];
        xHeII[i] = xs[1];
        xHeIII[i] = xs[2];
        T[i] = Tc;
        if (nacc) nacc[i] = a;
        if (natt) natt[i] = t;
    }
    return flags;
}

unsigned or_thermochem(const or_params *p, double dt, double *N, double *F, double *xHII,
                       double *xHeII, double *xHeIII, double *T, const double *nH,
                       int *nacc, int *natt)
{
    return or_thermochem_rates(p, dt, N, F, NULL, NULL, xHII, xHeII, xHeIII, T, nH, nacc, natt);
}

/* Transport and thermochemistry of selected cells only (for sampled checks
 * of large grids): for each listed cell, the transport of every group from
 * the source arrays (N, F: already injected), then its thermochemistry.
 * Outputs per listed cell: Nout[c*M+g], Fout[(c*M+g)*3+d], xs[c*3+0..2],
 * Tout[c], nacc[c], natt[c].  Returns the OR of the chemistry flags. */
unsigned or_step_cells_smooth(const or_params *p, double dt, const double *N, const double *F,
                              const double *Npre, const double *xHII, const double *xHeII, const double *xHeIII,
                              const double *T, const double *nH, int ncells, const long long *cells, double *Nout,
                              double *Fout, double *xs, double *Tout, int *nacc, int *natt);

unsigned or_step_cells(const or_params *p, double dt, const double *N, const double *F, const double *xHII,
                       const double *xHeII, const double *xHeIII, const double *T, const double *nH, int ncells,
                       const long long *cells, double *Nout, double *Fout, double *xs, double *Tout, int *nacc,
                       int *natt)
{
    return or_step_cells_smooth(p, dt, N, F, NULL, xHII, xHeII, xHeIII, T, nH, ncells, cells, Nout, Fout, xs, Tout,
                                nacc, natt);
}

/* As or_step_cells; with Npre (layout of N: the photon densities before the
 * injection) the step is smoothed (Sec. 4.4): the chemistry starts from
 * Npre and the source flux F and takes the transport result as rates. */
unsigned or_step_cells_smooth(const or_params *p, double dt, const double *N, const double *F,
                              const double *Npre, const double *xHII, const double *xHeII, const double *xHeIII,
                              const double *T, const double *nH, int ncells, const long long *cells, double *Nout,
                              double *Fout, double *xs, double *Tout, int *nacc, int *natt)
{
    int nx = p->nx, ny = p->ny;
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    double k = dt / p->dx;
    unsigned flags = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
    for (int c = 0; c < ncells; c++) {
        long long i = cells[c];
        int ix = (int)(i % nx);
        int iy = (int)((i / nx) % ny);
        int iz = (int)(i / ((long long)nx * ny));
        double Nc[3], Fc[9], x3[3], Tc;
        for (int g = 0; g < p->M; g++) {
            double UC[4], UL[4], UR[4], Pm[4], Pp[4], acc[4] = {0, 0, 0, 0};
            load_U(N, F, nc, g, (size_t)i, UC);
            for (int d = 0; d < 3; d++) {
                neighbour_U(p, N, F, g, ix, iy, iz, d, -1, UL);
                neighbour_U(p, N, F, g, ix, iy, iz, d, +1, UR);
                or_face_flux(p, d, UL, UC, Pm);
                or_face_flux(p, d, UC, UR, Pp);
                for (int m = 0; m < 4; m++) acc[m] += Pm[m] - Pp[m];
            }
            double Un[4];
            for (int m = 0; m < 4; m++) Un[m] = UC[m] + k * acc[m];
            if (p->flux == OR_FLUX_HLL) limit_flux(Un, p->c_r);
            Nc[g] = Un[0];
            for (int d = 0; d < 3; d++) Fc[3 * g + d] = Un[1 + d];
        }
        x3[0] = xHII[i];
        x3[1] = xHeII[i];
        x3[2] = xHeIII[i];
        Tc = T[i];
        int a, t;
        if (Npre) {
            /* eqs. smoothrate1, smoothrate2 */
            double Nr[3], Fr[9];
            for (int g = 0; g < p->M; g++) {
                double N0 = Npre[(size_t)g * nc + (size_t)i];
                Nr[g] = (Nc[g] - N0) / dt;
                Nc[g] = N0;
                for (int d = 0; d < 3; d++) {
                    double F0 = F[(size_t)(3 * g + d) * nc + (size_t)i];
                    Fr[3 * g + d] = (Fc[3 * g + d] - F0) / dt;
                    Fc[3 * g + d] = F0;
                }
            }
            flags |= or_thermo_cell_rates(p, dt, nH[i], Nc, Fc, Nr, Fr, x3, &Tc, &a, &t);
        } else {
            flags |= or_thermo_cell(p, dt, nH[i], Nc, Fc, x3, &Tc, &a, &t);
        }
        for (int g = 0; g < p->M; g++) {
            Nout[(size_t)c * p->M + g] = Nc[g];
            for (int d = 0; d < 3; d++) Fout[((size_t)c * p->M + g) * 3 + d] = Fc[3 * g + d];
        }
        for (int q = 0; q < 3; q++) xs[(size_t)c * 3 + q] = x3[q];
        Tout[c] = Tc;
        nacc[c] = a;
        natt[c] = t;
    }
    return flags;
}

/* Courant-limited RT time step, Sec. 4.1 with the Courant factor of the tests */
double or_courant_dt(double dx, double c_r, double courant)
{
    return courant * dx / (3.0 * c_r);
}

/* set the number of threads of the oracle's parallel loops */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* threads the oracle's parallel loops use */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================
 * Diagnostics of a step (the photon budget of the operator split, Sec. 3):
 * photons per group, ionised hydrogen, largest reduced flux, smallest
 * photon density, and the photons carried through the boundary faces.
 * ====================================================================== */

/* out[0..2]: sum over cells of N_g dx^3 (groups >= M: 0); out[3]: sum of
 * x_HII n_H dx^3; out[4]: max over cells and groups with N > 0 of
 * |F|/(c_r N); out[5]: min over cells and groups of N.  Plain loops in
 * cell order. */
void or_diagnostics(const or_params *p, const double *N, const double *F, const double *xHII,
                    const double *nH, double *out)
{
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    double V = p->dx * p->dx * p->dx;
    double ph[3] = {0.0, 0.0, 0.0}, ion = 0.0, maxf = 0.0, minN = INFINITY;
    for (int g = 0; g < p->M; g++) {
        for (size_t i = 0; i < nc; i++) {
            double n = N[(size_t)g * nc + i];
            double Fv[3];
            for (int d = 0; d < 3; d++) Fv[d] = F[(size_t)(3 * g + d) * nc + i];
            ph[g] += n;
            if (n < minN) minN = n;
            if (n > 0.0) {
                double f = norm3(Fv) / (p->c_r * n);
                if (f > maxf) maxf = f;
            }
        }
    }
    for (size_t i = 0; i < nc; i++) ion += xHII[i] * nH[i];
    for (int g = 0; g < 3; g++) out[g] = ph[g] * V;
    out[3] = ion * V;
    out[4] = maxf;
    out[5] = minN;
}

/* Photons that one transport step of length dt carries out of the grid
 * through its boundary (non-periodic) faces, per group: the N component
 * of the face flux (eq. glf or hll, against the ghost cell of the face's
 * boundary condition) times the face area dx^2 and dt, counted positive
 * outwards (an inflow face counts its entering beam negative).  out[g],
 * groups >= M: 0.  N, F: the state the transport starts from. */
void or_boundary_outflow(const or_params *p, double dt, const double *N, const double *F, double *out)
{
    int n[3] = {p->nx, p->ny, p->nz};
    size_t nc = (size_t)p->nx * p->ny * p->nz;
    for (int g = 0; g < 3; g++) out[g] = 0.0;
    for (int g = 0; g < p->M; g++) {
        double sum = 0.0;
        for (int d = 0; d < 3; d++) {
            for (int side = 0; side < 2; side++) {
                if (p->bc[2 * d + side] == OR_BC_PERIODIC) continue;
                int c[3];
                /* every cell of the face layer */
                int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
                for (int j2 = 0; j2 < n[a2]; j2++)
                    for (int j1 = 0; j1 < n[a1]; j1++) {
                        c[d] = side ? n[d] - 1 : 0;
                        c[a1] = j1;
                        c[a2] = j2;
                        size_t i = (size_t)c[0] + (size_t)p->nx * ((size_t)c[1] + (size_t)p->ny * c[2]);
                        double UC[4], UG[4], Phi[4];
                        load_U(N, F, nc, g, i, UC);
                        neighbour_U(p, N, F, g, c[0], c[1], c[2], d, side ? +1 : -1, UG);
                        if (side) {
                            or_face_flux(p, d, UC, UG, Phi);
                            sum += Phi[0];
                        } else {
                            or_face_flux(p, d, UG, UC, Phi);
                            sum -= Phi[0];
                        }
                    }
            }
        }
        out[g] = sum * dt * p->dx * p->dx;
    }
}
