// rt_api.hip -- the C ABI of include/rtm1.h: validation, library tables
// (HLL eigenvalues, sources, statistics), and the launch sequence of the
// operator-split RT step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rt_internal.h"
#include "rtm1.h"

using namespace rtm1;

struct rt_ctx {
    int device = 0;            // the HIP device current at rt_init
    KGrid grid;
    rt_groups groups;
    rt_params params;
    KChem kchem;
    KChem *dkchem = nullptr;   // device copy read by the chemistry kernels
    bool fp32 = false;
    int nf = 101, nth = 101;
    std::vector<double> hll_host;
    void *hll_dev = nullptr;
    rt_state st;
    bool bound = false;
    int cur = 0;
    hipStream_t stream = nullptr;
    int nsrc = 0;
    int32_t *src_cell = nullptr;
    double *src_rate = nullptr;
    int nsrc_in = 0;                 // sources as given (for the injection adjoint)
    int32_t *src_in_cell = nullptr;
    double *src_in_rate = nullptr;   // group-0 rate of each given source
    // smoothed RT: source index per cell, each source cell's N before the
    // injection, and where the step stands (0: nothing yet, 1: injected,
    // 2: transported; injected says whether 1 preceded 2)
    double *src_prev = nullptr;
    int sm_phase = 0;
    bool sm_injected = false;
    // expansion factor of the super-comoving state (Sec. 5.4); 1: static box
    double a_cosmo = 1.0;
    DevStats *dstats = nullptr;
    RedOut *dred = nullptr;
    unsigned qcap = 0;               // chemistry queue capacity (cells)
    unsigned qcap_max = 0;           // capacity the scratch size is computed for
    int head_attempts = HEAD_ATTEMPTS;
    int chem_path = RT_CHEM_AUTO;     // chemistry after a separate transport: one pass or head + tail
    // kernel arrangement of the transport (rt_set_transport_path) and the
    // transport blocks whose accounting partials the step's ledger sums
    int path = RT_PATH_AUTO;
    unsigned acct_nblk = 0;
    // photon accounting
    bool acct = false;
    bool acct_pending = false;       // transport partials of the current step
    double injected[3] = {0, 0, 0};  // photons injected since the last reset (host sum)
    std::vector<double> src_rate_host;
    // kernel timing
    bool timing = false;
    struct Pend {
        hipEvent_t a, b;
        int cls;
    };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> pool;
    double t_ms[RT_TIMING_CLASSES] = {};
    long long t_n[RT_TIMING_CLASSES] = {};
    std::string err;
};

enum { TM_INJECT = 0, TM_TRANSPORT = 1, TM_HEAD = 2, TM_TAIL = 3, TM_OTHER = 4, TM_ACCT = 5 };

static hipEvent_t ev_take(rt_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void fold_timing(rt_ctx *c)
{
    if (c->pend.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pend) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->t_ms[p.cls] += ms;
            c->t_n[p.cls] += 1;
        }
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pend.clear();
}

// run f() between two events of class cls when timing is on
template <class Fn>
static rt_status timed(rt_ctx *c, int cls, Fn f)
{
    if (!c->timing) return f();
    if (c->pend.size() > 20000) fold_timing(c);
    hipEvent_t a = ev_take(c), b = ev_take(c);
    if (!a || !b) return f();
    (void)hipEventRecord(a, c->stream);
    rt_status r = f();
    (void)hipEventRecord(b, c->stream);
    c->pend.push_back({a, b, cls});
    return r;
}

static thread_local std::string g_init_err;

#define RT_FAIL(ctx, code, ...)                                                    \
    do {                                                                           \
        char _b[512];                                                              \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                                     \
        (ctx)->err = _b;                                                           \
        return code;                                                               \
    } while (0)

#define RT_HIP(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t _e = (call);                                                                    \
        if (_e != hipSuccess)                                                                      \
            RT_FAIL(ctx, RT_EHIP, "%s failed: %s", #call, hipGetErrorString(_e));                 \
    } while (0)

// ---------------------------------------------------------------------------
// Scratch of rt_step_noalloc: one file-scope device array of a fixed size;
// every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host it
// stands for no device address): rt_init looks up its address on the
// context's device once per device and keeps it in g_noalloc_ptr.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_noalloc_mu;

// the address of this device's array (looked up on first use of the device)
static hipError_t noalloc_setup(int dev)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = ptr;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// HLL eigenvalue table (Sec. 3.2).  Extreme eigenvalues of the M1 flux
// Jacobian dG_x/dU at c = 1, N = 1, F = f (cos t, sin t, 0).  With
// s = f^2, a(s) = (1-chi)/2 and b(s) = (3chi-1)/(2s) the pressure row is
// P_xj = a N d_xj + b F_x F_j / N, whose derivatives give the Jacobian in
// closed form.  The z-flux mode decouples with speed b f cos t; it is also
// a root of the (E, F_x, F_y) block, whose other two roots follow from the
// block's trace and principal minors.  The f = 1 row (a beam) is the limit
// where all speeds equal cos t.
// ---------------------------------------------------------------------------
static void hll_speeds_closed_form(double f, double t, double &lmin, double &lmax)
{
    const double s = f * f;
    const double r = std::sqrt(4.0 - 3.0 * s);
    const double q = 5.0 + 2.0 * r;
    const double chi = (3.0 + 4.0 * s) / q;
    const double chis = (4.0 * q + (3.0 + 4.0 * s) * 3.0 / r) / (q * q);
    const double a = 0.5 * (1.0 - chi);
    const double ap = -0.5 * chis;
    const double b = (3.0 / (2.0 + r) + 6.0) / q;
    const double drds = -1.5 / r;
    const double bp = drds * (-3.0 * q / ((2.0 + r) * (2.0 + r)) - 2.0 * (3.0 / (2.0 + r) + 6.0)) / (q * q);
    const double fx = f * std::cos(t), fy = f * std::sin(t);
    double J[3][3];
    J[0][0] = 0.0;
    J[0][1] = 1.0;
    J[0][2] = 0.0;
    J[1][0] = a - 2.0 * s * ap + fx * fx * (-b - 2.0 * s * bp);
    J[1][1] = 2.0 * ap * fx + 2.0 * b * fx + 2.0 * bp * fx * fx * fx;
    J[1][2] = 2.0 * ap * fy + 2.0 * bp * fx * fx * fy;
    J[2][0] = fx * fy * (-b - 2.0 * s * bp);
    J[2][1] = b * fy + 2.0 * bp * fx * fx * fy;
    J[2][2] = b * fx + 2.0 * bp * fx * fy * fy;
    const double lz = b * fx;
    const double S = J[0][0] + J[1][1] + J[2][2] - lz;
    const double M2 = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) + (J[0][0] * J[2][2] - J[0][2] * J[2][0]) +
                      (J[1][1] * J[2][2] - J[1][2] * J[2][1]);
    const double P = M2 - lz * S;
    double disc = 0.25 * S * S - P;
    disc = disc > 0.0 ? std::sqrt(disc) : 0.0;
    const double lm = 0.5 * S - disc, lp = 0.5 * S + disc;
    lmin = lm < lz ? lm : lz;
    lmax = lp > lz ? lp : lz;
}

static void build_hll(int nf, int nth, std::vector<double> &tab)
{
    tab.assign((size_t)nf * nth * 2, 0.0);
    for (int i = 0; i < nf; ++i) {
        const double f = (double)i / (nf - 1);
        for (int k = 0; k < nth; ++k) {
            const double t = M_PI * (double)k / (nth - 1);
            double lo, hi;
            if (i == nf - 1) {
                lo = hi = std::cos(t);
            } else {
                hll_speeds_closed_form(f, t, lo, hi);
            }
            tab[((size_t)i * nth + k) * 2 + 0] = lo;
            tab[((size_t)i * nth + k) * 2 + 1] = hi;
        }
    }
}

// ---------------------------------------------------------------------------
// Group attributes (Sec. 2, eqs. csn_multi, egy_multi, cse_multi) of a
// blackbody by composite Gauss-Legendre quadrature in ln(energy), panels
// split at the ionisation thresholds; the open last group is cut where the
// Planck factor has fallen by e^-200.
// ---------------------------------------------------------------------------
static const double EPS_ION[3] = {13.60, 24.59, 54.42};
// Verner et al. (1996) parameters of App. E.4 (HeI eps0 = 13.61 eV)
static const double VER[3][7] = {{0.4298, 5.475e-14, 2.963, 32.88, 0.0, 0.0, 0.0},
                                 {13.61, 9.492e-16, 3.188, 1.469, 2.039, 0.4434, 2.136},
                                 {1.720, 1.369e-14, 2.963, 32.88, 0.0, 0.0, 0.0}};

static double verner(double e, int j)
{
    if (e < EPS_ION[j]) return 0.0;
    const double *p = VER[j];
    const double x = e / p[0] - p[5];
    const double y = std::sqrt(x * x + p[6] * p[6]);
    return p[1] * ((x - 1.0) * (x - 1.0) + p[4] * p[4]) * std::pow(y, 0.5 * p[2] - 5.5) *
           std::pow(1.0 + std::sqrt(y / p[3]), -p[2]);
}

static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// integral over [a,b] (eV) of e^k J(e)/e^? ... : returns {photons, energy,
// sigma_j * photons (3), sigma_j * energy (3)}
static void bb_moments(double kT, double a, double b, double out[8])
{
    for (int q = 0; q < 8; ++q) out[q] = 0.0;
    std::vector<double> pts;
    pts.push_back(a);
    for (double e : EPS_ION)
        if (e > a && e < b) pts.push_back(e);
    pts.push_back(b);
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    for (size_t s = 0; s + 1 < pts.size(); ++s) {
        const double la = std::log(pts[s]), lb = std::log(pts[s + 1]);
        const int npan = 96;
        for (int p = 0; p < npan; ++p) {
            const double l0 = la + (lb - la) * p / npan, l1 = la + (lb - la) * (p + 1) / npan;
            const double hm = 0.5 * (l1 - l0), cm = 0.5 * (l1 + l0);
            for (size_t k = 0; k < gx.size(); ++k) {
                const double l = cm + hm * gx[k];
                const double e = std::exp(l);
                const double u = e / kT;
                if (u > 700.0) continue;
                // J(e) de = e^3/(exp(e/kT)-1) de, de = e dl
                const double J = e * e * e / std::expm1(u) * e * hm * gw[k];
                const double Jn = J / e;
                out[0] += Jn;
                out[1] += J;
                for (int j = 0; j < 3; ++j) {
                    const double sg = verner(e, j);
                    out[2 + j] += sg * Jn;
                    out[5 + j] += sg * J;
                }
            }
        }
    }
}

extern "C" rt_status rt_group_attributes(double T_bb, int M, const double *edges_eV, double sigN[3][3],
                                         double sigE[3][3], double ebar[3], double frac[3])
{
    if (!(T_bb > 0) || M < 1 || M > 3 || !edges_eV || !sigN || !sigE || !ebar || !frac) return RT_EINVAL;
    for (int g = 0; g < M; ++g)
        if (!(edges_eV[g + 1] > edges_eV[g]) || !(edges_eV[g] > 0)) return RT_EINVAL;
    const double kT = 8.617333262e-5 * T_bb;
    const double EVE = 1.602176634e-12;
    for (int g = 0; g < 3; ++g) {
        ebar[g] = frac[g] = 0.0;
        for (int j = 0; j < 3; ++j) sigN[g][j] = sigE[g][j] = 0.0;
    }
    double mom[3][8];
    double ntot = 0.0;
    for (int g = 0; g < M; ++g) {
        double a = edges_eV[g], b = edges_eV[g + 1];
        if (!std::isfinite(b) || b > a + 200.0 * kT) b = std::isfinite(b) ? std::fmin(b, a + 200.0 * kT) : a + 200.0 * kT;
        bb_moments(kT, a, b, mom[g]);
        ntot += mom[g][0];
    }
    for (int g = 0; g < M; ++g) {
        frac[g] = mom[g][0] / ntot;
        ebar[g] = mom[g][1] / mom[g][0] * EVE;
        for (int j = 0; j < 3; ++j) {
            sigN[g][j] = mom[g][2 + j] / mom[g][0];
            sigE[g][j] = mom[g][5 + j] / mom[g][1];
        }
    }
    return RT_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static rt_status validate(const rt_grid *g, const rt_groups *gr, const rt_params *p, std::string &err)
{
    char b[256];
    if (!g || !gr || !p) { err = "null argument"; return RT_EINVAL; }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) { err = "grid dimensions must be >= 1"; return RT_EINVAL; }
    if ((double)g->nx * g->ny * g->nz > 2.0e9) { err = "grid too large (> 2e9 cells)"; return RT_EINVAL; }
    if (!(g->dx > 0) || !std::isfinite(g->dx)) { err = "dx must be positive"; return RT_EINVAL; }
    for (int f = 0; f < 6; ++f)
        if (g->bc[f] < 0 || g->bc[f] > 3) { snprintf(b, sizeof b, "bc[%d] invalid", f); err = b; return RT_EINVAL; }
    for (int d = 0; d < 3; ++d)
        if ((g->bc[2 * d] == RT_BC_PERIODIC) != (g->bc[2 * d + 1] == RT_BC_PERIODIC)) {
            snprintf(b, sizeof b, "axis %d: periodic must be set on both faces", d);
            err = b;
            return RT_EINVAL;
        }
    if (gr->M < 1 || gr->M > 3) { err = "M must be 1..3"; return RT_EINVAL; }
    if (!(gr->c_r > 0)) { err = "c_r must be positive"; return RT_EINVAL; }
    for (int i = 0; i < gr->M; ++i) {
        if (!(gr->ebar[i] >= 0)) { err = "ebar must be >= 0"; return RT_EINVAL; }
        for (int j = 0; j < 3; ++j)
            if (!(gr->sigN[i][j] >= 0) || !(gr->sigE[i][j] >= 0)) { err = "cross sections must be >= 0"; return RT_EINVAL; }
    }
    if (p->flux != RT_FLUX_GLF && p->flux != RT_FLUX_HLL) { err = "flux must be GLF or HLL"; return RT_EINVAL; }
    if (p->otsa != 0 && p->otsa != 1) { err = "otsa must be 0 or 1"; return RT_EINVAL; }
    if (!p->otsa)
        for (int j = 0; j < 3; ++j)
            if (gr->brec[j] < -1 || gr->brec[j] >= gr->M) {
                snprintf(b, sizeof b, "brec[%d] must be -1 or a group index below M", j);
                err = b;
                return RT_EINVAL;
            }
    if (p->prec != RT_PREC_FP64 && p->prec != RT_PREC_FP32_TRANSPORT) { err = "prec invalid"; return RT_EINVAL; }
    if (!(p->X > 0) || !(p->Y >= 0) || p->X + p->Y > 1.0 + 1e-12) { err = "need X > 0, Y >= 0, X + Y <= 1"; return RT_EINVAL; }
    if (!(p->gamma > 1)) { err = "gamma must be > 1"; return RT_EINVAL; }
    if (!(p->a_exp > 0)) { err = "a_exp must be > 0"; return RT_EINVAL; }
    if (!(p->x_min > 0) || !(p->x_min < 1)) { err = "x_min must be in (0,1)"; return RT_EINVAL; }
    if (!(p->N_floor >= 0)) { err = "N_floor must be >= 0"; return RT_EINVAL; }
    if (p->max_attempts < 1) { err = "max_attempts must be >= 1"; return RT_EINVAL; }
    if (p->smooth != 0 && p->smooth != 1) { err = "smooth must be 0 or 1"; return RT_EINVAL; }
    return RT_OK;
}

extern "C" rt_status rt_init(const rt_grid *grid, const rt_groups *groups, const rt_params *params, rt_ctx **out)
{
    if (!out) return RT_EINVAL;
    *out = nullptr;
    std::string err;
    rt_status v = validate(grid, groups, params, err);
    if (v != RT_OK) {
        g_init_err = err;
        return v;
    }
    int dev = 0;
    {
        hipError_t e0 = hipGetDevice(&dev);
        if (e0 == hipSuccess) e0 = noalloc_setup(dev);
        if (e0 != hipSuccess) {
            g_init_err = std::string("device set-up failed: ") + hipGetErrorString(e0);
            return RT_EHIP;
        }
    }
    rt_ctx *c = new rt_ctx();
    c->device = dev;
    c->grid.nx = grid->nx;
    c->grid.ny = grid->ny;
    c->grid.nz = grid->nz;
    for (int f = 0; f < 6; ++f) c->grid.bc[f] = grid->bc[f];
    c->grid.ncell = (size_t)grid->nx * grid->ny * grid->nz;
    c->grid.dx = grid->dx;
    memset(c->grid.inflow, 0, sizeof c->grid.inflow);
    c->groups = *groups;
    c->params = *params;
    c->fp32 = params->prec == RT_PREC_FP32_TRANSPORT;
    KChem &k = c->kchem;
    k.M = groups->M;
    k.isothermal = params->isothermal ? 1 : 0;
    k.cr = groups->c_r;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            k.sN[i][j] = i < groups->M ? groups->sigN[i][j] : 0.0;
            k.sE[i][j] = i < groups->M ? groups->sigE[i][j] : 0.0;
        }
        k.eb[i] = i < groups->M ? groups->ebar[i] : 0.0;
    }
    k.X = params->X;
    k.Y = params->Y;
    k.Kfac = (params->gamma - 1.0) * params->X / 1.380649e-16;
    k.a_exp = params->a_exp;
    k.x_min = params->x_min;
    k.N_floor = params->N_floor;
    k.max_att = params->max_attempts;
    k.otsa = params->otsa;
    for (int g = 0; g < 3; ++g)
        for (int j = 0; j < 3; ++j) k.brec[g][j] = (!params->otsa && groups->brec[j] == g) ? 1.0 : 0.0;
    kchem_derive(k);

    build_hll(c->nf, c->nth, c->hll_host);
    hipError_t e;
    const size_t ntab = c->hll_host.size();
    if (c->fp32) {
        std::vector<float> tf(ntab);
        for (size_t i = 0; i < ntab; ++i) tf[i] = (float)c->hll_host[i];
        e = hipMalloc(&c->hll_dev, ntab * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(c->hll_dev, tf.data(), ntab * sizeof(float), hipMemcpyHostToDevice);
    } else {
        e = hipMalloc(&c->hll_dev, ntab * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(c->hll_dev, c->hll_host.data(), ntab * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&c->dstats, sizeof(DevStats));
    if (e == hipSuccess) e = hipMemset(c->dstats, 0, sizeof(DevStats));
    if (e == hipSuccess) e = hipMalloc((void **)&c->dred, sizeof(RedOut));
    if (e == hipSuccess) e = hipMalloc((void **)&c->dkchem, sizeof(KChem));
    if (e == hipSuccess) e = hipMemcpy(c->dkchem, &c->kchem, sizeof(KChem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        g_init_err = std::string("device table allocation failed: ") + hipGetErrorString(e);
        rt_free(c);
        return RT_ENOMEM;
    }
    memset(&c->st, 0, sizeof(c->st));
    {
        // queue for the cells still subcycling after the head pass: room
        // for every cell, so that no cell has to finish in the head pass
        const size_t cap = c->grid.ncell;
        c->qcap = (unsigned)cap;
        c->qcap_max = (unsigned)cap;
    }
    *out = c;
    return RT_OK;
}

// per-cell attempt counts of the previous chemistry pass (one byte per cell)
static size_t prev_att_bytes(const rt_ctx *c) { return (c->grid.ncell + 255) & ~(size_t)255; }

// smoothed RT: the source index of every cell (int32, -1: none)
static size_t src_map_bytes(const rt_ctx *c)
{
    return c->params.smooth ? (c->grid.ncell * sizeof(int32_t) + 255) & ~(size_t)255 : 0;
}

// accounting partials: 6 doubles per block of either transport kernel
static size_t acct_region(const rt_ctx *c)
{
    const size_t zb = (size_t)transport_z_blocks(c->fp32, c->grid, c->groups.M) * 6 * sizeof(double);
    const size_t cb = acct_bytes(c->grid.ncell);
    return ((zb > cb ? zb : cb) + 255) & ~(size_t)255;
}

static size_t scratch_need(const rt_ctx *c)
{
    return ((reduction_scratch_bytes() + 255) & ~(size_t)255) + queue_bytes(c->qcap_max, c->params.smooth != 0) +
           acct_region(c) + prev_att_bytes(c) + src_map_bytes(c);
}

// accounting partials: after the reduction partials and the queue
static double *acct_part(const rt_ctx *c)
{
    return (double *)((char *)c->st.scratch + ((reduction_scratch_bytes() + 255) & ~(size_t)255) +
                      queue_bytes(c->qcap_max, c->params.smooth != 0));
}

// previous-pass attempt counts: after the accounting partials
static uint8_t *prev_att(const rt_ctx *c) { return (uint8_t *)acct_part(c) + acct_region(c); }

// the source map (smoothed RT): after the attempt counts, null without scratch
static int32_t *src_map(const rt_ctx *c)
{
    if (!c->params.smooth || !c->st.scratch) return nullptr;
    return (int32_t *)(prev_att(c) + prev_att_bytes(c));
}

// write the source map of the current sources (smoothed RT, scratch bound)
static hipError_t rebuild_src_map(rt_ctx *c)
{
    int32_t *map = src_map(c);
    if (!map) return hipSuccess;
    return launch_source_map(map, c->grid.ncell, c->src_cell, c->nsrc, c->stream);
}

// whether the transport runs as the z-marching kernel (else per cell)
static bool use_zmarch(const rt_ctx *c)
{
    return c->path != RT_PATH_CELL && transport_z_fits(c->fp32, c->grid);
}

extern "C" size_t rt_scratch_bytes(const rt_ctx *c)
{
    if (!c) return 0;
    return scratch_need(c);
}

extern "C" rt_status rt_bind(rt_ctx *c, const rt_state *s)
{
    if (!c) return RT_EINVAL;
    if (!s) RT_FAIL(c, RT_EINVAL, "null state");
    if (!s->N[0] || !s->N[1] || !s->F[0] || !s->F[1]) RT_FAIL(c, RT_EINVAL, "radiation buffers must be non-null");
    if (s->N[0] == s->N[1] || s->F[0] == s->F[1]) RT_FAIL(c, RT_EINVAL, "the two radiation sets must differ");
    if (!s->xHII || !s->xHeII || !s->xHeIII || !s->T || !s->nH) RT_FAIL(c, RT_EINVAL, "gas arrays must be non-null");
    if (s->scratch && s->scratch_bytes < scratch_need(c))
        RT_FAIL(c, RT_EINVAL, "scratch must hold rt_scratch_bytes() = %zu bytes", scratch_need(c));
    if (!s->scratch && s->scratch_bytes != 0) RT_FAIL(c, RT_EINVAL, "null scratch with a nonzero size");
    c->st = *s;
    c->bound = true;
    c->cur = 0;
    c->sm_phase = 0;
    // no previous pass yet: every count starts at zero
    if (c->st.scratch) RT_HIP(c, hipMemset(prev_att(c), 0, c->grid.ncell));
    RT_HIP(c, rebuild_src_map(c));
    return RT_OK;
}

extern "C" rt_status rt_set_stream(rt_ctx *c, void *stream)
{
    if (!c) return RT_EINVAL;
    c->stream = (hipStream_t)stream;
    return RT_OK;
}

extern "C" int rt_current(const rt_ctx *c) { return c ? c->cur : -1; }

extern "C" rt_status rt_set_current(rt_ctx *c, int set)
{
    if (!c) return RT_EINVAL;
    if (set != 0 && set != 1) RT_FAIL(c, RT_EINVAL, "set must be 0 or 1");
    c->cur = set;
    c->sm_phase = 0;
    return RT_OK;
}

extern "C" rt_status rt_set_sources(rt_ctx *c, int n, const int32_t *ijk, const double *ndot)
{
    if (!c) return RT_EINVAL;
    if (n < 0) RT_FAIL(c, RT_EINVAL, "n < 0");
    if (n > 0 && (!ijk || !ndot)) RT_FAIL(c, RT_EINVAL, "null source arrays");
    const int M = c->groups.M;
    // merge sources per cell, in input order
    std::vector<int32_t> cells;
    std::vector<double> rates;
    for (int s = 0; s < n; ++s) {
        const int ix = ijk[3 * s], iy = ijk[3 * s + 1], iz = ijk[3 * s + 2];
        if (ix < 0 || ix >= c->grid.nx || iy < 0 || iy >= c->grid.ny || iz < 0 || iz >= c->grid.nz)
            RT_FAIL(c, RT_EINVAL, "source %d outside the grid", s);
        for (int g = 0; g < M; ++g)
            if (!(ndot[(size_t)s * M + g] >= 0) || !std::isfinite(ndot[(size_t)s * M + g]))
                RT_FAIL(c, RT_EINVAL, "source %d: rates must be finite and >= 0", s);
        const int32_t cell = (int32_t)((size_t)ix + (size_t)c->grid.nx * ((size_t)iy + (size_t)c->grid.ny * iz));
        size_t pos = cells.size();
        for (size_t q = 0; q < cells.size(); ++q)
            if (cells[q] == cell) { pos = q; break; }
        if (pos == cells.size()) {
            cells.push_back(cell);
            for (int g = 0; g < M; ++g) rates.push_back(ndot[(size_t)s * M + g]);
        } else {
            for (int g = 0; g < M; ++g) rates[pos * M + g] += ndot[(size_t)s * M + g];
        }
    }
    // work in flight may still read the old tables
    RT_HIP(c, hipStreamSynchronize(c->stream));
    if (c->src_cell) { (void)hipFree(c->src_cell); c->src_cell = nullptr; }
    if (c->src_rate) { (void)hipFree(c->src_rate); c->src_rate = nullptr; }
    if (c->src_in_cell) { (void)hipFree(c->src_in_cell); c->src_in_cell = nullptr; }
    if (c->src_in_rate) { (void)hipFree(c->src_in_rate); c->src_in_rate = nullptr; }
    if (c->src_prev) { (void)hipFree(c->src_prev); c->src_prev = nullptr; }
    c->nsrc = 0;
    c->nsrc_in = 0;
    c->src_rate_host.clear();
    c->sm_phase = 0;
    if (cells.empty()) {
        RT_HIP(c, rebuild_src_map(c));
        return RT_OK;
    }
    {
        std::vector<int32_t> in_cell(n);
        std::vector<double> in_rate(n);
        for (int s = 0; s < n; ++s) {
            in_cell[s] = (int32_t)((size_t)ijk[3 * s] +
                                   (size_t)c->grid.nx * ((size_t)ijk[3 * s + 1] + (size_t)c->grid.ny * ijk[3 * s + 2]));
            in_rate[s] = ndot[(size_t)s * M];
        }
        RT_HIP(c, hipMalloc((void **)&c->src_in_cell, n * sizeof(int32_t)));
        RT_HIP(c, hipMalloc((void **)&c->src_in_rate, n * sizeof(double)));
        RT_HIP(c, hipMemcpy(c->src_in_cell, in_cell.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        RT_HIP(c, hipMemcpy(c->src_in_rate, in_rate.data(), n * sizeof(double), hipMemcpyHostToDevice));
        c->nsrc_in = n;
    }
    RT_HIP(c, hipMalloc((void **)&c->src_cell, cells.size() * sizeof(int32_t)));
    RT_HIP(c, hipMalloc((void **)&c->src_rate, rates.size() * sizeof(double)));
    RT_HIP(c, hipMemcpy(c->src_cell, cells.data(), cells.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(c->src_rate, rates.data(), rates.size() * sizeof(double), hipMemcpyHostToDevice));
    c->nsrc = (int)cells.size();
    c->src_rate_host = rates;
    if (c->params.smooth) RT_HIP(c, hipMalloc((void **)&c->src_prev, rates.size() * sizeof(double)));
    RT_HIP(c, rebuild_src_map(c));
    return RT_OK;
}

extern "C" rt_status rt_set_inflow(rt_ctx *c, int face, const double *flux)
{
    if (!c) return RT_EINVAL;
    if (face < 0 || face > 5) RT_FAIL(c, RT_EINVAL, "face must be 0..5");
    if (c->grid.bc[face] != RT_BC_INFLOW) RT_FAIL(c, RT_EINVAL, "face %d is not an RT_BC_INFLOW face", face);
    if (!flux) RT_FAIL(c, RT_EINVAL, "null flux");
    for (int g = 0; g < c->groups.M; ++g)
        if (!(flux[g] >= 0) || !std::isfinite(flux[g])) RT_FAIL(c, RT_EINVAL, "flux must be finite and >= 0");
    for (int g = 0; g < 3; ++g) c->grid.inflow[face][g] = g < c->groups.M ? flux[g] : 0.0;
    return RT_OK;
}

extern "C" rt_status rt_set_tuning(rt_ctx *c, int head_attempts, long long queue_cap)
{
    if (!c) return RT_EINVAL;
    if (head_attempts == 0 || head_attempts > 1000000) RT_FAIL(c, RT_EINVAL, "head_attempts must be 1..1000000");
    if (queue_cap > (long long)c->qcap_max)
        RT_FAIL(c, RT_EINVAL, "queue_cap %lld exceeds the scratch capacity %u", queue_cap, c->qcap_max);
    if (head_attempts > 0) c->head_attempts = head_attempts;
    if (queue_cap >= 0) c->qcap = (unsigned)queue_cap;
    return RT_OK;
}

extern "C" rt_status rt_courant_dt(const rt_ctx *c, double courant, double *dt)
{
    if (!c || !dt || !(courant > 0)) return RT_EINVAL;
    *dt = courant * c->a_cosmo * c->grid.dx / (3.0 * c->groups.c_r);
    return RT_OK;
}

// largest step the transport allows: the physical cell a dx over 3 c_r
static double dt_limit(const rt_ctx *c) { return c->a_cosmo * c->grid.dx / (3.0 * c->groups.c_r); }

extern "C" rt_status rt_set_expansion(rt_ctx *c, double a)
{
    if (!c) return RT_EINVAL;
    if (!(a > 0) || !std::isfinite(a)) RT_FAIL(c, RT_EINVAL, "a must be positive and finite");
    RT_HIP(c, hipStreamSynchronize(c->stream));
    c->a_cosmo = a;
    c->kchem.a_exp = a;
    RT_HIP(c, hipMemcpy(c->dkchem, &c->kchem, sizeof(KChem), hipMemcpyHostToDevice));
    return RT_OK;
}

static rt_status check_ready(rt_ctx *c, double dt)
{
    if (!c->bound) RT_FAIL(c, RT_ESTATE, "no state bound");
    if (!(dt > 0) || !std::isfinite(dt)) RT_FAIL(c, RT_EINVAL, "dt must be positive and finite");
    return RT_OK;
}

// the chemistry passes, the accounting and the diagnostics work in scratch
static rt_status need_scratch(rt_ctx *c)
{
    if (!c->st.scratch) RT_FAIL(c, RT_ESTATE, "no scratch bound (bind rt_scratch_bytes() of scratch, or use rt_step_noalloc)");
    return RT_OK;
}

static rt_status do_inject(rt_ctx *c, double dt)
{
    const double V = c->grid.dx * c->grid.dx * c->grid.dx;
    if (c->params.smooth) {
        if (c->sm_phase != 0) RT_FAIL(c, RT_ESTATE, "smoothed RT: one injection per step, before the transport");
        if (c->nsrc == 0) return RT_OK;
        c->sm_phase = 1;
    }
    if (c->nsrc == 0) return RT_OK;
    if (c->acct)
        for (int q = 0; q < c->nsrc; ++q)
            for (int g = 0; g < c->groups.M; ++g) c->injected[g] += c->src_rate_host[(size_t)q * c->groups.M + g] * dt;
    return timed(c, TM_INJECT, [&]() -> rt_status {
        RT_HIP(c, launch_inject(c->fp32, c->st.N[c->cur], c->grid.ncell, c->groups.M, c->nsrc, c->src_cell,
                                c->src_rate, dt / V, c->params.smooth ? c->src_prev : nullptr, c->stream));
        return RT_OK;
    });
}

static rt_status do_transport(rt_ctx *c, double dt)
{
    const double dtmax = dt_limit(c);
    if (dt > dtmax * (1.0 + 1e-12)) RT_FAIL(c, RT_EINVAL, "dt = %g exceeds the Courant limit a dx/(3 c_r) = %g", dt, dtmax);
    if (c->params.smooth && c->sm_phase == 2)
        RT_FAIL(c, RT_ESTATE, "smoothed RT: the step's transport has run; its thermochemistry comes next");
    const int s = c->cur, d = 1 - c->cur;
    const bool zm = use_zmarch(c);
    rt_status r = timed(c, TM_TRANSPORT, [&]() -> rt_status {
        // super-comoving variables: light speed a c_r over dt / a^2 (Sec. 5.4)
        const double a = c->a_cosmo;
        if (zm)
            RT_HIP(c, launch_transport_z(c->fp32, c->params.flux, c->grid, c->groups.M, a * c->groups.c_r, dt / (a * a),
                                         c->st.N[s], c->st.F[s], c->st.N[d], c->st.F[d], c->hll_dev, c->nf, c->nth,
                                         c->acct ? acct_part(c) : nullptr, c->stream));
        else
            RT_HIP(c, launch_transport(c->fp32, c->params.flux, c->grid, c->groups.M, a * c->groups.c_r, dt / (a * a),
                                       c->st.N[s], c->st.F[s], c->st.N[d], c->st.F[d], c->hll_dev, c->nf, c->nth,
                                       c->acct ? acct_part(c) : nullptr, c->stream));
        return RT_OK;
    });
    c->acct_nblk = zm ? transport_z_blocks(c->fp32, c->grid, c->groups.M) : acct_blocks(c->grid.ncell);
    if (r != RT_OK) return r;
    c->cur = d;
    c->acct_pending = c->acct;
    if (c->params.smooth) {
        c->sm_injected = c->sm_phase == 1;
        c->sm_phase = 2;
    }
    return RT_OK;
}

// photon totals of the current radiation set: per-block partials in the
// scratch's reduction area (the ledger sums them)
static rt_status acct_reduce(rt_ctx *c)
{
    return timed(c, TM_ACCT, [&]() -> rt_status {
        RT_HIP(c, launch_sum_n(c->fp32, c->grid.ncell, c->groups.M, c->st.N[c->cur], (double *)c->st.scratch,
                               c->stream));
        return RT_OK;
    });
}

// close the step's ledger after the chemistry
static rt_status acct_close(rt_ctx *c, double dt)
{
    const double V = c->grid.dx * c->grid.dx * c->grid.dx;
    rt_status r = acct_reduce(c);
    if (r != RT_OK) return r;
    r = timed(c, TM_ACCT, [&]() -> rt_status {
        RT_HIP(c, launch_ledger(c->acct_pending ? 2 : 1, acct_part(c), c->acct_nblk, (const double *)c->st.scratch,
                                c->groups.M, V, dt / (c->a_cosmo * c->a_cosmo) * c->grid.dx * c->grid.dx, c->dstats,
                                c->stream));
        return RT_OK;
    });
    c->acct_pending = false;
    return r;
}

// smoothed RT: the radiation set before the step and the source table
static SmoothArgs smooth_args(const rt_ctx *c, int pre_set, bool injected)
{
    SmoothArgs a;
    a.N = c->st.N[pre_set];
    a.F = c->st.F[pre_set];
    a.map = injected ? src_map(c) : nullptr;
    a.prev = c->src_prev;
    return a;
}

// One pass or two for the chemistry after a separate transport.  Measured
// on the lognormal workload (mixed precision, n/256 x 200 sources, steps
// 1-40, ms per step, one pass / two passes): 96^3 1.00 / 0.85, 128^3 1.30 /
// 1.19, 160^3 1.76 / 1.90, 192^3 2.16 / 2.51, 224^3 3.17 / 3.97; at 128^3
// with more I-front cells the one pass is ahead (FP64, 50 sources, 200
// steps: 1.18 / 1.24; the shadow test: 0.94 / 1.07).  On small grids the
// lockstep head pass, with many more waves in flight, hides the latency of
// taking cells better than the persistent lanes do; long chains favour the
// one pass, which starts them first.
constexpr size_t CHEM_ONE_PASS_MIN_CELLS = 2000000;

static bool use_one_pass(const rt_ctx *c)
{
    if (c->chem_path == RT_CHEM_ONE_PASS) return true;
    if (c->chem_path == RT_CHEM_TWO_PASS) return false;
    return c->grid.ncell >= CHEM_ONE_PASS_MIN_CELLS;
}

static rt_status do_chem(rt_ctx *c, double dt)
{
    SmoothArgs sa;
    if (c->params.smooth) {
        if (c->sm_phase != 2) RT_FAIL(c, RT_ESTATE, "smoothed RT: the thermochemistry needs the step's transport first");
        sa = smooth_args(c, 1 - c->cur, c->sm_injected);
        c->sm_phase = 0;
    }
    const SmoothArgs *sm = c->params.smooth ? &sa : nullptr;
    const QueueView q = queue_view(c->st.scratch, c->qcap, c->qcap_max);
    if (c->acct && !c->acct_pending) {
        // no transport before this chemistry: its input totals come from a reduction
        rt_status r = acct_reduce(c);
        if (r != RT_OK) return r;
        const double V = c->grid.dx * c->grid.dx * c->grid.dx;
        r = timed(c, TM_ACCT, [&]() -> rt_status {
            RT_HIP(c, launch_ledger(0, nullptr, 0, (const double *)c->st.scratch, c->groups.M, V, 0.0, c->dstats,
                                    c->stream));
            return RT_OK;
        });
        if (r != RT_OK) return r;
    }
    unsigned long long *hist = c->acct ? c->dstats->hist : nullptr;
    if (use_one_pass(c)) {
        rt_status r = timed(c, TM_HEAD, [&]() -> rt_status {
            RT_HIP(c, launch_chem_all(c->fp32, c->grid, c->kchem, c->dkchem, dt, c->st.N[c->cur], c->st.F[c->cur],
                                      c->st.xHII, c->st.xHeII, c->st.xHeIII, c->st.T, c->st.nH, c->st.nacc,
                                      c->st.natt, q, hist, sm, c->a_cosmo, prev_att(c), c->dstats, c->stream));
            return RT_OK;
        });
        if (r != RT_OK) return r;
        return c->acct ? acct_close(c, dt) : RT_OK;
    }
    for (int part = 1; part <= 2; ++part) {
        rt_status r = timed(c, part == 1 ? TM_HEAD : TM_TAIL, [&]() -> rt_status {
            RT_HIP(c, launch_chem(part, c->fp32, c->grid, c->kchem, c->dkchem, dt, c->st.N[c->cur], c->st.F[c->cur], c->st.xHII,
                                  c->st.xHeII, c->st.xHeIII, c->st.T, c->st.nH, c->st.nacc, c->st.natt, q,
                                  c->head_attempts, hist, sm, c->a_cosmo, prev_att(c), c->dstats, c->stream));
            return RT_OK;
        });
        if (r != RT_OK) return r;
    }
    return c->acct ? acct_close(c, dt) : RT_OK;
}

// transport and thermochemistry in one pass over the grid (source set ->
// destination set), then the queued cells
static rt_status do_fused(rt_ctx *c, double dt)
{
    const double dtmax = dt_limit(c);
    if (dt > dtmax * (1.0 + 1e-12)) RT_FAIL(c, RT_EINVAL, "dt = %g exceeds the Courant limit a dx/(3 c_r) = %g", dt, dtmax);
    const int s = c->cur, d = 1 - c->cur;
    SmoothArgs sa;
    if (c->params.smooth) {
        if (c->sm_phase > 1) RT_FAIL(c, RT_ESTATE, "smoothed RT: the step's transport has already run");
        sa = smooth_args(c, s, c->sm_phase == 1);
        c->sm_phase = 0;
    }
    const SmoothArgs *sm = c->params.smooth ? &sa : nullptr;
    const QueueView q = queue_view(c->st.scratch, c->qcap, c->qcap_max);
    for (int part = 1; part <= 2; ++part) {
        rt_status r = timed(c, part == 1 ? TM_HEAD : TM_TAIL, [&]() -> rt_status {
            RT_HIP(c, launch_step_fused(part, c->fp32, c->params.flux, c->grid, c->kchem, c->dkchem, dt, c->st.N[s], c->st.F[s],
                                        c->st.N[d], c->st.F[d], c->st.xHII, c->st.xHeII, c->st.xHeIII, c->st.T,
                                        c->st.nH, c->st.nacc, c->st.natt, c->hll_dev, c->nf, c->nth, q,
                                        c->head_attempts, c->acct ? acct_part(c) : nullptr,
                                        c->acct ? c->dstats->hist : nullptr, sm, c->a_cosmo, prev_att(c), c->dstats,
                                        c->stream));
            return RT_OK;
        });
        if (r != RT_OK) return r;
    }
    c->cur = d;
    if (!c->acct) return RT_OK;
    c->acct_pending = true;
    c->acct_nblk = acct_blocks(c->grid.ncell);
    return acct_close(c, dt);
}

extern "C" rt_status rt_inject(rt_ctx *c, double dt)
{
    if (!c) return RT_EINVAL;
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    return do_inject(c, dt);
}

extern "C" rt_status rt_transport(rt_ctx *c, double dt)
{
    if (!c) return RT_EINVAL;
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    if (c->acct && (r = need_scratch(c)) != RT_OK) return r;
    return do_transport(c, dt);
}

extern "C" rt_status rt_thermochem(rt_ctx *c, double dt)
{
    if (!c) return RT_EINVAL;
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    if ((r = need_scratch(c)) != RT_OK) return r;
    return do_chem(c, dt);
}

static rt_status step_loop(rt_ctx *c, double dt, int nsteps)
{
    rt_status r = RT_OK;
    const bool zm = use_zmarch(c);
    for (int k = 0; k < nsteps; ++k) {
        if ((r = do_inject(c, dt)) != RT_OK) return r;
        if (zm) {
            // the z-marching transport, then the chemistry passes
            if ((r = do_transport(c, dt)) != RT_OK) return r;
            if ((r = do_chem(c, dt)) != RT_OK) return r;
        } else {
            if ((r = do_fused(c, dt)) != RT_OK) return r;
        }
    }
    return RT_OK;
}

extern "C" rt_status rt_step(rt_ctx *c, double dt, int nsteps)
{
    if (!c) return RT_EINVAL;
    if (nsteps < 0) RT_FAIL(c, RT_EINVAL, "nsteps < 0");
    if (!(dt > 0)) dt = 0.8 * dt_limit(c);
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    if ((r = need_scratch(c)) != RT_OK) return r;
    return step_loop(c, dt, nsteps);
}

// rt_step in the device's static scratch array: the same launches with the
// reduction partials, the chemistry queue (of the capacity that fits; cells
// beyond it finish in the first pass, which leaves results unchanged), the
// accounting partials and the previous-pass attempt counts laid out there.
extern "C" rt_status rt_step_noalloc(rt_ctx *c, double dt, int nsteps)
{
    if (!c) return RT_EINVAL;
    if (nsteps < 0) RT_FAIL(c, RT_EINVAL, "nsteps < 0");
    if (!(dt > 0)) dt = 0.8 * dt_limit(c);
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    if (c->params.smooth) RT_FAIL(c, RT_EUNSUPPORTED, "rt_step_noalloc: smoothed RT is not supported");
    void *ptr = (c->device >= 0 && c->device < NOALLOC_MAX_DEVICES) ? g_noalloc_ptr[c->device] : nullptr;
    if (!ptr) RT_FAIL(c, RT_ESTATE, "rt_step_noalloc: no static scratch on device %d", c->device);
    // the layout with an empty queue, then as many queue cells as fit
    const unsigned save_cap = c->qcap, save_max = c->qcap_max;
    c->qcap = c->qcap_max = 0;
    const size_t fixed = scratch_need(c);
    c->qcap = save_cap;
    c->qcap_max = save_max;
    if (fixed > NOALLOC_SCRATCH_BYTES)
        RT_FAIL(c, RT_EINVAL, "rt_step_noalloc: the grid needs %zu bytes of scratch, more than the %zu-byte static buffer",
                fixed, NOALLOC_SCRATCH_BYTES);
    const size_t spare = NOALLOC_SCRATCH_BYTES - fixed;
    size_t cap = spare > 512 ? (spare - 512) / queue_cell_bytes(false) : 0;
    if (cap > c->grid.ncell) cap = c->grid.ncell;
    // swap the static layout in (no timing: its events would be created)
    void *save_scr = c->st.scratch;
    const size_t save_bytes = c->st.scratch_bytes;
    const bool save_timing = c->timing;
    c->st.scratch = ptr;
    c->st.scratch_bytes = NOALLOC_SCRATCH_BYTES;
    c->qcap = c->qcap_max = (unsigned)cap;
    c->timing = false;
    if (scratch_need(c) > NOALLOC_SCRATCH_BYTES) {
        r = RT_EINVAL;
        c->err = "rt_step_noalloc: layout exceeds the static buffer";
    } else {
        // the array keeps the last call's contents: clear the attempt counts
        // that order the queue (the counters and partials are reset or
        // overwritten by the step's own kernels)
        const hipError_t e = launch_fill_u8(prev_att(c), c->grid.ncell, 0, c->stream);
        if (e != hipSuccess) {
            r = RT_EHIP;
            c->err = std::string("rt_step_noalloc: ") + hipGetErrorString(e);
        } else {
            r = step_loop(c, dt, nsteps);
        }
    }
    c->st.scratch = save_scr;
    c->st.scratch_bytes = save_bytes;
    c->qcap = save_cap;
    c->qcap_max = save_max;
    c->timing = save_timing;
    return r;
}

extern "C" rt_status rt_set_transport_path(rt_ctx *c, int path)
{
    if (!c) return RT_EINVAL;
    if (path < RT_PATH_AUTO || path > RT_PATH_ZMARCH) RT_FAIL(c, RT_EINVAL, "path must be RT_PATH_AUTO, _CELL or _ZMARCH");
    if (path == RT_PATH_ZMARCH && !transport_z_fits(c->fp32, c->grid))
        RT_FAIL(c, RT_EINVAL, "the z-marching transport needs nx <= %d", c->fp32 ? 1024 : 512);
    c->path = path;
    return RT_OK;
}

extern "C" rt_status rt_set_chem_path(rt_ctx *c, int path)
{
    if (!c) return RT_EINVAL;
    if (path < RT_CHEM_AUTO || path > RT_CHEM_ONE_PASS)
        RT_FAIL(c, RT_EINVAL, "path must be RT_CHEM_AUTO, _TWO_PASS or _ONE_PASS");
    c->chem_path = path;
    return RT_OK;
}

extern "C" rt_status rt_get_stats(rt_ctx *c, rt_stats *out)
{
    if (!c || !out) return RT_EINVAL;
    if (!c->bound) RT_FAIL(c, RT_ESTATE, "no state bound");
    if (need_scratch(c) != RT_OK) return RT_ESTATE;
    const double V = c->grid.dx * c->grid.dx * c->grid.dx;
    RT_HIP(c, launch_reduce(c->fp32, c->grid.ncell, c->groups.M, c->groups.c_r, V, c->st.N[c->cur], c->st.F[c->cur],
                            c->st.xHII, c->st.nH, c->st.scratch, c->dred, c->stream));
    RedOut r;
    DevStats d;
    RT_HIP(c, hipMemcpyAsync(&r, c->dred, sizeof r, hipMemcpyDeviceToHost, c->stream));
    RT_HIP(c, hipMemcpyAsync(&d, c->dstats, sizeof d, hipMemcpyDeviceToHost, c->stream));
    RT_HIP(c, hipStreamSynchronize(c->stream));
    for (int g = 0; g < 3; ++g) out->photons[g] = r.photons[g];
    out->ionised_H = r.ionised;
    out->max_f = r.maxf;
    out->min_N = r.minN;
    out->substeps_total = (long long)d.acc_total;
    out->attempts_total = (long long)d.att_total;
    out->attempts_max = (long long)d.att_max;
    out->flags = d.flags;
    for (int g = 0; g < 3; ++g) {
        out->injected[g] = c->injected[g];
        out->absorbed[g] = d.absorbed[g];
        out->outflow[g] = d.outflow[g];
    }
    for (int b = 0; b < 64; ++b) out->substep_hist[b] = (long long)d.hist[b];
    return RT_OK;
}

extern "C" rt_status rt_reset_stats(rt_ctx *c)
{
    if (!c) return RT_EINVAL;
    RT_HIP(c, hipMemsetAsync(c->dstats, 0, sizeof(DevStats), c->stream));
    for (int g = 0; g < 3; ++g) c->injected[g] = 0.0;
    return RT_OK;
}

extern "C" rt_status rt_set_accounting(rt_ctx *c, int enabled)
{
    if (!c) return RT_EINVAL;
    c->acct = enabled != 0;
    c->acct_pending = false;
    return RT_OK;
}

extern "C" rt_status rt_hll_table(const rt_ctx *c, const double **table, int *nf, int *nth)
{
    if (!c || !table || !nf || !nth) return RT_EINVAL;
    *table = c->hll_host.data();
    *nf = c->nf;
    *nth = c->nth;
    return RT_OK;
}

extern "C" rt_status rt_build_hll_table(int nf, int nth, double *out)
{
    if (nf < 2 || nth < 2 || !out) return RT_EINVAL;
    std::vector<double> t;
    build_hll(nf, nth, t);
    memcpy(out, t.data(), t.size() * sizeof(double));
    return RT_OK;
}

extern "C" rt_status rt_set_timing(rt_ctx *c, int enabled)
{
    if (!c) return RT_EINVAL;
    if (!enabled) fold_timing(c);
    c->timing = enabled != 0;
    return RT_OK;
}

extern "C" rt_status rt_get_timing(rt_ctx *c, rt_timing *out)
{
    if (!c || !out) return RT_EINVAL;
    fold_timing(c);
    for (int k = 0; k < RT_TIMING_CLASSES; ++k) {
        out->ms[k] = c->t_ms[k];
        out->launches[k] = c->t_n[k];
        c->t_ms[k] = 0.0;
        c->t_n[k] = 0;
    }
    return RT_OK;
}

// ---------------------------------------------------------------------------
// Differentiation form: record and reverse one step.
// ---------------------------------------------------------------------------
static rt_status adj_supported(rt_ctx *c, double dt)
{
    rt_status r = check_ready(c, dt);
    if (r != RT_OK) return r;
    if (c->groups.M != 1) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs one photon group (M = %d)", c->groups.M);
    if (c->params.Y != 0.0) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs hydrogen-only gas (Y = 0)");
    if (c->params.flux != RT_FLUX_GLF) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs the GLF flux");
    if (c->params.smooth) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs smooth = 0");
    if (!c->params.otsa) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs the on-the-spot approximation (otsa = 1)");
    if (c->a_cosmo != 1.0) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs a static box (expansion factor 1)");
    for (int f = 0; f < 6; ++f)
        if (c->grid.bc[f] != RT_BC_PERIODIC) RT_FAIL(c, RT_EUNSUPPORTED, "the adjoint needs periodic boundaries");
    const double dtmax = dt_limit(c);
    if (dt > dtmax * (1.0 + 1e-12)) RT_FAIL(c, RT_EINVAL, "dt = %g exceeds the Courant limit a dx/(3 c_r) = %g", dt, dtmax);
    return RT_OK;
}

static rt_status tape_ok(rt_ctx *c, const rt_tape *t)
{
    if (!t || !t->Na || !t->Fa || !t->counts || !t->off || !t->trace)
        RT_FAIL(c, RT_EINVAL, "tape arrays must be non-null");
    if (t->cap < (long long)c->grid.ncell) RT_FAIL(c, RT_EINVAL, "tape cap %lld < ncell", t->cap);
    return RT_OK;
}

// the photon accounting covers rt_step, rt_transport and rt_thermochem: it
// is paused while a step is recorded or replayed
struct AcctPause {
    rt_ctx *c;
    bool was;
    explicit AcctPause(rt_ctx *ctx) : c(ctx), was(ctx->acct) { c->acct = false; }
    ~AcctPause() { c->acct = was; }
};

extern "C" size_t rt_tape_offsets_len(const rt_ctx *c)
{
    if (!c) return 0;
    return c->grid.ncell + 1 + adj_scan_parts(c->grid.ncell);
}

extern "C" rt_status rt_step_record(rt_ctx *c, double dt, const rt_tape *t)
{
    if (!c) return RT_EINVAL;
    rt_status r = adj_supported(c, dt);
    if (r != RT_OK) return r;
    if ((r = tape_ok(c, t)) != RT_OK) return r;
    AcctPause pause(c);
    const size_t nc = c->grid.ncell;
    RT_HIP(c, launch_offsets(t->counts, nc, t->off, c->stream));
    if ((r = do_inject(c, dt)) != RT_OK) return r;
    if (c->fp32) {
        RT_HIP(c, launch_widen((const float *)c->st.N[c->cur], t->Na, nc, c->stream));
        RT_HIP(c, launch_widen((const float *)c->st.F[c->cur], t->Fa, 3 * nc, c->stream));
    } else {
        RT_HIP(c, hipMemcpyAsync(t->Na, c->st.N[c->cur], nc * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        RT_HIP(c, hipMemcpyAsync(t->Fa, c->st.F[c->cur], 3 * nc * sizeof(double), hipMemcpyDeviceToDevice,
                                 c->stream));
    }
    if ((r = do_transport(c, dt)) != RT_OK) return r;
    return timed(c, TM_OTHER, [&]() -> rt_status {
        if (c->fp32)
            RT_HIP(c, launch_chem_record(c->dkchem, nc, dt, (float *)c->st.N[c->cur], (float *)c->st.F[c->cur],
                                         c->st.xHII, c->st.T, c->st.nH, t->counts, t->off, t->cap, t->trace,
                                         c->dstats, c->stream));
        else
            RT_HIP(c, launch_chem_record(c->dkchem, nc, dt, (double *)c->st.N[c->cur], (double *)c->st.F[c->cur],
                                         c->st.xHII, c->st.T, c->st.nH, t->counts, t->off, t->cap, t->trace,
                                         c->dstats, c->stream));
        return RT_OK;
    });
}

extern "C" rt_status rt_step_replay(rt_ctx *c, double dt, const rt_tape *t)
{
    if (!c) return RT_EINVAL;
    rt_status r = adj_supported(c, dt);
    if (r != RT_OK) return r;
    if ((r = tape_ok(c, t)) != RT_OK) return r;
    AcctPause pause(c);
    const size_t nc = c->grid.ncell;
    if ((r = do_inject(c, dt)) != RT_OK) return r;
    if ((r = do_transport(c, dt)) != RT_OK) return r;
    return timed(c, TM_OTHER, [&]() -> rt_status {
        if (c->fp32)
            RT_HIP(c, launch_chem_replay(c->dkchem, nc, (float *)c->st.N[c->cur], (float *)c->st.F[c->cur],
                                         c->st.xHII, c->st.T, c->st.nH, t->counts, t->off, t->cap, t->trace,
                                         c->stream));
        else
            RT_HIP(c, launch_chem_replay(c->dkchem, nc, (double *)c->st.N[c->cur], (double *)c->st.F[c->cur],
                                         c->st.xHII, c->st.T, c->st.nH, t->counts, t->off, t->cap, t->trace,
                                         c->stream));
        return RT_OK;
    });
}

extern "C" rt_status rt_step_adjoint(rt_ctx *c, double dt, const rt_tape *t, const rt_adj *lam, double *g_lnNdot,
                                     double *g_lnnH)
{
    if (!c) return RT_EINVAL;
    rt_status r = adj_supported(c, dt);
    if (r != RT_OK) return r;
    if ((r = tape_ok(c, t)) != RT_OK) return r;
    if (!lam || !lam->N || !lam->F || !lam->xHII || !lam->T || !lam->wN || !lam->wF)
        RT_FAIL(c, RT_EINVAL, "adjoint arrays must be non-null");
    if (!g_lnnH) RT_FAIL(c, RT_EINVAL, "g_lnnH must be non-null");
    if (c->nsrc_in > 0 && !g_lnNdot) RT_FAIL(c, RT_EINVAL, "g_lnNdot must be non-null when there are sources");
    const size_t nc = c->grid.ncell;
    const double V = c->grid.dx * c->grid.dx * c->grid.dx;
    return timed(c, TM_OTHER, [&]() -> rt_status {
        RT_HIP(c, launch_chem_adj(c->dkchem, nc, c->st.nH, t->counts, t->off, t->cap, t->trace, lam->N, lam->F,
                                  lam->xHII, lam->T, lam->wN, lam->wF, g_lnnH, c->stream));
        RT_HIP(c, launch_transport_adj(c->grid, c->groups.c_r, dt / c->grid.dx, t->Na, t->Fa, lam->wN, lam->wF, lam->N,
                                       lam->F, c->stream));
        RT_HIP(c, launch_inject_adj(lam->N, c->nsrc_in, c->src_in_cell, c->src_in_rate, dt / V, g_lnNdot,
                                    c->stream));
        return RT_OK;
    });
}

extern "C" const char *rt_last_error(const rt_ctx *c)
{
    if (!c) return g_init_err.c_str();
    return c->err.c_str();
}

extern "C" void rt_free(rt_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->hll_dev) (void)hipFree(c->hll_dev);
    if (c->src_cell) (void)hipFree(c->src_cell);
    if (c->src_rate) (void)hipFree(c->src_rate);
    if (c->src_in_cell) (void)hipFree(c->src_in_cell);
    if (c->src_in_rate) (void)hipFree(c->src_in_rate);
    if (c->src_prev) (void)hipFree(c->src_prev);
    if (c->dstats) (void)hipFree(c->dstats);
    if (c->dred) (void)hipFree(c->dred);
    if (c->dkchem) (void)hipFree(c->dkchem);
    for (auto &p : c->pend) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}
