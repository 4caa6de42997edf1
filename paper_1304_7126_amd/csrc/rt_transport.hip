// rt_transport.hip -- the unsplit transport of one RT step (Sec. 3.2,
// eq. dUdt_sol with the fluxes of eqs. glf/hll, App. D source and
// destination copies) as a z-marching stencil for gfx950.
//
// A workgroup owns whole x-rows: a tile of H rows (nx * H <= NT threads,
// one cell per thread) of one photon group, and marches it through a chunk
// of z-planes.  Each cell's closure (m1_pressure) and HLL wave speeds are
// evaluated once, when its plane is next in line, and reach the faces that
// need them through
//   - registers for the z-faces: the flux through a cell's +z face is kept
//     and becomes the -z face of the cell above;
//   - LDS for the x- and y-faces: every thread publishes its state, the row
//     of the pressure tensor and the speed pair along x and along y; the
//     rows just outside the tile (y halo) are evaluated by the tile's edge
//     threads.  In FP32 with HLL fluxes the wave-speed table is read from
//     an LDS copy.
// Each x- and y-face flux is evaluated once, by the cell on its low side,
// and reaches the cell on its high side through LDS.  The next plane's
// state is loaded one iteration ahead of its use.  Every face flux is
// evaluated with the same functions and operands as the per-cell transport
// (transport_cell), and a cell's six fluxes are summed in the same order,
// so both give the same bits.
#include "rt_cell.h"

namespace rtm1 {

// A cell as seen across a face along axis d: its state, row d of its
// pressure tensor c^2 P and its wave-speed pair along d.
template <typename R>
struct FaceSide {
    U4<R> u;
    R p[6];  // only row d is set (prow(p, d) reads it)
    R lm, lp;
};

template <typename R, int FLUX>
__device__ __forceinline__ void side_of(const R *__restrict__ tab, int nf, int nth, const U4<R> &u, int d, R c,
                                        FaceSide<R> &s)
{
    s.u = u;
    m1_pressure(u.n, u.fx, u.fy, u.fz, c, s.p);
    s.lm = R(0);
    s.lp = R(0);
    if (FLUX == 1) hll_speeds(tab, nf, nth, u.n, u.fx, u.fy, u.fz, d, c, s.lm, s.lp);
}

// A cell's closure and its wave speeds along all three axes.
template <typename R>
struct CellEval {
    U4<R> u;
    R p[6];
    R lm[3], lp[3];
};

template <typename R, int FLUX>
__device__ __forceinline__ void eval_cell(const R *__restrict__ tab, int nf, int nth, const U4<R> &u, R c,
                                          CellEval<R> &e)
{
    e.u = u;
    m1_pressure(u.n, u.fx, u.fy, u.fz, c, e.p);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e.lm[d] = R(0);
        e.lp[d] = R(0);
    }
    if (FLUX == 1) {
        // the table row and the flux direction are shared by the three axes
        const HllPrep<R> hp = hll_prep(nf, u.n, u.fx, u.fy, u.fz, c);
#pragma unroll
        for (int d = 0; d < 3; ++d) hll_axis(tab, nth, hp, d, e.lm[d], e.lp[d]);
    }
}

template <typename R>
__device__ __forceinline__ void side_from_eval(const CellEval<R> &e, int d, FaceSide<R> &s)
{
    s.u = e.u;
#pragma unroll
    for (int k = 0; k < 6; ++k) s.p[k] = e.p[k];
    s.lm = e.lm[d];
    s.lp = e.lp[d];
}

// The ghost state across boundary face f (axis d = f/2) of a cell whose
// state is u: outflow copies it, reflect negates the normal flux, inflow
// holds the entering beam (as in transport_cell).
template <typename R>
__device__ __forceinline__ U4<R> ghost_of(const KGrid &g, const U4<R> &u, int f, int grp, R c)
{
    const int d = f >> 1;
    if (g.bc[f] == 3) return beam<R>(g.inflow[f][grp], d, (f & 1) ? -1.0 : 1.0, c);
    U4<R> o = u;
    if (g.bc[f] == 2) {
        if (d == 0) o.fx = -o.fx;
        else if (d == 1) o.fy = -o.fy;
        else o.fz = -o.fz;
    }
    return o;
}

template <typename R>
__device__ __forceinline__ U4<R> load_plane(const R *__restrict__ N, const R *__restrict__ F, size_t nc, size_t i)
{
    U4<R> u;
    u.n = N[i];
    u.fx = F[i];
    u.fy = F[nc + i];
    u.fz = F[2 * nc + i];
    return u;
}

// LDS record of a thread: state (4), row x of c^2 P (3) and the speed pair
// along x (2), row y (3) and the speed pair along y (2)
constexpr int XREC = 14;



template <typename R, int NT>
__device__ __forceinline__ void publish(R (*sh)[NT], int t, const CellEval<R> &e)
{
    sh[0][t] = e.u.n;
    sh[1][t] = e.u.fx;
    sh[2][t] = e.u.fy;
    sh[3][t] = e.u.fz;
    R px, py, pz;
    prow(e.p, 0, px, py, pz);
    sh[4][t] = px;
    sh[5][t] = py;
    sh[6][t] = pz;
    sh[7][t] = e.lm[0];
    sh[8][t] = e.lp[0];
    prow(e.p, 1, px, py, pz);
    sh[9][t] = px;
    sh[10][t] = py;
    sh[11][t] = pz;
    sh[12][t] = e.lm[1];
    sh[13][t] = e.lp[1];
}

// the record of slot t as the side of a face along d (0: x, 1: y)
template <typename R, int NT>
__device__ __forceinline__ void fetch(R (*sh)[NT], int t, int d, FaceSide<R> &s)
{
    s.u.n = sh[0][t];
    s.u.fx = sh[1][t];
    s.u.fy = sh[2][t];
    s.u.fz = sh[3][t];
    const int o = d == 0 ? 4 : 9;
    const R px = sh[o][t], py = sh[o + 1][t], pz = sh[o + 2][t];
    // place the row where prow(p, d) reads it
#pragma unroll
    for (int k = 0; k < 6; ++k) s.p[k] = R(0);
    if (d == 0) {
        s.p[0] = px;
        s.p[3] = py;
        s.p[4] = pz;
    } else {
        s.p[3] = px;
        s.p[1] = py;
        s.p[5] = pz;
    }
    s.lm = sh[o + 3][t];
    s.lp = sh[o + 4][t];
}

template <typename R, int FLUX>
__device__ __forceinline__ void flux_between(const FaceSide<R> &L, const FaceSide<R> &Rt, int d, R c, R Phi[4])
{
    face_flux<R, FLUX>(L.u, L.p, L.lm, L.lp, Rt.u, Rt.p, Rt.lm, Rt.lp, d, c, Phi);
}

// Block-wide fixed-order sum of two doubles per thread (the block may have
// fewer than NT threads); thread 0 returns it.
template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double &sa, double &sb)
{
    __shared__ double rs[2][NT];
    const int t = threadIdx.x;
    const int n = blockDim.x;
    rs[0][t] = a;
    rs[1][t] = b;
    __syncthreads();
    // halve from the power of two at or above n: slots [o, 2o) are added
    // into [0, o), in the same order on every run
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int o = p2 / 2; o > 0; o >>= 1) {
        if (t < o && t + o < n) {
            rs[0][t] += rs[0][t + o];
            rs[1][t] += rs[1][t + o];
        }
        __syncthreads();
    }
    sa = rs[0][0];
    sb = rs[1][0];
}

// grid: (y tiles, z chunks, groups); block: NT threads, of which nx * H
// own cells.  acct (or null): per block of a group, the sum of the new N
// and of the outward boundary flux of the group, at acct[6 b + grp] and
// acct[6 b + 3 + grp] with b = blockIdx.x + gridDim.x * blockIdx.y.
// Two barriers per plane: records are written before the first and read
// between the two; face fluxes are written between the two and read after
// the second.  A thread writes the next plane's records only after the
// second barrier, when every thread has read this plane's, and its next
// fluxes only after the next first barrier, when every thread has read
// these: one buffer of each suffices.
// AHEAD: the plane above and the halo rows are loaded one plane before
// their use (more registers); otherwise at the start of their plane.
// FP32 HLL: the wave-speed table (101 x 101 nodes of float pairs, 80 KiB)
// is copied into LDS when the block starts, so that the twelve bilinear
// corner reads of a cell (three axes) and those of the halo rows are LDS
// reads instead of L2 gathers; with the single record buffer it fits the
// 160 KiB a workgroup may hold.
constexpr int LTAB_CAP = 101 * 101 * 2;
template <typename R, int FLUX, int NT, bool AHEAD>
__global__ __launch_bounds__(NT) void k_transport_z(KGrid g, int H, int zc, R c, R kdx, const R *__restrict__ Nin,
                                                    const R *__restrict__ Fin, R *__restrict__ Nout,
                                                    R *__restrict__ Fout, const R *__restrict__ gtab, int nf, int nth,
                                                    double *__restrict__ acct)
{
    constexpr bool LT = FLUX == 1 && sizeof(R) == 4;
    __shared__ R sh[XREC][NT];
    __shared__ R shf[8][NT];  // the fluxes through each cell's +x and +y faces
    __shared__ R stab[LT ? LTAB_CAP : 1];
    const R *__restrict__ tab = gtab;
    if constexpr (LT) {
        for (int k = threadIdx.x; k < nf * nth * 2; k += blockDim.x) stab[k] = gtab[k];
        __syncthreads();
        tab = stab;
    }
    const int grp = blockIdx.z;
    const int t = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int r = t / nx, x = t - r * nx;
    const int y = (int)blockIdx.x * H + r;
    const bool act = r < H && y < ny;
    const int z0 = (int)blockIdx.y * zc;
    const int z1 = min(z0 + zc, nz);
    const size_t nc = g.ncell;
    const size_t nxy = (size_t)nx * ny;
    const R *__restrict__ N = Nin + (size_t)grp * nc;
    const R *__restrict__ F = Fin + (size_t)3 * grp * nc;
    R *__restrict__ No = Nout + (size_t)grp * nc;
    R *__restrict__ Fo = Fout + (size_t)3 * grp * nc;
    const bool perx = g.bc[0] == 0, pery = g.bc[2] == 0, perz = g.bc[4] == 0;

    // where the neighbours come from: an LDS slot, or -1 a ghost, -2 the
    // halo row (y only, loaded and evaluated by this thread)
    const int tl = x > 0 ? t - 1 : (perx ? t + nx - 1 : -1);
    const int tr = x < nx - 1 ? t + 1 : (perx ? t - (nx - 1) : -1);
    const int tdn = y > 0 ? (r > 0 ? t - nx : -2) : (pery ? -2 : -1);
    const int tup = y < ny - 1 ? (r < H - 1 ? t + nx : -2) : (pery ? -2 : -1);
    const size_t row_dn = (size_t)x + (size_t)nx * (size_t)(y > 0 ? y - 1 : ny - 1);
    const size_t row_up = (size_t)x + (size_t)nx * (size_t)(y < ny - 1 ? y + 1 : 0);
    const size_t row = (size_t)x + (size_t)nx * (size_t)(act ? y : 0);

    CellEval<R> cur;
    R Phzm[4];
    U4<R> nxt_u, hdn_u, hup_u;
    double sumN = 0.0, sumB = 0.0;
    if (act) {
        eval_cell<R, FLUX>(tab, nf, nth, load_plane(N, F, nc, row + (size_t)z0 * nxy), c, cur);
        // the face below the chunk
        FaceSide<R> below;
        if (z0 > 0 || perz) {
            const int zp = z0 > 0 ? z0 - 1 : nz - 1;
            side_of<R, FLUX>(tab, nf, nth, load_plane(N, F, nc, row + (size_t)zp * nxy), 2, c, below);
        } else {
            side_of<R, FLUX>(tab, nf, nth, ghost_of(g, cur.u, 4, grp, c), 2, c, below);
        }
        face_flux<R, FLUX>(below.u, below.p, below.lm, below.lp, cur.u, cur.p, cur.lm[2], cur.lp[2], 2, c, Phzm);
        if constexpr (AHEAD) {
            if (z0 + 1 < nz) nxt_u = load_plane(N, F, nc, row + (size_t)(z0 + 1) * nxy);
            else if (perz) nxt_u = load_plane(N, F, nc, row);
            if (tdn == -2) hdn_u = load_plane(N, F, nc, row_dn + (size_t)z0 * nxy);
            if (tup == -2) hup_u = load_plane(N, F, nc, row_up + (size_t)z0 * nxy);
        }
    }

    for (int z = z0; z < z1; ++z) {
        R(*buf)[NT] = sh;
        // loads for the next plane, in flight during this one
        U4<R> pre_u, pre_dn, pre_up;
        const bool more = z + 1 < z1;
        if constexpr (AHEAD) {
            if (act && more) {
                const int zn = z + 2;
                if (zn < nz) pre_u = load_plane(N, F, nc, row + (size_t)zn * nxy);
                else if (perz) pre_u = load_plane(N, F, nc, row + (size_t)(zn - nz) * nxy);
                if (tdn == -2) pre_dn = load_plane(N, F, nc, row_dn + (size_t)(z + 1) * nxy);
                if (tup == -2) pre_up = load_plane(N, F, nc, row_up + (size_t)(z + 1) * nxy);
            }
        } else if (act) {
            if (z + 1 < nz) nxt_u = load_plane(N, F, nc, row + (size_t)(z + 1) * nxy);
            else if (perz) nxt_u = load_plane(N, F, nc, row);
            if (tdn == -2) hdn_u = load_plane(N, F, nc, row_dn + (size_t)z * nxy);
            if (tup == -2) hup_u = load_plane(N, F, nc, row_up + (size_t)z * nxy);
        }
        if (act) publish<R, NT>(buf, t, cur);
        __syncthreads();
        if (act) {
            // the +x and +y faces: evaluated here, published for the cells
            // on their other side, whose -x and -y faces they are
            R Px[4], Py[4];
            {
                FaceSide<R> s;
                if (tr >= 0) fetch<R, NT>(buf, tr, 0, s);
                else side_of<R, FLUX>(tab, nf, nth, ghost_of(g, cur.u, 1, grp, c), 0, c, s);
                face_flux<R, FLUX>(cur.u, cur.p, cur.lm[0], cur.lp[0], s.u, s.p, s.lm, s.lp, 0, c, Px);
            }
            {
                FaceSide<R> s;
                if (tup >= 0) fetch<R, NT>(buf, tup, 1, s);
                else side_of<R, FLUX>(tab, nf, nth, tup == -2 ? hup_u : ghost_of(g, cur.u, 3, grp, c), 1, c, s);
                face_flux<R, FLUX>(cur.u, cur.p, cur.lm[1], cur.lp[1], s.u, s.p, s.lm, s.lp, 1, c, Py);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                shf[m][t] = Px[m];
                shf[4 + m][t] = Py[m];
            }
        }
        __syncthreads();
        if (act) {
            R Pm[4], Pp[4];
            R acc[4] = {R(0), R(0), R(0), R(0)};
            double bout = 0.0;
            // x faces
            if (tl >= 0) {
#pragma unroll
                for (int m = 0; m < 4; ++m) Pm[m] = shf[m][tl];
            } else {
                FaceSide<R> s;
                side_of<R, FLUX>(tab, nf, nth, ghost_of(g, cur.u, 0, grp, c), 0, c, s);
                face_flux<R, FLUX>(s.u, s.p, s.lm, s.lp, cur.u, cur.p, cur.lm[0], cur.lp[0], 0, c, Pm);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) Pp[m] = shf[m][t];
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m] += Pm[m] - Pp[m];
            if (x == 0 && !perx) bout -= (double)Pm[0];
            if (x == nx - 1 && !perx) bout += (double)Pp[0];
            // y faces
            if (tdn >= 0) {
#pragma unroll
                for (int m = 0; m < 4; ++m) Pm[m] = shf[4 + m][tdn];
            } else {
                FaceSide<R> s;
                side_of<R, FLUX>(tab, nf, nth, tdn == -2 ? hdn_u : ghost_of(g, cur.u, 2, grp, c), 1, c, s);
                face_flux<R, FLUX>(s.u, s.p, s.lm, s.lp, cur.u, cur.p, cur.lm[1], cur.lp[1], 1, c, Pm);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) Pp[m] = shf[4 + m][t];
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m] += Pm[m] - Pp[m];
            if (y == 0 && !pery) bout -= (double)Pm[0];
            if (y == ny - 1 && !pery) bout += (double)Pp[0];
            // z faces: the one below was kept from the previous plane; the
            // cell above is next in line and keeps its evaluation
            CellEval<R> nxt;
            if (z + 1 < nz || perz) {
                eval_cell<R, FLUX>(tab, nf, nth, nxt_u, c, nxt);
                face_flux<R, FLUX>(cur.u, cur.p, cur.lm[2], cur.lp[2], nxt.u, nxt.p, nxt.lm[2], nxt.lp[2], 2, c, Pp);
            } else {
                FaceSide<R> s;
                side_of<R, FLUX>(tab, nf, nth, ghost_of(g, cur.u, 5, grp, c), 2, c, s);
                face_flux<R, FLUX>(cur.u, cur.p, cur.lm[2], cur.lp[2], s.u, s.p, s.lm, s.lp, 2, c, Pp);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m] += Phzm[m] - Pp[m];
            if (z == 0 && !perz) bout -= (double)Phzm[0];
            if (z == nz - 1 && !perz) bout += (double)Pp[0];
            U4<R> o;
            o.n = cur.u.n + kdx * acc[0];
            o.fx = cur.u.fx + kdx * acc[1];
            o.fy = cur.u.fy + kdx * acc[2];
            o.fz = cur.u.fz + kdx * acc[3];
            if (FLUX == 1) limit_flux(o.n, o.fx, o.fy, o.fz, c);
            const size_t i = row + (size_t)z * nxy;
            No[i] = o.n;
            Fo[i] = o.fx;
            Fo[nc + i] = o.fy;
            Fo[2 * nc + i] = o.fz;
            sumN += (double)o.n;
            sumB += bout;
            // shift the window
#pragma unroll
            for (int m = 0; m < 4; ++m) Phzm[m] = Pp[m];
            if (more) {
                cur = nxt;
                if constexpr (AHEAD) {
                    nxt_u = pre_u;
                    hdn_u = pre_dn;
                    hup_u = pre_up;
                }
            }
        }
    }
    if (acct) {
        double a, b;
        block_sum2<NT>(sumN, sumB, a, b);
        if (t == 0) {
            const size_t blk = (size_t)blockIdx.x + (size_t)gridDim.x * blockIdx.y;
            acct[6 * blk + grp] = a;
            acct[6 * blk + 3 + grp] = b;
        }
    }
}

// threads per workgroup and load schedule
#ifndef RT_TZ_NT32
#define RT_TZ_NT32 768
#endif
#ifndef RT_TZ_NT64
#define RT_TZ_NT64 512
#endif
#ifndef RT_TZ_AHEAD32
#define RT_TZ_AHEAD32 1
#endif
#ifndef RT_TZ_AHEAD64
#define RT_TZ_AHEAD64 0
#endif
template <typename R>
constexpr int transport_nt() { return sizeof(R) == 4 ? RT_TZ_NT32 : RT_TZ_NT64; }
template <typename R>
constexpr bool transport_ahead() { return sizeof(R) == 4 ? RT_TZ_AHEAD32 : RT_TZ_AHEAD64; }

bool transport_z_fits(bool fp32, const KGrid &g) { return g.nx <= (fp32 ? transport_nt<float>() : transport_nt<double>()); }

// tile height, z chunk and grid of the z-marching transport
static void transport_z_shape(int NT, const KGrid &g, int M, int &H, int &zc, dim3 &grid)
{
    H = NT / g.nx;
    if (H > g.ny) H = g.ny;
    if (H < 1) H = 1;
    const int nyt = (g.ny + H - 1) / H;
    // about 1,536 workgroups (six per CU), but at least 8 planes per chunk
    long long want = (long long)g.nz * nyt * M / 1536;
    zc = (int)(want < 8 ? 8 : want);
    if (zc > g.nz) zc = g.nz;
    const int nzc = (g.nz + zc - 1) / zc;
    grid = dim3((unsigned)nyt, (unsigned)nzc, (unsigned)M);
}

unsigned transport_z_blocks(bool fp32, const KGrid &g, int M)
{
    int H, zc;
    dim3 gr;
    transport_z_shape(fp32 ? transport_nt<float>() : transport_nt<double>(), g, M, H, zc, gr);
    return gr.x * gr.y;
}

template <typename R>
static hipError_t launch_z(int flux, const KGrid &g, int M, double c, double kdx, const void *Nin, const void *Fin,
                           void *Nout, void *Fout, const void *hll, int nf, int nth, double *acct, hipStream_t s)
{
    constexpr int NT = transport_nt<R>();
    constexpr bool AH = transport_ahead<R>();
    int H, zc;
    dim3 gr;
    transport_z_shape(NT, g, M, H, zc, gr);
    int threads = g.nx * H;
    threads = (threads + 63) / 64 * 64;
    if (threads > NT) threads = NT;
    if (flux)
        hipLaunchKernelGGL((k_transport_z<R, 1, NT, AH>), gr, dim3(threads), 0, s, g, H, zc, (R)c, (R)kdx, (const R *)Nin,
                           (const R *)Fin, (R *)Nout, (R *)Fout, (const R *)hll, nf, nth, acct);
    else
        hipLaunchKernelGGL((k_transport_z<R, 0, NT, AH>), gr, dim3(threads), 0, s, g, H, zc, (R)c, (R)kdx, (const R *)Nin,
                           (const R *)Fin, (R *)Nout, (R *)Fout, (const R *)hll, nf, nth, acct);
    return hipGetLastError();
}

hipError_t launch_transport_z(bool fp32, int flux, const KGrid &g, int M, double c, double dt, const void *Nin,
                              const void *Fin, void *Nout, void *Fout, const void *hll, int nf, int nth, double *acct,
                              hipStream_t s)
{
    // the FP32 HLL kernel holds the table in LDS (rt_init builds 101 x 101)
    if (!transport_z_fits(fp32, g) || (fp32 && flux && nf * nth * 2 > LTAB_CAP)) return hipErrorInvalidValue;
    const double kdx = dt / g.dx;
    return fp32 ? launch_z<float>(flux, g, M, c, kdx, Nin, Fin, Nout, Fout, hll, nf, nth, acct, s)
                : launch_z<double>(flux, g, M, c, kdx, Nin, Fin, Nout, Fout, hll, nf, nth, acct, s);
}

}  // namespace rtm1
