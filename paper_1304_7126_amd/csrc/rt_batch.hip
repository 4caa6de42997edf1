// rt_batch.hip -- the batched form: many independent periodic boxes of
// uneven size (and 1-3 photon groups each) advanced together, one graph
// launch per step.
//
// A step is: k_binject (all boxes' sources), k_bhead (persistent: waves pop
// 64-cell chunks of any box from one queue ordered largest box first, then
// transport and the first K chemistry attempts of each chunk; a chunk never
// straddles two boxes, so box constants stay uniform across the wave),
// k_btail (persistent: lanes refill themselves with the cells still
// subcycling, whatever their box).  No wave ever waits on another, so every
// wave exits once the queues are drained.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rt_cell.h"
#include "rtm1.h"

namespace rtm1 {

struct BoxDev {
    KGrid g;
    int M;
    double kdx;  // dt / dx of the step the graphs were built for
    void *N[2], *F[2];
    double *xHII, *xHeII, *xHeIII, *T;
    const double *nH;
    int32_t *nacc, *natt;
    const KChem *kchem;
};

struct Chunk {
    uint32_t box;
    uint32_t start;
};

struct BSrc {
    uint32_t box, cell;
    double rate[3];
};

// scratch: [3 counters + pad: 256 B][cell, box, acc, att: 4 x cap int32][QV x cap doubles]
struct BQueue {
    unsigned *ctr;  // [0] chunks taken, [1] cells queued, [2] queued cells taken
    int32_t *cell, *box, *acc, *att;
    double *v;
    unsigned cap;
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t bqueue_bytes(unsigned cap) { return 256 + al256((size_t)cap * 4 * 4) + (size_t)QV * cap * 8; }

static BQueue bqueue_view(void *scratch, unsigned cap, unsigned layout_cap)
{
    char *b = (char *)scratch;
    BQueue q;
    q.ctr = (unsigned *)b;
    b += 256;
    q.cell = (int32_t *)b;
    q.box = q.cell + layout_cap;
    q.acc = q.box + layout_cap;
    q.att = q.acc + layout_cap;
    b += al256((size_t)layout_cap * 16);
    q.v = (double *)b;
    q.cap = cap;
    return q;
}

__device__ __forceinline__ void bq_store(const BQueue &q, unsigned stride, uint32_t p, uint32_t box, uint32_t cell,
                                         const CS &s)
{
    q.cell[p] = (int32_t)cell;
    q.box[p] = (int32_t)box;
    q.acc[p] = s.acc;
    q.att[p] = s.att;
    double *v = q.v + p;
    const size_t c = stride;
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
}

__device__ __forceinline__ void bq_load(const BQueue &q, unsigned stride, uint32_t p, uint32_t &box, uint32_t &cell,
                                        CS &s)
{
    cell = (uint32_t)q.cell[p];
    box = (uint32_t)q.box[p];
    s.acc = q.acc[p];
    s.att = q.att[p];
    const double *v = q.v + p;
    const size_t c = stride;
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
}

// write the finished state of a cell of a box with M groups (runtime M);
// fp holds the transported flux (in hand, so that no load sits between the
// stores), written rescaled by fs
template <typename R>
__device__ __forceinline__ void bstore(const BoxDev &b, int dst, uint32_t i, const CS &s, double T, const R *fp)
{
    const size_t nc = b.g.ncell;
    R *N = (R *)b.N[dst];
    R *F = (R *)b.F[dst];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        if (g >= b.M) break;
        N[(size_t)g * nc + i] = (R)s.N[g];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[(size_t)(3 * g + d) * nc + i] = (R)((double)fp[3 * g + d] * s.fs[g]);
    }
    b.xHII[i] = s.x;
    b.xHeII[i] = s.y2;
    b.xHeIII[i] = s.y3;
    b.T[i] = T;
    if (b.nacc) b.nacc[i] = s.acc;
    if (b.natt) b.natt[i] = s.att;
}

// injection with the radiation type known
template <typename R>
__global__ void k_binject_t(const BoxDev *__restrict__ boxes, const BSrc *__restrict__ src, int nsrc, int set,
                            double dt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    const BSrc e = src[s];
    const BoxDev &b = boxes[e.box];
    const double dtV = dt / (b.g.dx * b.g.dx * b.g.dx);
    R *N = (R *)b.N[set];
    for (int g = 0; g < b.M; ++g) {
        R *p = N + (size_t)g * b.g.ncell + e.cell;
        *p = R((double)*p + e.rate[g] * dtV);
    }
}

__global__ void k_bzero(unsigned *p) { if (threadIdx.x < 3) p[threadIdx.x] = 0u; }

// one 64-cell chunk of box b: transport of the M groups from the source
// set, then up to K chemistry attempts; the unfinished cells are queued
template <typename R, int M, int FLUX>
__device__ __forceinline__ void head_chunk(const BoxDev &b, uint32_t box, uint32_t start, int src, double dt, R c,
                                           const R *__restrict__ tab, int nf, int nth, const BQueue &q,
                                           unsigned stride, int K, unsigned long long &a_acc,
                                           unsigned long long &a_att, unsigned long long &a_max, unsigned &fl)
{
    const KChem &k = *b.kchem;
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t i = start + (uint32_t)lane;
    const bool valid = i < (uint32_t)b.g.ncell;
    const size_t nc = b.g.ncell;
    CS s;
    CC cc{1.0, 0.0, 0.0, 0.0};
    bool done = true;
    // the transported flux stays in registers: a queued cell's goes to the
    // destination for the tail, a finished cell's is written once, rescaled
    R fo[3 * M];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        s.N[g] = 0.0;
        s.fs[g] = 1.0;
    }
    if (valid) {
        int ix, iy, iz;
        cell_coords(b.g, i, ix, iy, iz);
        const Nbr nb = neighbours(b.g, i, ix, iy, iz);
        const R *Nin = (const R *)b.N[src];
        const R *Fin = (const R *)b.F[src];
        bool fin = true;
#pragma unroll
        for (int grp = 0; grp < M; ++grp) {
            double bout = 0.0;  // boundary outflow (not accounted in batches)
            const U4<R> o = transport_cell<R, FLUX>(nb, i, nc, Nin + (size_t)grp * nc, Fin + (size_t)3 * grp * nc, c,
                                                    (R)b.kdx, tab, nf, nth, bout, b.g, grp);
            s.N[grp] = (double)o.n;
            fo[3 * grp] = o.fx;
            fo[3 * grp + 1] = o.fy;
            fo[3 * grp + 2] = o.fz;
            fin = fin && isfinite(o.fx) && isfinite(o.fy) && isfinite(o.fz);
        }
        s.x = b.xHII[i];
        s.y2 = b.xHeII[i];
        s.y3 = b.xHeIII[i];
        cc = make_cc(k, b.nH[i], b.T[i]);
        if (chem_init<CM>(k, dt, cc.Tiso, fin, s)) {
            done = false;
            for (int a = 0; a < K && !done; ++a) done = chem_attempt<CM>(k, cc, s, fl);
        } else {
            fl |= 2u;
        }
    }
    const bool want = !done;
    const unsigned long long m = __ballot(want);
    bool queued = false;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned base = 0;
        if (lane == leader) base = atomicAdd(q.ctr + 1, (unsigned)__popcll(m));
        base = __shfl(base, leader);
        if (want) {
            const unsigned p = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
            if (p < q.cap) {
                bq_store(q, stride, p, box, i, s);
                R *Fout = (R *)b.F[1 - src];
#pragma unroll
                for (int j = 0; j < 3 * M; ++j) Fout[(size_t)j * nc + i] = fo[j];
                queued = true;
            }
        }
    }
    if (want && !queued) {
        while (!done) done = chem_attempt<CM>(k, cc, s, fl);
    }
    if (valid && !queued) {
        const double T = chem_finish<CM>(k, cc, s, fl);
        bstore<R>(b, 1 - src, i, s, T, fo);
        a_acc += (unsigned long long)s.acc;
        a_att += (unsigned long long)s.att;
        a_max = a_max > (unsigned long long)s.att ? a_max : (unsigned long long)s.att;
    }
}

__device__ __forceinline__ void bblock_stats(DevStats *st, unsigned long long acc, unsigned long long att,
                                             unsigned long long mx, unsigned fl)
{
    __shared__ unsigned long long s_acc[256], s_att[256], s_max[256];
    __shared__ unsigned s_fl[256];
    const int t = threadIdx.x;
    s_acc[t] = acc;
    s_att[t] = att;
    s_max[t] = mx;
    s_fl[t] = fl;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
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

template <typename R, int FLUX>
__global__ __launch_bounds__(256) void k_bhead(const BoxDev *__restrict__ boxes, const Chunk *__restrict__ chunks,
                                               unsigned nchunks, BQueue q, unsigned stride, int K, int src,
                                               double dt, R c, const R *__restrict__ tab, int nf, int nth,
                                               DevStats *__restrict__ st)
{
    const int lane = (int)(threadIdx.x & 63u);
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    unsigned fl = 0;
    while (true) {
        unsigned ci = 0;
        if (lane == 0) ci = atomicAdd(q.ctr, 1u);
        ci = __shfl(ci, 0);
        if (ci >= nchunks) break;
        const Chunk ch = chunks[ci];
        const BoxDev &b = boxes[ch.box];
        if (b.M == 1)
            head_chunk<R, 1, FLUX>(b, ch.box, ch.start, src, dt, c, tab, nf, nth, q, stride, K, a_acc, a_att, a_max, fl);
        else if (b.M == 2)
            head_chunk<R, 2, FLUX>(b, ch.box, ch.start, src, dt, c, tab, nf, nth, q, stride, K, a_acc, a_att, a_max, fl);
        else
            head_chunk<R, 3, FLUX>(b, ch.box, ch.start, src, dt, c, tab, nf, nth, q, stride, K, a_acc, a_att, a_max, fl);
    }
    bblock_stats(st, a_acc, a_att, a_max, fl);
}

// Tail: lanes hold cells of any box (the attempt runs with three groups, as
// in every chemistry kernel).
template <typename R>
__global__ __launch_bounds__(256) void k_btail(const BoxDev *__restrict__ boxes, BQueue q, unsigned stride, int dst,
                                               double dt, DevStats *__restrict__ st)
{
    const int lane = (int)(threadIdx.x & 63u);
    const unsigned n = min(q.ctr[1], q.cap);
    CS s;
    R fpre[9];  // the cell's transported flux, loaded with the cell (used when it is written)
    uint32_t cell = 0, box = 0;
    CC cc{1.0, 0.0, 0.0, 0.0};
    bool active = false, exhausted = false;
    unsigned rbase = 0, ravail = 0;  // positions this wave has reserved and not yet handed out
    unsigned fl = 0;
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    while (true) {
        if (!exhausted) {
            const bool need = !active;
            const unsigned long long m = __ballot(need);
            if (m) {
                // as in the grid's tail: reservations of a wave's width
                const unsigned nneed = (unsigned)__popcll(m);
                const unsigned r = (unsigned)__popcll(m & ((1ull << lane) - 1ull));
                unsigned p;
                if (ravail >= nneed) {
                    p = rbase + r;
                    rbase += nneed;
                    ravail -= nneed;
                } else {
                    const unsigned more = nneed - ravail;
                    const unsigned take = more > TAIL_CHUNK ? more : TAIL_CHUNK;
                    const int leader = __ffsll((long long)m) - 1;
                    unsigned base = 0;
                    if (lane == leader) base = atomicAdd(q.ctr + 2, take);
                    base = __shfl(base, leader);
                    p = r < ravail ? rbase + r : base + (r - ravail);
                    rbase = base + more;
                    ravail = take - more;
                }
                if (rbase >= n) exhausted = true;
                if (need && p < n) {
                    bq_load(q, stride, p, box, cell, s);
                    const BoxDev &bb = boxes[box];
                    cc = make_cc(*bb.kchem, bb.nH[cell], bb.T[cell]);
                    const R *F = (const R *)bb.F[dst];
#pragma unroll
                    for (int j = 0; j < 9; ++j) fpre[j] = j < 3 * bb.M ? F[(size_t)j * bb.g.ncell + cell] : R(0);
                    active = true;
                }
            }
        }
        if (!__any(active)) break;
        if (active) {
            const KChem &k = *boxes[box].kchem;
            if (chem_attempt<CM>(k, cc, s, fl)) {
                const double T = chem_finish<CM>(k, cc, s, fl);
                bstore<R>(boxes[box], dst, cell, s, T, fpre);
                a_acc += (unsigned long long)s.acc;
                a_att += (unsigned long long)s.att;
                a_max = a_max > (unsigned long long)s.att ? a_max : (unsigned long long)s.att;
                active = false;
            }
        }
    }
    bblock_stats(st, a_acc, a_att, a_max, fl);
}

}  // namespace rtm1

using namespace rtm1;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct rt_batch {
    int nbox = 0;
    bool fp32 = false;
    int flux = 0;
    double c_r = 0;
    std::vector<BoxDev> boxes;      // host copy of the descriptors
    std::vector<KChem> kchem;       // one per box
    std::vector<double> dx;
    BoxDev *dboxes = nullptr;
    KChem *dkchem = nullptr;
    Chunk *dchunks = nullptr;
    unsigned nchunks = 0;
    void *hll = nullptr;
    int nf = 101, nth = 101;
    std::vector<std::vector<BSrc>> src;  // per box, merged per cell
    BSrc *dsrc = nullptr;
    int nsrc = 0;
    bool src_dirty = true;
    DevStats *dstats = nullptr;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    unsigned qcap = 0, qcap_max = 0;
    bool bound = false;
    int cur = 0;
    hipStream_t stream = nullptr;
    // tuning
    int head_blocks_per_cu = 4;
    int head_attempts = HEAD_ATTEMPTS;
    int tail_blocks = TAIL_BLOCKS;
    int use_graph = 1;
    int ncu = 256;
    // graphs of one step starting from set 0 and from set 1
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    double graph_dt = -1.0;
    double kdx_dt = -1.0;
    std::string err;
};

#define BT_FAIL(b, code, ...)                                                     \
    do {                                                                          \
        char _m[512];                                                             \
        snprintf(_m, sizeof(_m), __VA_ARGS__);                                    \
        (b)->err = _m;                                                            \
        return code;                                                              \
    } while (0)

#define BT_HIP(b, call)                                                                             \
    do {                                                                                            \
        hipError_t _e = (call);                                                                     \
        if (_e != hipSuccess) BT_FAIL(b, RT_EHIP, "%s failed: %s", #call, hipGetErrorString(_e));  \
    } while (0)

static thread_local std::string g_batch_err;

static void drop_graphs(rt_batch *b)
{
    for (int k = 0; k < 2; ++k)
        if (b->gexec[k]) {
            (void)hipGraphExecDestroy(b->gexec[k]);
            b->gexec[k] = nullptr;
        }
    b->graph_dt = -1.0;
}

extern "C" rt_status rt_batch_init(int nbox, const rt_grid *grids, const rt_groups *groups, const rt_params *params,
                                   rt_batch **out)
{
    if (!out) return RT_EINVAL;
    *out = nullptr;
    if (nbox < 1 || nbox > 65535 || !grids || !groups || !params) {
        g_batch_err = "need 1..65535 boxes and non-null grids, groups, params";
        return RT_EINVAL;
    }
    // validate each box through a single-grid context description
    for (int i = 0; i < nbox; ++i) {
        if (groups[i].c_r != groups[0].c_r) {
            g_batch_err = "all boxes must share c_r";
            return RT_EINVAL;
        }
        if (grids[i].nx < 1 || grids[i].ny < 1 || grids[i].nz < 1 || !(grids[i].dx > 0)) {
            g_batch_err = "box grid dimensions and dx must be positive";
            return RT_EINVAL;
        }
        for (int d = 0; d < 3; ++d)
            if ((grids[i].bc[2 * d] == RT_BC_PERIODIC) != (grids[i].bc[2 * d + 1] == RT_BC_PERIODIC) ||
                grids[i].bc[2 * d] < 0 || grids[i].bc[2 * d] > 2 || grids[i].bc[2 * d + 1] < 0 ||
                grids[i].bc[2 * d + 1] > 2) {
                g_batch_err = "invalid boundary conditions (periodic must be set on both faces)";
                return RT_EINVAL;
            }
        if (groups[i].M < 1 || groups[i].M > 3 || !(groups[i].c_r > 0)) {
            g_batch_err = "each box needs 1..3 groups and c_r > 0";
            return RT_EINVAL;
        }
    }
    if (params->smooth) {
        g_batch_err = "the batch runs without smoothed RT (smooth = 0)";
        return RT_EUNSUPPORTED;
    }
    if (params->otsa != 1) {
        g_batch_err = "the batch runs with the on-the-spot approximation (otsa = 1)";
        return RT_EUNSUPPORTED;
    }
    if (params->flux != RT_FLUX_GLF && params->flux != RT_FLUX_HLL) { g_batch_err = "flux invalid"; return RT_EINVAL; }
    if (params->prec != RT_PREC_FP64 && params->prec != RT_PREC_FP32_TRANSPORT) { g_batch_err = "prec invalid"; return RT_EINVAL; }
    if (!(params->X > 0) || !(params->Y >= 0) || params->X + params->Y > 1 + 1e-12 || !(params->gamma > 1) ||
        !(params->a_exp > 0) || !(params->x_min > 0) || !(params->x_min < 1) || !(params->N_floor >= 0) ||
        params->max_attempts < 1) {
        g_batch_err = "invalid method parameters";
        return RT_EINVAL;
    }
    double tot = 0;
    for (int i = 0; i < nbox; ++i) tot += (double)grids[i].nx * grids[i].ny * grids[i].nz;
    if (tot > 2.0e9) { g_batch_err = "too many cells in total (> 2e9)"; return RT_EINVAL; }

    rt_batch *b = new rt_batch();
    b->nbox = nbox;
    b->fp32 = params->prec == RT_PREC_FP32_TRANSPORT;
    b->flux = params->flux;
    b->c_r = groups[0].c_r;
    b->boxes.resize(nbox);
    b->kchem.resize(nbox);
    b->dx.resize(nbox);
    b->src.assign(nbox, {});
    size_t ncell_tot = 0;
    for (int i = 0; i < nbox; ++i) {
        BoxDev &bd = b->boxes[i];
        memset(&bd, 0, sizeof bd);
        bd.g.nx = grids[i].nx;
        bd.g.ny = grids[i].ny;
        bd.g.nz = grids[i].nz;
        for (int f = 0; f < 6; ++f) bd.g.bc[f] = grids[i].bc[f];
        bd.g.ncell = (size_t)grids[i].nx * grids[i].ny * grids[i].nz;
        bd.g.dx = grids[i].dx;
        bd.M = groups[i].M;
        b->dx[i] = grids[i].dx;
        ncell_tot += bd.g.ncell;
        KChem &k = b->kchem[i];
        memset(&k, 0, sizeof k);
        k.M = groups[i].M;
        k.isothermal = params->isothermal ? 1 : 0;
        k.cr = groups[i].c_r;
        for (int g = 0; g < groups[i].M; ++g) {
            for (int j = 0; j < 3; ++j) {
                k.sN[g][j] = groups[i].sigN[g][j];
                k.sE[g][j] = groups[i].sigE[g][j];
            }
            k.eb[g] = groups[i].ebar[g];
        }
        k.X = params->X;
        k.Y = params->Y;
        k.Kfac = (params->gamma - 1.0) * params->X / 1.380649e-16;
        k.a_exp = params->a_exp;
        k.x_min = params->x_min;
        k.N_floor = params->N_floor;
        k.max_att = params->max_attempts;
        kchem_derive(k);
    }
    // chunk order: largest boxes (cells x groups) first, cells in order
    std::vector<int> order(nbox);
    for (int i = 0; i < nbox; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return b->boxes[a].g.ncell * (size_t)b->boxes[a].M > b->boxes[c].g.ncell * (size_t)b->boxes[c].M;
    });
    std::vector<Chunk> chunks;
    for (int i : order)
        for (size_t s = 0; s < b->boxes[i].g.ncell; s += 64) chunks.push_back({(uint32_t)i, (uint32_t)s});
    b->nchunks = (unsigned)chunks.size();
    // room for every cell, so that no cell has to finish in the head pass
    const size_t cap = ncell_tot;
    b->qcap = b->qcap_max = (unsigned)cap;

    std::vector<double> tab((size_t)b->nf * b->nth * 2);
    rt_build_hll_table(b->nf, b->nth, tab.data());
    hipError_t e = hipSuccess;
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc((void **)&b->dboxes, nbox * sizeof(BoxDev));
    if (e == hipSuccess) e = hipMalloc((void **)&b->dkchem, nbox * sizeof(KChem));
    if (e == hipSuccess) e = hipMemcpy(b->dkchem, b->kchem.data(), nbox * sizeof(KChem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&b->dchunks, chunks.size() * sizeof(Chunk));
    if (e == hipSuccess) e = hipMemcpy(b->dchunks, chunks.data(), chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&b->dstats, sizeof(DevStats));
    if (e == hipSuccess) e = hipMemset(b->dstats, 0, sizeof(DevStats));
    if (b->fp32) {
        std::vector<float> tf(tab.size());
        for (size_t i = 0; i < tab.size(); ++i) tf[i] = (float)tab[i];
        if (e == hipSuccess) e = hipMalloc(&b->hll, tf.size() * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(b->hll, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice);
    } else {
        if (e == hipSuccess) e = hipMalloc(&b->hll, tab.size() * sizeof(double));
        if (e == hipSuccess) e = hipMemcpy(b->hll, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        g_batch_err = std::string("device table allocation failed: ") + hipGetErrorString(e);
        rt_batch_free(b);
        return RT_ENOMEM;
    }
    for (int i = 0; i < nbox; ++i) b->boxes[i].kchem = b->dkchem + i;
    *out = b;
    return RT_OK;
}

extern "C" size_t rt_batch_scratch_bytes(const rt_batch *b) { return b ? bqueue_bytes(b->qcap_max) : 0; }

extern "C" rt_status rt_batch_bind(rt_batch *b, const rt_state *states, void *scratch, size_t scratch_bytes)
{
    if (!b) return RT_EINVAL;
    if (!states) BT_FAIL(b, RT_EINVAL, "null states");
    if (!scratch || scratch_bytes < bqueue_bytes(b->qcap_max))
        BT_FAIL(b, RT_EINVAL, "scratch must hold rt_batch_scratch_bytes() = %zu bytes", bqueue_bytes(b->qcap_max));
    for (int i = 0; i < b->nbox; ++i) {
        const rt_state &s = states[i];
        if (!s.N[0] || !s.N[1] || !s.F[0] || !s.F[1] || s.N[0] == s.N[1] || s.F[0] == s.F[1] || !s.xHII ||
            !s.xHeII || !s.xHeIII || !s.T || !s.nH)
            BT_FAIL(b, RT_EINVAL, "box %d: missing or aliased state arrays", i);
        BoxDev &bd = b->boxes[i];
        for (int k = 0; k < 2; ++k) {
            bd.N[k] = s.N[k];
            bd.F[k] = s.F[k];
        }
        bd.xHII = s.xHII;
        bd.xHeII = s.xHeII;
        bd.xHeIII = s.xHeIII;
        bd.T = s.T;
        bd.nH = s.nH;
        bd.nacc = s.nacc;
        bd.natt = s.natt;
    }
    b->scratch = scratch;
    b->scratch_bytes = scratch_bytes;
    BT_HIP(b, hipMemcpy(b->dboxes, b->boxes.data(), b->nbox * sizeof(BoxDev), hipMemcpyHostToDevice));
    b->bound = true;
    b->cur = 0;
    b->kdx_dt = -1.0;
    drop_graphs(b);
    return RT_OK;
}

extern "C" rt_status rt_batch_set_stream(rt_batch *b, void *stream)
{
    if (!b) return RT_EINVAL;
    if ((hipStream_t)stream != b->stream) drop_graphs(b);
    b->stream = (hipStream_t)stream;
    return RT_OK;
}

extern "C" int rt_batch_current(const rt_batch *b) { return b ? b->cur : -1; }

extern "C" rt_status rt_batch_set_current(rt_batch *b, int set)
{
    if (!b) return RT_EINVAL;
    if (set != 0 && set != 1) BT_FAIL(b, RT_EINVAL, "set must be 0 or 1");
    b->cur = set;
    return RT_OK;
}

extern "C" rt_status rt_batch_set_sources(rt_batch *b, int box, int n, const int32_t *ijk, const double *ndot)
{
    if (!b) return RT_EINVAL;
    if (box < 0 || box >= b->nbox) BT_FAIL(b, RT_EINVAL, "box %d out of range", box);
    if (n < 0 || (n > 0 && (!ijk || !ndot))) BT_FAIL(b, RT_EINVAL, "bad source arrays");
    const BoxDev &bd = b->boxes[box];
    std::vector<BSrc> v;
    for (int s = 0; s < n; ++s) {
        const int ix = ijk[3 * s], iy = ijk[3 * s + 1], iz = ijk[3 * s + 2];
        if (ix < 0 || ix >= bd.g.nx || iy < 0 || iy >= bd.g.ny || iz < 0 || iz >= bd.g.nz)
            BT_FAIL(b, RT_EINVAL, "box %d source %d outside the grid", box, s);
        const uint32_t cell = (uint32_t)((size_t)ix + (size_t)bd.g.nx * ((size_t)iy + (size_t)bd.g.ny * iz));
        size_t pos = v.size();
        for (size_t q = 0; q < v.size(); ++q)
            if (v[q].cell == cell) { pos = q; break; }
        if (pos == v.size()) {
            BSrc e;
            e.box = (uint32_t)box;
            e.cell = cell;
            e.rate[0] = e.rate[1] = e.rate[2] = 0.0;
            v.push_back(e);
        }
        for (int g = 0; g < bd.M; ++g) {
            const double r = ndot[(size_t)s * bd.M + g];
            if (!(r >= 0) || !std::isfinite(r)) BT_FAIL(b, RT_EINVAL, "box %d source %d: bad rate", box, s);
            v[pos].rate[g] += r;
        }
    }
    b->src[box] = v;
    b->src_dirty = true;
    drop_graphs(b);
    return RT_OK;
}

extern "C" rt_status rt_batch_set_tuning(rt_batch *b, int head_blocks_per_cu, int head_attempts, int tail_blocks,
                                         int use_graph)
{
    if (!b) return RT_EINVAL;
    if (head_blocks_per_cu == 0 || head_blocks_per_cu > 64) BT_FAIL(b, RT_EINVAL, "head_blocks_per_cu must be 1..64");
    if (head_attempts == 0 || head_attempts > 1000000) BT_FAIL(b, RT_EINVAL, "head_attempts must be 1..1000000");
    if (tail_blocks == 0 || tail_blocks > 65536) BT_FAIL(b, RT_EINVAL, "tail_blocks must be 1..65536");
    if (head_blocks_per_cu > 0) b->head_blocks_per_cu = head_blocks_per_cu;
    if (head_attempts > 0) b->head_attempts = head_attempts;
    if (tail_blocks > 0) b->tail_blocks = tail_blocks;
    if (use_graph >= 0) b->use_graph = use_graph != 0;
    drop_graphs(b);
    return RT_OK;
}

static rt_status upload_sources(rt_batch *b)
{
    if (!b->src_dirty) return RT_OK;
    std::vector<BSrc> all;
    for (auto &v : b->src) all.insert(all.end(), v.begin(), v.end());
    if (b->dsrc) { (void)hipFree(b->dsrc); b->dsrc = nullptr; }
    b->nsrc = (int)all.size();
    if (!all.empty()) {
        BT_HIP(b, hipMalloc((void **)&b->dsrc, all.size() * sizeof(BSrc)));
        BT_HIP(b, hipMemcpy(b->dsrc, all.data(), all.size() * sizeof(BSrc), hipMemcpyHostToDevice));
    }
    b->src_dirty = false;
    return RT_OK;
}

// enqueue one step from radiation set `src` (no host synchronisation)
static rt_status enqueue_step(rt_batch *b, double dt, int src)
{
    const BQueue q = bqueue_view(b->scratch, b->qcap, b->qcap_max);
    hipStream_t s = b->stream;
    hipLaunchKernelGGL(k_bzero, dim3(1), dim3(64), 0, s, q.ctr);
    if (b->nsrc > 0) {
        if (b->fp32)
            hipLaunchKernelGGL(k_binject_t<float>, dim3((b->nsrc + 63) / 64), dim3(64), 0, s, b->dboxes, b->dsrc, b->nsrc,
                               src, dt);
        else
            hipLaunchKernelGGL(k_binject_t<double>, dim3((b->nsrc + 63) / 64), dim3(64), 0, s, b->dboxes, b->dsrc,
                               b->nsrc, src, dt);
    }
    const unsigned hb = (unsigned)(b->head_blocks_per_cu * b->ncu);
    const unsigned tb = (unsigned)b->tail_blocks;
    if (b->fp32) {
        auto hk = b->flux ? k_bhead<float, 1> : k_bhead<float, 0>;
        hipLaunchKernelGGL(hk, dim3(hb), dim3(256), 0, s, b->dboxes, b->dchunks, b->nchunks, q, b->qcap_max,
                           b->head_attempts, src, dt, (float)b->c_r, (const float *)b->hll, b->nf, b->nth, b->dstats);
        hipLaunchKernelGGL(k_btail<float>, dim3(tb), dim3(256), 0, s, b->dboxes, q, b->qcap_max, 1 - src, dt,
                           b->dstats);
    } else {
        auto hk = b->flux ? k_bhead<double, 1> : k_bhead<double, 0>;
        hipLaunchKernelGGL(hk, dim3(hb), dim3(256), 0, s, b->dboxes, b->dchunks, b->nchunks, q, b->qcap_max,
                           b->head_attempts, src, dt, b->c_r, (const double *)b->hll, b->nf, b->nth, b->dstats);
        hipLaunchKernelGGL(k_btail<double>, dim3(tb), dim3(256), 0, s, b->dboxes, q, b->qcap_max, 1 - src, dt,
                           b->dstats);
    }
    BT_HIP(b, hipGetLastError());
    return RT_OK;
}

// the largest step every box's transport allows: the finest box's dx over 3 c_r
static double batch_dt_limit(const rt_batch *b)
{
    double dxmin = b->dx[0];
    for (double v : b->dx) dxmin = v < dxmin ? v : dxmin;
    return dxmin / (3.0 * b->c_r);
}

extern "C" rt_status rt_batch_courant_dt(const rt_batch *b, double courant, double *dt)
{
    if (!b || !dt || !(courant > 0)) return RT_EINVAL;
    *dt = courant * batch_dt_limit(b);
    return RT_OK;
}

extern "C" rt_status rt_batch_step(rt_batch *b, double dt, int nsteps)
{
    if (!b) return RT_EINVAL;
    if (!b->bound) BT_FAIL(b, RT_ESTATE, "no state bound");
    if (nsteps < 0) BT_FAIL(b, RT_EINVAL, "nsteps < 0");
    const double dxmin = batch_dt_limit(b) * 3.0 * b->c_r;
    if (!(dt > 0)) dt = 0.8 * dxmin / (3.0 * b->c_r);
    if (dt > dxmin / (3.0 * b->c_r) * (1.0 + 1e-12))
        BT_FAIL(b, RT_EINVAL, "dt = %g exceeds the Courant limit of the finest box", dt);
    rt_status r = upload_sources(b);
    if (r != RT_OK) return r;
    if (dt != b->kdx_dt) {
        for (int i = 0; i < b->nbox; ++i) b->boxes[i].kdx = dt / b->dx[i];
        BT_HIP(b, hipMemcpyAsync(b->dboxes, b->boxes.data(), b->nbox * sizeof(BoxDev), hipMemcpyHostToDevice,
                                 b->stream));
        BT_HIP(b, hipStreamSynchronize(b->stream));
        b->kdx_dt = dt;
        drop_graphs(b);
    }
    const bool graphs = b->use_graph && b->stream != nullptr;
    if (graphs && (b->graph_dt != dt || !b->gexec[0] || !b->gexec[1])) {
        drop_graphs(b);
        for (int p = 0; p < 2; ++p) {
            hipGraph_t g = nullptr;
            BT_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            rt_status rr = enqueue_step(b, dt, p);
            hipError_t ee = hipStreamEndCapture(b->stream, &g);
            if (rr != RT_OK) return rr;
            BT_HIP(b, ee);
            ee = hipGraphInstantiate(&b->gexec[p], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            BT_HIP(b, ee);
        }
        b->graph_dt = dt;
    }
    for (int k = 0; k < nsteps; ++k) {
        if (graphs) {
            BT_HIP(b, hipGraphLaunch(b->gexec[b->cur], b->stream));
        } else {
            r = enqueue_step(b, dt, b->cur);
            if (r != RT_OK) return r;
        }
        b->cur = 1 - b->cur;
    }
    return RT_OK;
}

extern "C" rt_status rt_batch_get_stats(rt_batch *b, rt_stats *out)
{
    if (!b || !out) return RT_EINVAL;
    DevStats d;
    BT_HIP(b, hipMemcpyAsync(&d, b->dstats, sizeof d, hipMemcpyDeviceToHost, b->stream));
    BT_HIP(b, hipStreamSynchronize(b->stream));
    memset(out, 0, sizeof *out);
    out->substeps_total = (long long)d.acc_total;
    out->attempts_total = (long long)d.att_total;
    out->attempts_max = (long long)d.att_max;
    out->flags = d.flags;
    return RT_OK;
}

extern "C" rt_status rt_batch_reset_stats(rt_batch *b)
{
    if (!b) return RT_EINVAL;
    BT_HIP(b, hipMemsetAsync(b->dstats, 0, sizeof(DevStats), b->stream));
    return RT_OK;
}

extern "C" const char *rt_batch_last_error(const rt_batch *b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

extern "C" void rt_batch_free(rt_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    drop_graphs(b);
    if (b->dboxes) (void)hipFree(b->dboxes);
    if (b->dkchem) (void)hipFree(b->dkchem);
    if (b->dchunks) (void)hipFree(b->dchunks);
    if (b->dsrc) (void)hipFree(b->dsrc);
    if (b->dstats) (void)hipFree(b->dstats);
    if (b->hll) (void)hipFree(b->hll);
    delete b;
}
