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
#include "rt_cell.h"

namespace rtm1 {

// ------------------------------------------------------------------ inject
// The source cells are distinct (sources sharing a cell are merged on the
// host), so each thread owns its cell.  prev, when given, receives the
// photon density before the injection (smoothed RT).
template <typename R>
__global__ void k_inject(R *__restrict__ N, size_t ncell, int M, int nsrc, const int32_t *__restrict__ cell,
                         const double *__restrict__ rate, double dtV, double *__restrict__ prev)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsrc) return;
    const size_t i = (size_t)cell[s];
    for (int g = 0; g < M; ++g) {
        R *p = N + (size_t)g * ncell + i;
        const double n0 = (double)*p;
        if (prev) prev[(size_t)s * M + g] = n0;
        *p = R(n0 + rate[(size_t)s * M + g] * dtV);
    }
}

hipError_t launch_inject(bool fp32, void *N, size_t ncell, int M, int nsrc, const int32_t *cell,
                         const double *rate, double dt_over_V, double *prev, hipStream_t s)
{
    if (nsrc <= 0) return hipSuccess;
    dim3 b(64), gr((nsrc + 63) / 64);
    if (fp32)
        hipLaunchKernelGGL(k_inject<float>, gr, b, 0, s, (float *)N, ncell, M, nsrc, cell, rate, dt_over_V, prev);
    else
        hipLaunchKernelGGL(k_inject<double>, gr, b, 0, s, (double *)N, ncell, M, nsrc, cell, rate, dt_over_V, prev);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, size_t n, uint8_t v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_source_map(int32_t *map, const int32_t *__restrict__ cell, int nsrc)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsrc) map[cell[s]] = s;
}

hipError_t launch_source_map(int32_t *map, size_t ncell, const int32_t *cell, int nsrc, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, map, ncell, -1);
    if (nsrc > 0) hipLaunchKernelGGL(k_source_map, dim3((nsrc + 63) / 64), dim3(64), 0, s, map, cell, nsrc);
    return hipGetLastError();
}

// ---------------------------------------------------------- accounting
unsigned acct_blocks(size_t ncell) { return (unsigned)((ncell + ACCT_THREADS - 1) / ACCT_THREADS); }
size_t acct_bytes(size_t ncell) { return ((size_t)acct_blocks(ncell) * 6 * sizeof(double) + 255) & ~(size_t)255; }

// Fixed-order block sum of the per-thread values v[0..5] (transported N and
// outward boundary flux per group) into part[6 * blockIdx.x + q].  Called by
// every thread of a 256-thread block.
__device__ __forceinline__ void block_acct(double *part, const double v[6])
{
    __shared__ double sh[6][ACCT_THREADS];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 6; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int o = ACCT_THREADS / 2; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int q = 0; q < 6; ++q) sh[q][t] += sh[q][t + o];
        }
        __syncthreads();
    }
    if (t < 6) part[(size_t)6 * blockIdx.x + t] = sh[t][0];
}

// --------------------------------------------------------------- transport
template <typename R, int FLUX>
__global__ __launch_bounds__(256) void k_transport(KGrid g, int M, R c, R kdx, const R *__restrict__ Nin,
                                                   const R *__restrict__ Fin, R *__restrict__ Nout,
                                                   R *__restrict__ Fout, const R *__restrict__ tab, int nf,
                                                   int nth, double *__restrict__ acct)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nc = g.ncell;
    double av[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < (uint32_t)nc) {
        int ix, iy, iz;
        cell_coords(g, i, ix, iy, iz);
        const Nbr nb = neighbours(g, i, ix, iy, iz);
        for (int grp = 0; grp < M; ++grp) {
            double bout = 0.0;
            const U4<R> o = transport_cell<R, FLUX>(nb, i, nc, Nin + (size_t)grp * nc, Fin + (size_t)3 * grp * nc,
                                                    c, kdx, tab, nf, nth, bout, g, grp);
            Nout[(size_t)grp * nc + i] = o.n;
            R *Fo = Fout + (size_t)3 * grp * nc;
            Fo[i] = o.fx;
            Fo[nc + i] = o.fy;
            Fo[2 * nc + i] = o.fz;
            if (grp < 3) {
                av[grp] = (double)o.n;
                av[3 + grp] = bout;
            }
        }
    }
    if (acct) block_acct(acct, av);
}

hipError_t launch_transport(bool fp32, int flux, const KGrid &g, int M, double c, double dt, const void *Nin,
                            const void *Fin, void *Nout, void *Fout, const void *hll, int nf, int nth,
                            double *acct, hipStream_t s)
{
    dim3 b(256), gr((unsigned)((g.ncell + 255) / 256));
    const double k = dt / g.dx;
    if (fp32) {
        auto kern = flux ? k_transport<float, 1> : k_transport<float, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, M, (float)c, (float)k, (const float *)Nin, (const float *)Fin,
                           (float *)Nout, (float *)Fout, (const float *)hll, nf, nth, acct);
    } else {
        auto kern = flux ? k_transport<double, 1> : k_transport<double, 0>;
        hipLaunchKernelGGL(kern, gr, b, 0, s, g, M, c, k, (const double *)Nin, (const double *)Fin,
                           (double *)Nout, (double *)Fout, (const double *)hll, nf, nth, acct);
    }
    return hipGetLastError();
}

// --------------------------------------------------------- thermochemistry
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

// Histogram of accepted substeps per cell (bin 63: 63 or more), counted in
// LDS per block and added to the device statistics at the end of the block.
__device__ __forceinline__ void hist_init(unsigned *sh)
{
    if (threadIdx.x < 64) sh[threadIdx.x] = 0u;
    __syncthreads();
}
__device__ __forceinline__ void hist_add(unsigned *sh, int acc) { atomicAdd(&sh[acc < 63 ? acc : 63], 1u); }
__device__ __forceinline__ void hist_flush(const unsigned *sh, unsigned long long *hist)
{
    __syncthreads();
    if (threadIdx.x < 64 && sh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)sh[threadIdx.x]);
}

// Head pass: one thread per cell.  With FUSE the cell is first transported
// (all groups, source set -> registers); then up to K chemistry attempts.
// Cells that finish are written to the destination arrays; the rest go to
// the queue (or, when it is full, finish in place).
// Waves per SIMD the head kernel is compiled for: three (168 VGPRs, a few
// bytes of spill) measured faster than two without spills, also for the
// FP64 three-group variant (191 VGPRs at two waves: 8.7 -> 7.9 ms per head
// launch at 256^3 x 3 once multiply-adds fuse per expression) and for the
// smoothed one (140 bytes of spill at three: 6.9 against 7.5 ms at two).
template <typename R, int M>
constexpr int head_waves() { return 3; }

// V selects the method variant of the chemistry (V_SMOOTH: it starts from
// the radiation before injection and transport, io.sm, and takes their
// change as a rate; V_CASE_A: no on-the-spot approximation).
template <typename R, int M, int FUSE, int FLUX, int V>
__global__ __launch_bounds__(256, (head_waves<R, M>())) void k_head(KGrid g, const KChem *__restrict__ kp, double dt, R c, R kdx, const R *__restrict__ Nin,
                                              const R *__restrict__ Fin, ChemIO<R> io, const R *__restrict__ tab,
                                              int nf, int nth, QueueView q, int K, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < (uint32_t)g.ncell;
    const size_t nc = g.ncell;
    constexpr bool SM = (V & V_SMOOTH) != 0;
    std::conditional_t<SM, CSR, CS> s;
    CC cc{1.0, 0.0, 0.0, 0.0};
    bool done = true;
    unsigned fl = 0;
    double av[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    __shared__ unsigned s_hist[64];
    if (io.hist) hist_init(s_hist);
#pragma unroll
    for (int grp = 0; grp < CM; ++grp) {
        s.N[grp] = 0.0;
        s.fs[grp] = 1.0;
        if constexpr (SM) s.Nr[grp] = 0.0;
    }
    if (valid) {
        bool fin = true;
        if (FUSE) {
            // transport of every group; the flux goes straight to the
            // destination, where the chemistry rescales it at the end
            int ix, iy, iz;
            cell_coords(g, i, ix, iy, iz);
            const Nbr nb = neighbours(g, i, ix, iy, iz);
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                double bout = 0.0;
                const U4<R> o = transport_cell<R, FLUX>(nb, i, nc, Nin + (size_t)grp * nc,
                                                        Fin + (size_t)3 * grp * nc, c, kdx, tab, nf, nth, bout, g,
                                                        grp);
                s.N[grp] = (double)o.n * io.ia3;
                av[grp] = (double)o.n;
                av[3 + grp] = bout;
                io.F[(size_t)(3 * grp) * nc + i] = o.fx;
                io.F[(size_t)(3 * grp + 1) * nc + i] = o.fy;
                io.F[(size_t)(3 * grp + 2) * nc + i] = o.fz;
                fin = fin && isfinite(o.fx) && isfinite(o.fy) && isfinite(o.fz);
            }
        } else {
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                s.N[grp] = (double)io.N[(size_t)grp * nc + i] * io.ia3;
#pragma unroll
                for (int d = 0; d < 3; ++d) fin = fin && isfinite(io.F[(size_t)(3 * grp + d) * nc + i]);
            }
        }
        if constexpr (SM) {
            // N^t from the pre-step set, or for a source cell its value
            // before the injection; rate (N' - N^t)/dt (eq. smoothrate1)
            const int si = io.sm.map ? io.sm.map[i] : -1;
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                const double nt = (si >= 0 ? io.sm.prev[(size_t)si * M + grp] : (double)io.sm.N[(size_t)grp * nc + i]) *
                                  io.ia3;
                s.Nr[grp] = (s.N[grp] - nt) / dt;
                s.N[grp] = nt;
#pragma unroll
                for (int d = 0; d < 3; ++d) fin = fin && isfinite(io.sm.F[(size_t)(3 * grp + d) * nc + i]);
            }
        }
        s.x = io.xHII[i];
        s.y2 = io.xHeII[i];
        s.y3 = io.xHeIII[i];
        cc = make_cc(k, io.nH[i] * io.ia3, io.T[i]);
        if (chem_init<CM, V>(k, dt, cc.Tiso, fin, s)) {
            done = false;
            for (int a = 0; a < K && !done; ++a) done = chem_attempt<CM, V, false>(k, cc, s, fl);
        } else {
            fl |= 2u;
        }
    }
    if (FUSE && io.acct) block_acct(io.acct, av);
    // wave-aggregated enqueue of the unfinished cells, by expected length of
    // their chain of substeps: cells that took many attempts in the previous
    // pass (the fronts move little in a step), then cells that accepted no
    // substep in their K attempts here (a state that changes fast), then the
    // rest.  The tail works the regions off in this order, so that the
    // longest chains start first instead of draining the tail at its end.
    const bool want = !done;
    const int cls = !want ? 3
                          : (io.prev_att && (io.prev_att[i] & ATT_MASK) >= TAIL_LONG_ATTEMPTS) ? 0
                                                                                                 : (s.acc == 0 ? 1 : 2);
    unsigned p = ~0u;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const bool cand = want && p == ~0u && cls <= r;  // a full region passes its cells on
        const unsigned long long m = __ballot(cand);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            unsigned base = 0;
            if (lane_id() == leader) base = atomicAdd(q.cnt[r], (unsigned)__popcll(m));
            base = __shfl(base, leader);
            if (cand) {
                const unsigned k = base + (unsigned)__popcll(m & ((1ull << lane_id()) - 1ull));
                if (k < q.rlen[r]) p = q.rbeg[r] + k;
            }
        }
    }
    bool queued = false;
    if (p != ~0u) {
        q_store(q, p, i, s, cc);
        queued = true;
    }
    if (want && !queued) {
        while (!done) done = chem_attempt<CM, V>(k, cc, s, fl);
    }
    unsigned long long a_acc = 0, a_att = 0;
    if (valid && !queued) {
        const double T = chem_finish<CM>(k, cc, s, fl);
        store_cell<R, M>(io, i, s, T);
        a_acc = (unsigned long long)s.acc;
        a_att = (unsigned long long)s.att;
        if (io.hist) hist_add(s_hist, s.acc);
    }
    if (io.hist) hist_flush(s_hist, io.hist);
    block_stats(st, a_acc, a_att, a_att, fl);
}

// Tail pass over the queue: persistent waves whose lanes each take a queued
// cell, run one attempt per loop trip (an attempt that fails the photon
// check repeats at once with the halved substep), and refill from the
// wave's reservation of queue positions as soon as their cell has filled
// dt_RT, so that a few slow cells do not hold whole waves of finished
// lanes.  Compiled for three waves per SIMD: the smoothed
// variants would otherwise take 176-178 VGPRs and run two (a few bytes of
// spill at three: 4.6 -> 4.0 ms per tail at 256^3 x 3).
template <typename R, int M, int V>
__global__ __launch_bounds__(256, 3) void k_tail(const KChem *__restrict__ kp, ChemIO<R> io, QueueView q, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    // the regions in order: longest expected chains first
    const unsigned n0 = min(*q.cnt[0], q.rlen[0]);
    const unsigned n1 = min(*q.cnt[1], q.rlen[1]);
    const unsigned n = n0 + n1 + min(*q.cnt[2], q.rlen[2]);
    std::conditional_t<(V & V_SMOOTH) != 0, CSR, CS> s;
    // the cell's destination fluxes, loaded with the cell (as in k_chem_all)
    constexpr bool PRE = (V & V_SMOOTH) == 0;
    R fpre[PRE ? 3 * M : 1];
    uint32_t cell = 0;
    CC cc{1.0, 0.0, 0.0, 0.0};
    bool active = false, exhausted = false;
    bool raised = false;
    unsigned rbase = 0, ravail = 0;  // positions this wave has reserved and not yet handed out
    unsigned fl = 0;
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    __shared__ unsigned s_hist[64];
    if (io.hist) hist_init(s_hist);
    while (true) {
        if (!exhausted) {
            bool first = false;
            const bool need = !active;
            const unsigned long long m = __ballot(need);
            if (m) {
                const unsigned nneed = (unsigned)__popcll(m);
                const unsigned r = (unsigned)__popcll(m & ((1ull << lane_id()) - 1ull));
                unsigned t;
                if (ravail >= nneed) {
                    t = rbase + r;
                    rbase += nneed;
                    ravail -= nneed;
                } else {
                    // what is left of the reservation goes first; a new one
                    // of at least TAIL_CHUNK positions covers the rest
                    const unsigned more = nneed - ravail;
                    const unsigned take = more > TAIL_CHUNK ? more : TAIL_CHUNK;
                    const int leader = __ffsll((long long)m) - 1;
                    unsigned base = 0;
                    if (lane_id() == leader) base = atomicAdd(q.head, take);
                    base = __shfl(base, leader);
                    t = r < ravail ? rbase + r : base + (r - ravail);
                    rbase = base + more;
                    ravail = take - more;
                }
                // positions only grow: past n there is nothing left for this wave
                if (rbase >= n) exhausted = true;
                if (need && t < n) {
                    const unsigned pos = t < n0 ? t : (t < n0 + n1 ? q.rbeg[1] + (t - n0) : q.rbeg[2] + (t - n0 - n1));
                    cell = q_load(k, q, pos, s, cc);
                    if constexpr (PRE) {
#pragma unroll
                        for (int j = 0; j < 3 * M; ++j) fpre[j] = io.F[(size_t)j * io.ncell + cell];
                    }
                    active = true;
                    first = t < n0;
                }
            }
            // a wave holding cells of the first region (the longest chains)
            // issues ahead of the others for the rest of its life
            if (!raised && __any(first)) {
                __builtin_amdgcn_s_setprio(3);
                raised = true;
            }
        }
        if (!__any(active)) break;
        if (active) {
            if (chem_attempt<CM, V>(k, cc, s, fl)) {
                const double T = chem_finish<CM>(k, cc, s, fl);
                if constexpr (PRE) store_cell_with<R, M>(io, cell, s, T, fpre);
                else store_cell<R, M>(io, cell, s, T);
                if (io.hist) hist_add(s_hist, s.acc);
                a_acc += (unsigned long long)s.acc;
                a_att += (unsigned long long)s.att;
                a_max = a_max > (unsigned long long)s.att ? a_max : (unsigned long long)s.att;
                active = false;
            }
        }
    }
    if (io.hist) hist_flush(s_hist, io.hist);
    block_stats(st, a_acc, a_att, a_max, fl);
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    for (int k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0u;
}

// Before the one-pass chemistry: the cells whose previous pass took at least
// TAIL_LONG_ATTEMPTS attempts go to a list (the queue's cell array, as many
// as it holds) that the pass takes first, and are marked ATT_LISTED; every
// other mark is cleared.  The count of such cells goes to *cnt (it may
// exceed cap).  A thread takes four consecutive cells (one 4-byte word of
// counts; the array is padded to 256 bytes).
__global__ __launch_bounds__(256) void k_long_list(uint8_t *__restrict__ prev, size_t nc, int32_t *__restrict__ list,
                                                   unsigned cap, unsigned *__restrict__ cnt)
{
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // word index
    const size_t i0 = 4 * q;
    uint32_t o = 0;
    if (i0 < nc) o = reinterpret_cast<const uint32_t *>(prev)[q];
    unsigned want = 0;  // bit j: cell i0 + j is a long chain
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const unsigned v = (o >> (8 * j)) & ATT_MASK;
        if (i0 + j < nc && v >= (unsigned)TAIL_LONG_ATTEMPTS) want |= 1u << j;
    }
    // this lane's first slot: the wanted cells of the lanes before it
    const unsigned c = (unsigned)__popc(want);
    unsigned ex = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned u = __shfl_up(ex, d, 64);
        if (lane_id() >= d) ex += u;
    }
    const unsigned tot = __shfl(ex, 63, 64);
    ex -= c;
    unsigned base = 0;
    if (tot) {
        if (lane_id() == 0) base = atomicAdd(cnt, tot);
        base = __shfl(base, 0, 64);
    }
    uint32_t nw = 0;
    unsigned k = base + ex;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t b = (o >> (8 * j)) & ATT_MASK;
        if (want & (1u << j)) {
            if (k < cap) {
                list[k] = (int32_t)(i0 + j);
                b |= ATT_LISTED;
            }
            ++k;
        }
        nw |= b << (8 * j);
    }
    if (i0 < nc && nw != o) reinterpret_cast<uint32_t *>(prev)[q] = nw;
}

// The chemistry of every cell in one persistent launch (the pass after a
// separate transport): each lane takes a cell, runs its attempts one per
// loop trip (an attempt that fails the photon check repeats at once with the
// halved substep), writes it when it has filled dt_RT and takes the next,
// from its wave's reservation of positions.  Positions run over the list of
// long chains first (their waves issue ahead of the others), then over all
// cells in grid order, passing over the listed ones.  Every cell goes
// through the same attempt code as in the head and tail passes, so results
// are those of the two-pass chemistry bit for bit; what changes is that a
// lane whose cell is done no longer idles until its wave's other lanes are.
template <typename R, int M, int V>
__global__ __launch_bounds__(256, 3) void k_chem_all(const KChem *__restrict__ kp, double dt, ChemIO<R> io, QueueView q,
                                                     unsigned sweep_chunk, DevStats *__restrict__ st)
{
    const KChem &k = *kp;
    constexpr bool SM = (V & V_SMOOTH) != 0;
    const size_t nc = io.ncell;
    const unsigned nl = io.prev_att ? min(*q.cnt[0], q.cap) : 0u;
    const unsigned n = nl + (unsigned)nc;
    std::conditional_t<SM, CSR, CS> s;
    // the cell's destination fluxes, loaded with the cell (not with smoothed
    // RT, whose larger state leaves no registers for them)
    constexpr bool PRE = !SM;
    R fpre[PRE ? 3 * M : 1];
    uint32_t cell = 0;
    CC cc{1.0, 0.0, 0.0, 0.0};
    bool active = false, exhausted = false, raised = false;
    uint8_t mark = 0;
    unsigned rbase = 0, ravail = 0;  // positions this wave has reserved and not yet handed out
    unsigned fl = 0, cfl = 0;        // flags of the lane, flags of its current cell
    unsigned long long a_acc = 0, a_att = 0, a_max = 0;
    __shared__ unsigned s_hist[64];
    if (io.hist) hist_init(s_hist);
    // the cell's state as the head pass loads it, without the check of its
    // fluxes; returns chem_init's verdict
    auto load = [&](uint32_t c, bool fin) -> bool {
        const size_t i = c;
#pragma unroll
        for (int grp = 0; grp < CM; ++grp) {
            s.N[grp] = 0.0;
            s.fs[grp] = 1.0;
            if constexpr (SM) s.Nr[grp] = 0.0;
        }
#pragma unroll
        for (int grp = 0; grp < M; ++grp) s.N[grp] = (double)io.N[(size_t)grp * nc + i] * io.ia3;
        if constexpr (SM) {
            const int si = io.sm.map ? io.sm.map[i] : -1;
#pragma unroll
            for (int grp = 0; grp < M; ++grp) {
                const double nt =
                    (si >= 0 ? io.sm.prev[(size_t)si * M + grp] : (double)io.sm.N[(size_t)grp * nc + i]) * io.ia3;
                s.Nr[grp] = (s.N[grp] - nt) / dt;
                s.N[grp] = nt;
#pragma unroll
                for (int d = 0; d < 3; ++d) fin = fin && isfinite(io.sm.F[(size_t)(3 * grp + d) * nc + i]);
            }
        }
        s.x = io.xHII[i];
        s.y2 = io.xHeII[i];
        s.y3 = io.xHeIII[i];
        cc = make_cc(k, io.nH[i] * io.ia3, io.T[i]);
        // the fluxes are needed only when the cell is written: loaded now,
        // they arrive while the attempts run instead of stalling the wave
        // at the write
        if constexpr (PRE) {
#pragma unroll
            for (int j = 0; j < 3 * M; ++j) fpre[j] = io.F[(size_t)j * nc + i];
        }
        return chem_init<CM, V>(k, dt, cc.Tiso, fin, s);
    };
    // write a cell whose chemistry has ended.  Its fluxes are checked here,
    // where they are used: a non-finite one means the cell is written back
    // as loaded (what the head pass does when it finds one before the
    // chemistry), and the flags of the discarded attempts are dropped
    auto finish = [&]() {
        bool fin = true;
#pragma unroll
        for (int j = 0; j < 3 * M; ++j) fin = fin && isfinite(PRE ? fpre[j] : io.F[(size_t)j * nc + cell]);
        if (!fin) {
            load(cell, false);
            cfl = 2u;
        }
        fl |= cfl;
        const double T = chem_finish<CM>(k, cc, s, fl);
        if constexpr (PRE) store_cell_with<R, M>(io, cell, s, T, fpre, mark);
        else store_cell<R, M>(io, cell, s, T, mark);
        if (io.hist) hist_add(s_hist, s.acc);
        a_acc += (unsigned long long)s.acc;
        a_att += (unsigned long long)s.att;
        a_max = a_max > (unsigned long long)s.att ? a_max : (unsigned long long)s.att;
    };
    while (true) {
        if (!exhausted) {
            bool first = false;
            const bool need = !active;
            const unsigned long long m = __ballot(need);
            if (m) {
                const unsigned nneed = (unsigned)__popcll(m);
                const unsigned r = (unsigned)__popcll(m & ((1ull << lane_id()) - 1ull));
                unsigned t;
                if (ravail >= nneed) {
                    t = rbase + r;
                    rbase += nneed;
                    ravail -= nneed;
                } else {
                    // one wave's width at a time among the long chains, so
                    // that a wave does not hold a second set of them; more
                    // in the sweep (sweep_chunk), where each reservation is
                    // an atomic on the one counter every wave shares
                    const unsigned more = nneed - ravail;
                    const unsigned chunk = rbase < nl ? TAIL_CHUNK : sweep_chunk;
                    const unsigned take = more > chunk ? more : chunk;
                    const int leader = __ffsll((long long)m) - 1;
                    unsigned base = 0;
                    if (lane_id() == leader) base = atomicAdd(q.head, take);
                    base = __shfl(base, leader);
                    t = r < ravail ? rbase + r : base + (r - ravail);
                    rbase = base + more;
                    ravail = take - more;
                }
                if (rbase >= n) exhausted = true;
                if (need && t < n) {
                    bool take = true;
                    if (t < nl) {
                        cell = (uint32_t)q.cell[t];
                        mark = ATT_LISTED;
                        first = true;
                    } else {
                        cell = t - nl;
                        mark = 0;
                        take = !io.prev_att || !(io.prev_att[cell] & ATT_LISTED);
                    }
                    if (take) {
                        cfl = 0;
                        if (load(cell, true)) {
                            active = true;
                        } else {
                            // a non-finite input: the cell is written back as loaded
                            cfl = 2u;
                            finish();
                        }
                    }
                }
            }
            if (!raised && __any(first)) {
                __builtin_amdgcn_s_setprio(3);
                raised = true;
            }
        }
        if (!__any(active)) {
            if (exhausted) break;
            continue;
        }
        if (active && chem_attempt<CM, V>(k, cc, s, cfl)) {
            finish();
            active = false;
        }
    }
    if (io.hist) hist_flush(s_hist, io.hist);
    block_stats(st, a_acc, a_att, a_max, fl);
}

// part 1: reset the queue counters and run the head pass; part 2: the tail
template <typename R, int M, int FUSE, int FLUX, int V>
static void launch_head_tail(int part, const KGrid &g, const KChem &kc, const KChem *dk, double dt, R c, R kdx, const void *Nin,
                             const void *Fin, const ChemIO<R> &io, const void *tab, int nf, int nth,
                             const QueueView &q, int K, DevStats *st, hipStream_t s)
{
    if (part == 1) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, q.count, 65);
        hipLaunchKernelGGL((k_head<R, M, FUSE, FLUX, V>), dim3((unsigned)((g.ncell + 255) / 256)), dim3(256), 0, s, g,
                           dk, dt, c, kdx, (const R *)Nin, (const R *)Fin, io, (const R *)tab, nf, nth, q, K, st);
    } else {
        hipLaunchKernelGGL((k_tail<R, M, V>), dim3(TAIL_BLOCKS), dim3(256), 0, s, dk, io, q, st);
    }
}

template <typename R, int FUSE, int FLUX, int V>
static void dispatch_M(int part, const KGrid &g, const KChem &kc, const KChem *dk, double dt, R c, R kdx, const void *Nin, const void *Fin,
                       const ChemIO<R> &io, const void *tab, int nf, int nth, const QueueView &q, int K,
                       DevStats *st, hipStream_t s)
{
    if (kc.M == 1) launch_head_tail<R, 1, FUSE, FLUX, V>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else if (kc.M == 2) launch_head_tail<R, 2, FUSE, FLUX, V>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else launch_head_tail<R, 3, FUSE, FLUX, V>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
}

template <typename R, int FUSE, int FLUX>
static void dispatch_SM(int part, const KGrid &g, const KChem &kc, const KChem *dk, double dt, R c, R kdx, const void *Nin,
                        const void *Fin, const ChemIO<R> &io, const void *tab, int nf, int nth, const QueueView &q,
                        int K, DevStats *st, hipStream_t s)
{
    const int v = (io.sm.N ? V_SMOOTH : 0) | (kc.otsa ? 0 : V_CASE_A);
    if (v == 0) dispatch_M<R, FUSE, FLUX, 0>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else if (v == 1) dispatch_M<R, FUSE, FLUX, 1>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else if (v == 2) dispatch_M<R, FUSE, FLUX, 2>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
    else dispatch_M<R, FUSE, FLUX, 3>(part, g, kc, dk, dt, c, kdx, Nin, Fin, io, tab, nf, nth, q, K, st, s);
}

template <typename R>
static ChemIO<R> make_io(size_t ncell, void *N, void *F, double *xHII, double *xHeII, double *xHeIII, double *T,
                         const double *nH, int32_t *nacc, int32_t *natt, double *acct, unsigned long long *hist,
                         const SmoothArgs *sm, double dt, double a, uint8_t *prev_att)
{
    ChemIO<R> io;
    io.prev_att = prev_att;
    io.a3 = a * a * a;
    io.ia3 = 1.0 / io.a3;
    io.acct = acct;
    io.hist = hist;
    if (sm) {
        io.sm.N = (const R *)sm->N;
        io.sm.F = (const R *)sm->F;
        io.sm.map = sm->map;
        io.sm.prev = sm->prev;
        io.sm.dt = dt;
    }
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
                       const QueueView &q, int K, unsigned long long *hist, const SmoothArgs *sm, double a,
                       uint8_t *prev_att, DevStats *stats, hipStream_t s)
{
    if (fp32) {
        ChemIO<float> io = make_io<float>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt, nullptr, hist, sm, dt, a,
                                          prev_att);
        dispatch_SM<float, 0, 0>(part, g, kc, dk, dt, 0.f, 0.f, nullptr, nullptr, io, nullptr, 0, 0, q, K, stats, s);
    } else {
        ChemIO<double> io = make_io<double>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt, nullptr, hist, sm, dt, a,
                                            prev_att);
        dispatch_SM<double, 0, 0>(part, g, kc, dk, dt, 0.0, 0.0, nullptr, nullptr, io, nullptr, 0, 0, q, K, stats, s);
    }
    return hipGetLastError();
}

// Positions a wave reserves at a time in the sweep: a quarter of a wave's
// share of the grid, between one wave's width and CHEM_SWEEP_CHUNK (on a
// small grid large reservations would leave the work to a few waves).
static unsigned chem_sweep_chunk(size_t ncell)
{
    const size_t share = ncell / ((size_t)CHEM_ALL_BLOCKS * 4) / 4;
    const size_t c = share < TAIL_CHUNK ? TAIL_CHUNK : (share > CHEM_SWEEP_CHUNK ? CHEM_SWEEP_CHUNK : share);
    return (unsigned)c;
}

// one-pass chemistry: queue counters reset, the list of long chains, then
// the persistent kernel
template <typename R, int M, int V>
static void launch_all(const KChem *dk, double dt, const ChemIO<R> &io, const QueueView &q, DevStats *st,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, q.count, 65);
    if (io.prev_att && io.ncell > 0)
        hipLaunchKernelGGL(k_long_list, dim3((unsigned)((io.ncell + 1023) / 1024)), dim3(256), 0, s, io.prev_att,
                           io.ncell, q.cell, q.cap, q.cnt[0]);
    hipLaunchKernelGGL((k_chem_all<R, M, V>), dim3(CHEM_ALL_BLOCKS), dim3(256), 0, s, dk, dt, io, q,
                       chem_sweep_chunk(io.ncell), st);
}

template <typename R, int V>
static void dispatch_all_M(const KChem &kc, const KChem *dk, double dt, const ChemIO<R> &io, const QueueView &q,
                           DevStats *st, hipStream_t s)
{
    if (kc.M == 1) launch_all<R, 1, V>(dk, dt, io, q, st, s);
    else if (kc.M == 2) launch_all<R, 2, V>(dk, dt, io, q, st, s);
    else launch_all<R, 3, V>(dk, dt, io, q, st, s);
}

template <typename R>
static void dispatch_all(const KChem &kc, const KChem *dk, double dt, const ChemIO<R> &io, const QueueView &q,
                         DevStats *st, hipStream_t s)
{
    const int v = (io.sm.N ? V_SMOOTH : 0) | (kc.otsa ? 0 : V_CASE_A);
    if (v == 0) dispatch_all_M<R, 0>(kc, dk, dt, io, q, st, s);
    else if (v == 1) dispatch_all_M<R, 1>(kc, dk, dt, io, q, st, s);
    else if (v == 2) dispatch_all_M<R, 2>(kc, dk, dt, io, q, st, s);
    else dispatch_all_M<R, 3>(kc, dk, dt, io, q, st, s);
}

hipError_t launch_chem_all(bool fp32, const KGrid &g, const KChem &kc, const KChem *dk, double dt, void *N, void *F,
                           double *xHII, double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc,
                           int32_t *natt, const QueueView &q, unsigned long long *hist, const SmoothArgs *sm, double a,
                           uint8_t *prev_att, DevStats *stats, hipStream_t s)
{
    if (fp32) {
        ChemIO<float> io = make_io<float>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt, nullptr, hist, sm, dt, a,
                                          prev_att);
        dispatch_all<float>(kc, dk, dt, io, q, stats, s);
    } else {
        ChemIO<double> io = make_io<double>(g.ncell, N, F, xHII, xHeII, xHeIII, T, nH, nacc, natt, nullptr, hist, sm, dt,
                                            a, prev_att);
        dispatch_all<double>(kc, dk, dt, io, q, stats, s);
    }
    return hipGetLastError();
}

hipError_t launch_step_fused(int part, bool fp32, int flux, const KGrid &g, const KChem &kc, const KChem *dk, double dt, const void *Nin,
                             const void *Fin, void *Nout, void *Fout, double *xHII, double *xHeII, double *xHeIII,
                             double *T, const double *nH, int32_t *nacc, int32_t *natt, const void *hll, int nf,
                             int nth, const QueueView &q, int K, double *acct, unsigned long long *hist,
                             const SmoothArgs *sm, double a, uint8_t *prev_att, DevStats *stats, hipStream_t s)
{
    // super-comoving transport: light speed a c_r over dt / a^2
    const double kdx = dt / (a * a) / g.dx;
    const double ctr = a * kc.cr;
    if (fp32) {
        ChemIO<float> io = make_io<float>(g.ncell, Nout, Fout, xHII, xHeII, xHeIII, T, nH, nacc, natt, acct, hist, sm, dt, a,
                                          prev_att);
        if (flux)
            dispatch_SM<float, 1, 1>(part, g, kc, dk, dt, (float)ctr, (float)kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
        else
            dispatch_SM<float, 1, 0>(part, g, kc, dk, dt, (float)ctr, (float)kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
    } else {
        ChemIO<double> io = make_io<double>(g.ncell, Nout, Fout, xHII, xHeII, xHeIII, T, nH, nacc, natt, acct, hist, sm,
                                            dt, a, prev_att);
        if (flux)
            dispatch_SM<double, 1, 1>(part, g, kc, dk, dt, ctr, kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
        else
            dispatch_SM<double, 1, 0>(part, g, kc, dk, dt, ctr, kdx, Nin, Fin, io, hll, nf, nth, q, K, stats, s);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- reductions
size_t reduction_scratch_bytes() { return (size_t)RED_BLOCKS * sizeof(RedOut); }

// scratch layout: [reduction partials][queue counters, 512 B]
//                 [cell, acc, att: 3 x cap int32][QV_GRID (or QV_SMOOTH) x cap doubles]
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t queue_bytes(unsigned cap, bool smooth)
{
    return 512 + align256((size_t)cap * 3 * sizeof(int32_t)) +
           (size_t)(smooth ? QV_SMOOTH : QV_GRID) * cap * sizeof(double);
}

size_t queue_cell_bytes(bool smooth) { return 3 * sizeof(int32_t) + (size_t)(smooth ? QV_SMOOTH : QV_GRID) * sizeof(double); }

QueueView queue_view(void *scratch, unsigned cap, unsigned layout_cap)
{
    char *b = (char *)scratch + align256(reduction_scratch_bytes());
    QueueView q;
    q.count = (unsigned *)b;
    q.head = q.count + 1;
    q.cnt[0] = q.count + 64;
    q.cnt[1] = q.count + 32;
    q.cnt[2] = q.count;
    b += 512;
    q.cell = (int32_t *)b;
    q.acc = q.cell + layout_cap;
    q.att = q.acc + layout_cap;
    b += align256((size_t)layout_cap * 3 * sizeof(int32_t));
    q.v = (double *)b;
    q.cap = cap;
    q.rbeg[0] = 0;
    q.rlen[0] = cap / 16;
    q.rbeg[1] = q.rlen[0];
    q.rlen[1] = cap / 4;
    q.rbeg[2] = q.rbeg[1] + q.rlen[1];
    q.rlen[2] = cap - q.rbeg[2];
    q.stride = layout_cap;
    return q;
}

// Sum over the 64 lanes of a wavefront by butterfly exchanges: every lane
// ends with the same total, combined in the same order on every run.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// Diagnostics of a state (rt_get_stats): per block, grid-stride over the
// cells in a fixed order, then wave butterflies and the block's four waves
// in order.
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
    __shared__ double s[RED_THREADS / 64][6];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double v[6] = {wave_sum(ph[0]), wave_sum(ph[1]), wave_sum(ph[2]), wave_sum(ion), wave_max(mf),
                         wave_min(mn)};
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) s[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) a[q] = s[0][q];
        for (int k = 1; k < RED_THREADS / 64; ++k) {
            for (int q = 0; q < 4; ++q) a[q] += s[k][q];
            a[4] = s[k][4] > a[4] ? s[k][4] : a[4];
            a[5] = s[k][5] < a[5] ? s[k][5] : a[5];
        }
        RedOut r;
        for (int g = 0; g < 3; ++g) r.photons[g] = a[g] * V;
        r.ionised = a[3] * V;
        r.maxf = a[4];
        r.minN = a[5];
        part[blockIdx.x] = r;
    }
}

// The block partials in a fixed order: each of 256 threads combines the
// partials t, t + 256, ... in turn, then a tree over the threads.
__global__ __launch_bounds__(256) void k_reduce_final(const RedOut *__restrict__ part, int np, RedOut *__restrict__ out)
{
    __shared__ double s[6][256];
    const int t = threadIdx.x;
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 1e300};
    for (int b = t; b < np; b += 256) {
        const RedOut &r = part[b];
        for (int g = 0; g < 3; ++g) a[g] += r.photons[g];
        a[3] += r.ionised;
        a[4] = r.maxf > a[4] ? r.maxf : a[4];
        a[5] = r.minN < a[5] ? r.minN : a[5];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q][t] = a[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            for (int q = 0; q < 4; ++q) s[q][t] += s[q][t + o];
            s[4][t] = s[4][t + o] > s[4][t] ? s[4][t + o] : s[4][t];
            s[5][t] = s[5][t + o] < s[5][t] ? s[5][t + o] : s[5][t];
        }
        __syncthreads();
    }
    if (t == 0) {
        RedOut r;
        for (int g = 0; g < 3; ++g) r.photons[g] = s[g][0];
        r.ionised = s[3][0];
        r.maxf = s[4][0];
        r.minN = s[5][0];
        *out = r;
    }
}

// Four consecutive values of a group plane (16-byte aligned): one 16-byte
// load for FP32, two for FP64.
__device__ __forceinline__ void load4(const float *p, double v[4])
{
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
}
__device__ __forceinline__ void load4(const double *p, double v[4])
{
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// Photons per group of one radiation set, for the step's ledger: per block
// the sum of N of each group (grid-stride in a fixed order, wave
// butterflies, the four waves in order) at part[3 b + g].  When every group
// plane starts 16-byte aligned a thread takes four consecutive cells per
// round, two rounds' loads in flight before their sums.
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_sum_n(size_t nc, int M, const R *__restrict__ N,
                                                       double *__restrict__ part)
{
    double sg[3] = {0.0, 0.0, 0.0};
    const size_t T = (size_t)gridDim.x * blockDim.x, t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t i0 = 0;
    if (((uintptr_t)N & 15) == 0 && ((nc * sizeof(R)) & 15) == 0) {
        const size_t n4 = nc / 4;
        size_t q = t0;
        for (; q + T < n4; q += 2 * T) {
            double v[3][2][4];
#pragma unroll
            for (int g = 0; g < 3; ++g)
                if (g < M) {
                    load4(N + (size_t)g * nc + 4 * q, v[g][0]);
                    load4(N + (size_t)g * nc + 4 * (q + T), v[g][1]);
                }
#pragma unroll
            for (int g = 0; g < 3; ++g)
                if (g < M)
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int j = 0; j < 4; ++j) sg[g] += v[g][r][j];
        }
        for (; q < n4; q += T) {
#pragma unroll
            for (int g = 0; g < 3; ++g)
                if (g < M) {
                    double v[4];
                    load4(N + (size_t)g * nc + 4 * q, v);
#pragma unroll
                    for (int j = 0; j < 4; ++j) sg[g] += v[j];
                }
        }
        i0 = 4 * n4;
    }
    for (size_t i = i0 + t0; i < nc; i += T)
        for (int g = 0; g < M; ++g) sg[g] += (double)N[(size_t)g * nc + i];
    __shared__ double s[RED_THREADS / 64][3];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const double v = wave_sum(sg[g]);
        if (lane == 0) s[w][g] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double a = s[0][threadIdx.x];
        for (int k = 1; k < RED_THREADS / 64; ++k) a += s[k][threadIdx.x];
        part[(size_t)3 * blockIdx.x + threadIdx.x] = a;
    }
}

hipError_t launch_sum_n(bool fp32, size_t ncell, int M, const void *N, double *part, hipStream_t s)
{
    if (fp32)
        hipLaunchKernelGGL(k_sum_n<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, ncell, M, (const float *)N, part);
    else
        hipLaunchKernelGGL(k_sum_n<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, ncell, M, (const double *)N,
                           part);
    return hipGetLastError();
}

// Photon ledger of one step (fixed-order sums; see launch_ledger): the
// photons of the current set from the k_sum_n partials, and with mode 2 the
// transported photons and the boundary outflow from the transport partials.
__global__ __launch_bounds__(256) void k_ledger(int mode, const double *__restrict__ acct, unsigned nblk,
                                                const double *__restrict__ npart, int M, double V, double dtdx2,
                                                DevStats *__restrict__ st)
{
    __shared__ double sh[9][256];
    const int t = threadIdx.x;
    double v[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (mode == 2)
        for (unsigned b = t; b < nblk; b += 256)
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] += acct[(size_t)6 * b + q];
    for (unsigned b = t; b < (unsigned)RED_BLOCKS; b += 256)
#pragma unroll
        for (int g = 0; g < 3; ++g) v[6 + g] += npart[(size_t)3 * b + g];
#pragma unroll
    for (int q = 0; q < 9; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o)
#pragma unroll
            for (int q = 0; q < 9; ++q) sh[q][t] += sh[q][t + o];
        __syncthreads();
    }
    if (t != 0) return;
    for (int g = 0; g < M; ++g) {
        const double now = sh[6 + g][0] * V;
        if (mode == 0) {
            st->Tpre[g] = now;
            continue;
        }
        const double T0 = mode == 2 ? sh[g][0] * V : st->Tpre[g];
        st->absorbed[g] += T0 - now;
        if (mode == 2) st->outflow[g] += sh[3 + g][0] * dtdx2;
    }
}

hipError_t launch_ledger(int mode, const double *acct, unsigned nblk, const double *npart, int M, double V,
                         double dtdx2, DevStats *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_ledger, dim3(1), dim3(256), 0, s, mode, acct, nblk, npart, M, V, dtdx2, st);
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, part, RED_BLOCKS, dev_out);
    return hipGetLastError();
}

}  // namespace rtm1
