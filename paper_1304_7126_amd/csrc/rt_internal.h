// rt_internal.h -- launch interface between the C ABI (rt_api.hip) and the
// gfx950 kernels (rt_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rtm1 {

// everything a kernel needs to know about the grid and the groups
struct KGrid {
    int nx, ny, nz;
    int bc[6];
    size_t ncell;
    double dx;
    double inflow[6][3];  // RT_BC_INFLOW faces: photon flux [s^-1 cm^-2] entering, per group
};

struct KChem {
    int M;
    int isothermal;
    double cr;
    double sN[3][3];
    double sE[3][3];
    double eb[3];
    double csN[3][3];  // c_r sigN[g][j]: absorption and photoionisation rate per photon
    double hc[3][3];   // c_r (ebar_g sigE[g][j] - eps_j sigN[g][j]): photoheating per photon
    double X, Y;
    double Kfac;   // (gamma-1) X / k_B ; K = Kfac / n_H
    double a_exp;
    double x_min;
    double N_floor;
    long long max_att;
    int otsa;           // 1: on-the-spot approximation; 0: case A with recombination photons
    double brec[3][3];  // [group][HII, HeII, HeIII]: 1 where the species' recombination photons go
};

// device statistics block (in library memory)
struct DevStats {
    unsigned long long acc_total;
    unsigned long long att_total;
    unsigned long long att_max;
    unsigned int flags;
    unsigned int pad;
    // photon accounting (rt_set_accounting): photons absorbed by the
    // chemistry and carried out through boundary faces, per group; the
    // pre-chemistry total of a step; histogram of accepted substeps per cell
    double absorbed[3], outflow[3], Tpre[3];
    unsigned long long hist[64];
};

// final reduction record (in caller scratch)
struct RedOut {
    double photons[3];
    double ionised;
    double maxf;
    double minN;
};

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
size_t reduction_scratch_bytes();

// prev (nsrc*M doubles, or null): receives each source cell's N before the
// injection, for smoothed RT
hipError_t launch_inject(bool fp32, void *N, size_t ncell, int M, int nsrc, const int32_t *cell,
                         const double *rate, double dt_over_V, double *prev, hipStream_t s);

// p[0..n) = v with a kernel (no memset node in a captured graph)
hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s);

// map[cell] = index of the source in that cell, -1 elsewhere
hipError_t launch_source_map(int32_t *map, size_t ncell, const int32_t *cell, int nsrc, hipStream_t s);

// Inputs of smoothed RT: the radiation set before injection and transport
// (N, F), and for source cells their N before the injection (map, prev; map
// null when no injection preceded the transport).
struct SmoothArgs {
    const void *N, *F;
    const int32_t *map;
    const double *prev;
};

// accounting partials: 6 doubles per transport block (sum of transported N
// and of the outward boundary flux, per group), in caller scratch
constexpr int ACCT_THREADS = 256;
size_t acct_bytes(size_t ncell);
unsigned acct_blocks(size_t ncell);

hipError_t launch_transport(bool fp32, int flux, const KGrid &g, int M, double c, double dt,
                            const void *Nin, const void *Fin, void *Nout, void *Fout, const void *hll,
                            int nf, int nth, double *acct, hipStream_t s);

// The z-marching transport (rt_transport.hip): same results as
// launch_transport, for grids whose x-rows fit one workgroup (nx <= 1024 in
// FP32, 512 in FP64; transport_z_fits).  acct: per workgroup, the sum of the
// new N and of the outward boundary flux of its group, at 6 b + g and
// 6 b + 3 + g for b < transport_z_blocks().
bool transport_z_fits(bool fp32, const KGrid &g);
unsigned transport_z_blocks(bool fp32, const KGrid &g, int M);
hipError_t launch_transport_z(bool fp32, int flux, const KGrid &g, int M, double c, double dt, const void *Nin,
                              const void *Fin, void *Nout, void *Fout, const void *hll, int nf, int nth, double *acct,
                              hipStream_t s);

// per-block sums of N of each group of a radiation set: RED_BLOCKS x 3
// doubles at part (launch_ledger reads them)
hipError_t launch_sum_n(bool fp32, size_t ncell, int M, const void *N, double *part, hipStream_t s);

// mode 0: record the current photon totals as the pre-chemistry totals;
// mode 1: absorbed += pre-chemistry totals - current totals;
// mode 2: as 1 with the pre-chemistry totals and the outflow taken from the
// transport partials.  npart: launch_sum_n partials of the current set.
hipError_t launch_ledger(int mode, const double *acct, unsigned nblk, const double *npart, int M, double V,
                         double dtdx2, DevStats *st, hipStream_t s);

// queue of cells still subcycling after the head pass (caller scratch), in
// three regions the tail works off in order: cells that took many attempts
// in the previous pass, cells that accepted no substep in this one's first
// attempts, the rest.  A region that is full passes its cells to the next.
struct QueueView {
    unsigned *count;    // the counter block: [0] region 2, [1] cells taken by the tail, [32] region 1, [64] region 0
    unsigned *head;
    unsigned *cnt[3];   // cells queued per region (each on its own cache line)
    unsigned rbeg[3], rlen[3];  // region offsets and sizes
    int32_t *cell, *acc, *att;
    double *v;          // QV_GRID (smoothed RT: QV_SMOOTH) planes of `stride` doubles
    unsigned cap;       // cells the head pass may queue
    unsigned stride;    // plane length of the layout
};

template <typename R>
struct SmoothIn {
    const R *N = nullptr, *F = nullptr;  // radiation set before injection and transport
    const int32_t *map = nullptr;        // source index per cell, or null
    const double *prev = nullptr;        // N of each source cell before injection
    double dt = 0.0;
};

template <typename R>
struct ChemIO {
    size_t ncell;
    R *N, *F;  // destination radiation set
    double *xHII, *xHeII, *xHeIII, *T;
    const double *nH;
    int32_t *nacc, *natt;
    double *acct;               // transport partials (fused head), or null
    unsigned long long *hist;   // substep histogram, or null
    SmoothIn<R> sm;             // smoothed RT inputs (kernels instantiated for it)
    // super-comoving state (a != 1): the arrays hold a^3 N and a^3 n_H, the
    // chemistry works on N and n_H
    double a3 = 1.0, ia3 = 1.0;
    // attempts of each cell in the previous chemistry pass (capped at 255),
    // read to order the tail and rewritten; null: not kept
    uint8_t *prev_att = nullptr;
};

constexpr int TAIL_BLOCKS = 1024;
// workgroups of the one-pass chemistry kernel (persistent; 256 threads each)
#ifndef RT_CHEM_ALL_BLOCKS
#define RT_CHEM_ALL_BLOCKS 1024
#endif
constexpr int CHEM_ALL_BLOCKS = RT_CHEM_ALL_BLOCKS;
constexpr int HEAD_ATTEMPTS = 3;

// bytes of scratch for a queue of cap cells (after the reduction partials),
// laid out for smoothed RT when smooth is set
size_t queue_bytes(unsigned cap, bool smooth);
// bytes one queued cell takes (without the alignment of the layout)
size_t queue_cell_bytes(bool smooth);
// cap: cells the kernels may queue; layout_cap: capacity the scratch is laid out for
QueueView queue_view(void *scratch, unsigned cap, unsigned layout_cap);

// the chemistry in one persistent pass over all cells (same results as the
// head and tail passes); the queue's counters and cell array hold its
// position counter and its list of long chains
hipError_t launch_chem_all(bool fp32, const KGrid &g, const KChem &kc, const KChem *dk, double dt, void *N, void *F,
                           double *xHII, double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc,
                           int32_t *natt, const QueueView &q, unsigned long long *hist, const SmoothArgs *sm, double a,
                           uint8_t *prev_att, DevStats *stats, hipStream_t s);

// part 1: queue reset + head pass; part 2: tail pass
hipError_t launch_chem(int part, bool fp32, const KGrid &g, const KChem &kc, const KChem *dk, double dt, void *N, void *F, double *xHII,
                       double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc, int32_t *natt,
                       const QueueView &q, int K, unsigned long long *hist, const SmoothArgs *sm, double a,
                       uint8_t *prev_att, DevStats *stats, hipStream_t s);

hipError_t launch_step_fused(int part, bool fp32, int flux, const KGrid &g, const KChem &kc, const KChem *dk, double dt, const void *Nin,
                             const void *Fin, void *Nout, void *Fout, double *xHII, double *xHeII, double *xHeIII,
                             double *T, const double *nH, int32_t *nacc, int32_t *natt, const void *hll, int nf,
                             int nth, const QueueView &q, int K, double *acct, unsigned long long *hist,
                             const SmoothArgs *sm, double a, uint8_t *prev_att, DevStats *stats, hipStream_t s);

hipError_t launch_reduce(bool fp32, size_t ncell, int M, double c, double V, const void *N, const void *F,
                         const double *xHII, const double *nH, void *scratch, RedOut *dev_out,
                         hipStream_t s);

// ionisation energies of HI, HeI, HeII [erg] (App. E.4)
constexpr double EPS_ION_ERG[3] = {13.60 * 1.602176634e-12, 24.59 * 1.602176634e-12, 54.42 * 1.602176634e-12};

// fill the derived per-photon rates csN, hc from cr, sN, sE, eb
inline void kchem_derive(KChem &k)
{
    for (int g = 0; g < 3; ++g)
        for (int j = 0; j < 3; ++j) {
            k.csN[g][j] = k.sN[g][j] * k.cr;
            k.hc[g][j] = k.cr * (k.eb[g] * k.sE[g][j] - EPS_ION_ERG[j] * k.sN[g][j]);
        }
}

// differentiation form (rt_adjoint.hip)
size_t adj_scan_parts(size_t nc);
hipError_t launch_offsets(const int32_t *counts, size_t nc, int64_t *off, hipStream_t s);
template <typename R>
hipError_t launch_chem_record(const KChem *dk, size_t nc, double dt, R *N, R *F, double *xHII, double *T,
                              const double *nH, const int32_t *counts, const int64_t *off, long long cap,
                              double *trace, DevStats *st, hipStream_t s);
template <typename R>
hipError_t launch_chem_replay(const KChem *dk, size_t nc, R *N, R *F, double *xHII, double *T, const double *nH,
                              const int32_t *counts, const int64_t *off, long long cap, const double *trace,
                              hipStream_t s);
hipError_t launch_widen(const float *a, double *b, size_t n, hipStream_t s);
hipError_t launch_chem_adj(const KChem *dk, size_t nc, const double *nH, const int32_t *counts, const int64_t *off,
                           long long cap, const double *trace, const double *lN, const double *lF, double *lx,
                           double *lT, double *wN, double *wF, double *g, hipStream_t s);
hipError_t launch_transport_adj(const KGrid &g, double c, double kdx, const double *Na, const double *Fa,
                                const double *lNb, const double *lFb, double *lNa, double *lFa, hipStream_t s);
hipError_t launch_inject_adj(const double *lN, int nsrc, const int32_t *cell, const double *ndot, double dtV,
                             double *g, hipStream_t s);

}  // namespace rtm1
