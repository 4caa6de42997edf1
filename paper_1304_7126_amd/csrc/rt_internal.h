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
};

struct KChem {
    int M;
    int isothermal;
    double cr;
    double sN[3][3];
    double sE[3][3];
    double eb[3];
    double X, Y;
    double Kfac;   // (gamma-1) X / k_B ; K = Kfac / n_H
    double a_exp;
    double x_min;
    double N_floor;
    long long max_att;
};

// device statistics block (in library memory)
struct DevStats {
    unsigned long long acc_total;
    unsigned long long att_total;
    unsigned long long att_max;
    unsigned int flags;
    unsigned int pad;
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

hipError_t launch_inject(bool fp32, void *N, size_t ncell, int M, int nsrc, const int32_t *cell,
                         const double *rate, double dt_over_V, hipStream_t s);

hipError_t launch_transport(bool fp32, int flux, const KGrid &g, int M, double c, double dt,
                            const void *Nin, const void *Fin, void *Nout, void *Fout, const void *hll,
                            int nf, int nth, hipStream_t s);

hipError_t launch_chem(bool fp32, const KChem &kc, size_t ncell, double dt, void *N, void *F, double *xHII,
                       double *xHeII, double *xHeIII, double *T, const double *nH, int32_t *nacc,
                       int32_t *natt, DevStats *stats, hipStream_t s);

hipError_t launch_reduce(bool fp32, size_t ncell, int M, double c, double V, const void *N, const void *F,
                         const double *xHII, const double *nH, void *scratch, RedOut *dev_out,
                         hipStream_t s);

}  // namespace rtm1
