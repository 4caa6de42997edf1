/*
 * rtm1.h -- C ABI of the MI355X explicit M1 radiative-transfer step.
 *
 * The library advances, on one uniform Cartesian grid, the photon number
 * densities N_i and fluxes F_i of M <= 3 photon groups together with the
 * hydrogen/helium ionisation state and temperature of the gas, with the
 * method of Rosdahl et al. (2013), "RAMSES-RT":
 *   - injection of point-source photons          (Sec. 3.1, eq. injnum)
 *   - explicit GLF or HLL transport of (N, F) with the M1 closure at a
 *     reduced light speed c_r, unsplit in 3D     (Sec. 2; Sec. 3.2, eqs.
 *                                                   dUdt_sol, hll, glf;
 *                                                   Sec. 4.1; App. D)
 *   - per-cell non-equilibrium thermochemistry, subcycled by the 10% rule
 *                                                  (Sec. 3.3; App. A; App. E)
 * operator-split in that order over one time step (Sec. 3).
 *
 * Conventions for every entry point:
 *   - cgs units.  Radiation: N [cm^-3], F [cm^-2 s^-1].  T [K].
 *   - Grids are structure-of-arrays with x fastest: cell (ix,iy,iz) has
 *     linear index i = ix + nx*(iy + ny*iz), ncell = nx*ny*nz.
 *   - Device pointers are caller-owned (e.g. torch tensors) and must stay
 *     valid while bound.  The library allocates only its own small tables
 *     (HLL eigenvalue table, source list, statistics block); it never
 *     allocates or frees state arrays.
 *   - All device work is enqueued on the bound HIP stream and is
 *     asynchronous; only rt_get_stats and rt_free synchronise.
 *   - Host-side validation failures return a negative rt_status without
 *     enqueueing anything; rt_last_error() gives the message.  Device-side
 *     anomalies set bits in rt_stats.flags.
 *   - A context is not thread-safe.
 */
#ifndef RTM1_H
#define RTM1_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_EINVAL = -1,       /* invalid argument                           */
    RT_EHIP = -2,         /* a HIP runtime call failed                   */
    RT_ENOMEM = -3,       /* library table allocation failed             */
    RT_ESTATE = -4,       /* call not valid in the current context state */
    RT_EUNSUPPORTED = -5  /* option not supported                        */
} rt_status;

enum { RT_BC_PERIODIC = 0, RT_BC_OUTFLOW = 1, RT_BC_REFLECT = 2, RT_BC_INFLOW = 3 };
enum { RT_FLUX_GLF = 0, RT_FLUX_HLL = 1 };
/* RT_PREC_FP64: N, F stored and transported in FP64.
 * RT_PREC_FP32_TRANSPORT: N, F stored and transported in FP32; the
 * thermochemistry always runs in FP64. */
enum { RT_PREC_FP64 = 0, RT_PREC_FP32_TRANSPORT = 1 };

/* device-side anomaly bits of rt_stats.flags */
#define RT_FLAG_CAP 1u   /* a cell hit max_attempts before filling dt (left at its last accepted state) */
#define RT_FLAG_NAN 2u   /* a non-finite value was produced                                            */
#define RT_FLAG_NNEG 8u  /* a negative photon density after the chemistry                               */
#define RT_FLAG_TRACE 16u /* rt_step_record: a cell took another number of substeps than tape.counts,
                             or the trace capacity was too small (the adjoint of that cell is wrong)   */

/* Grid: nx, ny, nz >= 1 cells of width dx [cm].  bc[] for the faces
 * -x,+x,-y,+y,-z,+z: periodic (must be set on both faces of an axis),
 * outflow (ghost cell copies the boundary cell), reflect (ghost mirrors
 * the boundary cell with the normal flux component negated) or inflow
 * (ghost holds a beam entering the grid, set by rt_set_inflow; zero until
 * then). */
typedef struct {
    int nx, ny, nz;
    double dx;
    int bc[6];
} rt_grid;

/* Photon groups (Sec. 2): M in 1..3; reduced light speed c_r [cm/s];
 * group-averaged cross sections sigN (eq. csn_multi) and energy-weighted
 * cross sections sigE (eq. cse_multi) [cm^2], indexed [group][HI,HeI,HeII];
 * mean photon energies ebar (eq. egy_multi) [erg].  Rows >= M are ignored.
 * brec[j]: the group that receives the photons of recombinations straight to
 * the ground state of HII, HeII, HeIII (j = 0, 1, 2; the b^rec of eq.
 * cool_N_cr), normally the group holding the species' ionisation threshold;
 * -1: none.  Read only with otsa = 0. */
typedef struct {
    int M;
    double c_r;
    double sigN[3][3];
    double sigE[3][3];
    double ebar[3];
    int brec[3];
} rt_groups;

/* Method options.
 *   flux        RT_FLUX_GLF (eq. glf) or RT_FLUX_HLL (eq. hll)
 *   otsa        on-the-spot approximation (Sec. 3.3.2): 1 = case-B rates, no
 *               recombination photons; 0 = case-A recombination rates and
 *               recombination cooling, and the photons of recombinations
 *               straight to the ground state, (alpha_A - alpha_B) n_j n_e
 *               with the state at the start of each substep, added to group
 *               brec[j] (eq. cool_N_cr).  The batch and the adjoint need 1.
 *   isothermal  hold T fixed in the thermochemistry (no thermal update)
 *   prec        RT_PREC_FP64 or RT_PREC_FP32_TRANSPORT
 *   X, Y        hydrogen and helium mass fractions (X > 0, Y >= 0)
 *   gamma       ratio of specific heats (5/3)
 *   a_exp       expansion factor in the Compton term (1 for static boxes)
 *   x_min       floor on x_HII (1e-6 in the paper's tests)
 *   N_floor     photon densities <= N_floor skip the 10% check (0: only
 *               empty groups skip it, as written in App. A)
 *   max_attempts cap on chemistry attempts per cell per step (>= 1)
 *   smooth      smoothed RT (Sec. 4.4): 1 = the thermochemistry starts from
 *               N, F before the step's injection and transport and adds
 *               their change as constant rates (eqs. thchem_N_smooth,
 *               thchem_F_smooth, smoothrate1, smoothrate2); 0 = plain
 *               operator splitting.  The batch and the adjoint need 0. */
typedef struct {
    int flux;
    int otsa;
    int isothermal;
    int prec;
    double X, Y;
    double gamma;
    double a_exp;
    double x_min;
    double N_floor;
    long long max_attempts;
    int smooth;
} rt_params;

/* Caller-owned state.
 *   N[s]  radiation set s (s = 0, 1): M*ncell elements, layout [g][cell]
 *   F[s]  3*M*ncell elements, layout [g][axis][cell]
 *         element type: double (RT_PREC_FP64) or float (FP32 transport).
 *         Transport reads the current set and writes the other (the
 *         source/destination copies of App. D); rt_current() says which
 *         set holds the current state.
 *   xHII, xHeII, xHeIII, T   FP64, ncell each, updated in place
 *   nH    FP64, ncell, hydrogen number density [cm^-3], read only
 *   nacc, natt  optional int32 per-cell counters of accepted substeps and
 *         of attempts in the last thermochemistry pass (NULL: not written)
 *   scratch  device buffer of at least rt_scratch_bytes() bytes: reduction
 *         partials, the queue of cells still subcycling after the first
 *         chemistry pass, accounting partials, each cell's attempt count
 *         of the previous pass (which orders the queue; rt_bind clears it)
 *         and, with smooth = 1, each cell's source index (rt_bind and
 *         rt_set_sources write it).
 *         The library owns its contents while it is bound.  May be NULL
 *         (with scratch_bytes = 0) for a context stepped only with
 *         rt_step_noalloc: rt_step, rt_thermochem, rt_get_stats and the
 *         accounting then return RT_ESTATE. */
typedef struct {
    void *N[2];
    void *F[2];
    double *xHII, *xHeII, *xHeIII, *T;
    const double *nH;
    int32_t *nacc, *natt;
    void *scratch;
    size_t scratch_bytes;
} rt_state;

/* Diagnostics of the current state plus counters accumulated since the
 * last rt_reset_stats (Sec. 3.3.1 subcycling statistics). */
typedef struct {
    double photons[3];        /* sum_cells N_g dx^3                                 */
    double ionised_H;         /* sum_cells x_HII n_H dx^3 (H ions)                  */
    double max_f;             /* max reduced flux |F|/(c_r N) over cells with N > 0 */
    double min_N;             /* min N over all groups and cells                    */
    long long substeps_total; /* accepted chemistry substeps                        */
    long long attempts_total; /* chemistry attempts (accepted + restarted)          */
    long long attempts_max;   /* largest per-cell attempt count in one step         */
    unsigned flags;           /* RT_FLAG_* bits                                     */
    /* photon accounting, filled while rt_set_accounting is on (zero otherwise):
     * per group, photons injected by the sources, absorbed by the chemistry
     * (totals entering minus leaving each chemistry pass) and carried out of
     * the grid through outflow or reflecting faces by the transport; with
     * photons(t) = photons(t0) + injected - absorbed - outflow as the budget
     * (Sec. 3 operator split).  substep_hist[k] counts cell-steps with k
     * accepted chemistry substeps (k = 63: 63 or more). */
    double injected[3];
    double absorbed[3];
    double outflow[3];
    long long substep_hist[64];
} rt_stats;

typedef struct rt_ctx rt_ctx;

/* Create a context.  Validates the arguments, builds the HLL eigenvalue
 * table (Sec. 3.2: extreme eigenvalues of the M1 flux Jacobian on 101x101
 * nodes of reduced flux f in [0,1] and flux angle in [0,pi]) and uploads it.
 * Returns RT_OK and *out, or an error (then *out = NULL). */
rt_status rt_init(const rt_grid *grid, const rt_groups *groups, const rt_params *params, rt_ctx **out);

/* Bytes of device scratch the bound state must provide. */
size_t rt_scratch_bytes(const rt_ctx *ctx);

/* Bind caller memory (no copies).  Sets the current radiation set to 0. */
rt_status rt_bind(rt_ctx *ctx, const rt_state *state);

/* Enqueue all later work on this hipStream_t (NULL = the null stream). */
rt_status rt_set_stream(rt_ctx *ctx, void *hip_stream);

/* Which radiation set (0 or 1) holds the current N, F; and set it. */
int rt_current(const rt_ctx *ctx);
rt_status rt_set_current(rt_ctx *ctx, int set);

/* Point sources (Sec. 3.1 with f_esc = 1): n sources at host ijk[3*s+0..2]
 * = (ix,iy,iz), emitting host ndot[s*M + g] photons/s into group g.
 * Sources in one cell are summed in input order.  n = 0 removes all. */
rt_status rt_set_sources(rt_ctx *ctx, int n, const int32_t *ijk, const double *ndot);

/* Boundary-flux source (the x = 0 face of Iliev test 3, Sec. 6): face (0..5,
 * -x,+x,-y,+y,-z,+z) must be an RT_BC_INFLOW face; host flux[g] >= 0 is the
 * photon flux [s^-1 cm^-2] of group g entering through it, held by the
 * ghost cell as a beam N = flux / c_r along the inward normal.  Returns
 * RT_EINVAL for another face kind or a negative or non-finite flux. */
rt_status rt_set_inflow(rt_ctx *ctx, int face, const double *flux);

/* Super-comoving RT variables (Sec. 5.4) at expansion factor a > 0 (1: a
 * static box, the default).  With a != 1 the state arrays hold N~ = a^3 N,
 * F~ = a^4 F (the paper's variables in units with H_0 L = 1) and a^3 n_H,
 * and dx is the comoving cell width; the inflow fluxes of rt_set_inflow are
 * F~ as well.  The transport runs with light speed a c_r over dt / a^2, the
 * chemistry on N, n_H, and the Compton term at a (this sets rt_params.a_exp
 * to a); dt stays the physical step, at most a dx / (3 c_r).  Between calls
 * the caller may change a: N~, F~ held fixed dilute N as a^-3 and F as
 * a^-4.  Synchronises the stream.  The adjoint needs a = 1. */
rt_status rt_set_expansion(rt_ctx *ctx, double a);

/* Courant-limited step dt = courant * a dx / (3 c_r) (Sec. 4.1, eq.
 * dt_courant, with the factor 0.8 of the paper's tests). */
rt_status rt_courant_dt(const rt_ctx *ctx, double courant, double *dt);

/* Injection: N_g(cell) += ndot_g dt / dx^3 in the current set.
 * With smooth = 1 a step's calls must come in the order rt_inject (at most
 * once, optional), rt_transport, rt_thermochem; the library keeps each
 * source cell's N from before the injection, and a call out of that order
 * returns RT_ESTATE.  rt_bind, rt_set_current and rt_set_sources start a new
 * step. */
rt_status rt_inject(rt_ctx *ctx, double dt);

/* Transport (Sec. 3.2) of every group over dt from the current set into the
 * other set, which then becomes current.  dt must satisfy dt <= dx/(3 c_r).
 * With HLL a flux that comes out above c_r N (N > 0) is scaled back to
 * c_r N; without it an exact beam next to an inflow face is unstable. */
rt_status rt_transport(rt_ctx *ctx, double dt);

/* Thermochemistry (App. A) of every cell over dt on the current set.  With
 * smooth = 1 each cell starts from N^t, F^t (the other set, and for source
 * cells N before the injection) and receives (N' - N^t)/dt and
 * (F' - F^t)/dt, N', F' being the current set, as constant rates (Sec. 4.4). */
rt_status rt_thermochem(rt_ctx *ctx, double dt);

/* nsteps full steps: injection, transport, thermochemistry (Sec. 3).
 * The result equals rt_inject, rt_transport, rt_thermochem in sequence,
 * bit for bit, whichever transport kernel runs (rt_set_transport_path).
 * dt <= 0 uses the Courant step with factor 0.8. */
rt_status rt_step(rt_ctx *ctx, double dt, int nsteps);

/* rt_step without the bound scratch, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the state must be bound (rt_bind
 * accepts scratch = NULL, scratch_bytes = 0), and the reduction partials,
 * the chemistry queue, the accounting partials and the previous pass's
 * attempt counts go to a static device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends.  The queue takes
 * what the array has left (cells beyond it finish in the first chemistry
 * pass); results are the bits rt_step gives.  Allocates nothing and makes
 * no timing events.  RT_EINVAL when the grid needs more than the array
 * (about 1 + 48/256 bytes per cell besides the queue: up to ~56 M cells),
 * RT_EUNSUPPORTED with smooth = 1.  Every call on a GPU shares its array and
 * leaves its contents behind: calls that overlap on one GPU (two contexts on
 * two streams) race and must be serialised by the caller. */
rt_status rt_step_noalloc(rt_ctx *ctx, double dt, int nsteps);

/* Kernel arrangement of the transport (Sec. 3.2); results are the same bits
 * on every path:
 *   RT_PATH_AUTO    the z-marching kernel where it fits, else per cell
 *   RT_PATH_CELL    one thread per cell evaluates its whole 7-point stencil;
 *                   rt_step fuses it with the first chemistry pass
 *   RT_PATH_ZMARCH  workgroups march x-row tiles through z, evaluating each
 *                   cell's closure and wave speeds once and passing them to
 *                   the faces through LDS and registers; rt_step runs it,
 *                   then the chemistry passes.  Needs nx <= 1024 (FP32
 *                   transport) or nx <= 512 (FP64): RT_EINVAL otherwise. */
enum { RT_PATH_AUTO = 0, RT_PATH_CELL = 1, RT_PATH_ZMARCH = 2 };
rt_status rt_set_transport_path(rt_ctx *ctx, int path);

/* Kernel arrangement of the chemistry that follows a separate transport
 * (rt_thermochem, and rt_step on the z-marching path; App. A); results are
 * the same bits on every path:
 *   RT_CHEM_AUTO      one pass on grids of 2,000,000 cells or more, two
 *                     passes on smaller ones (the faster of the two there)
 *   RT_CHEM_TWO_PASS  a head pass of head_attempts attempts per cell in
 *                     lockstep, then the queued cells in a persistent tail
 *   RT_CHEM_ONE_PASS  one persistent pass whose lanes take the next cell as
 *                     soon as theirs has filled dt_RT, cells whose previous
 *                     pass took many attempts first
 * The per-cell transport path's rt_step always runs its fused head pass and
 * the tail. */
enum { RT_CHEM_AUTO = 0, RT_CHEM_TWO_PASS = 1, RT_CHEM_ONE_PASS = 2 };
rt_status rt_set_chem_path(rt_ctx *ctx, int path);

/* Launch tuning (results do not depend on it): head_attempts = chemistry
 * attempts per cell in the first pass before a cell is queued for the
 * compacted second pass (1..1000000); queue_cap = queue capacity in cells,
 * at most the capacity rt_scratch_bytes() was sized for (cells that do not
 * fit finish in the first pass).  Negative values keep the current one. */
rt_status rt_set_tuning(rt_ctx *ctx, int head_attempts, long long queue_cap);

/* Diagnostics of the current state and accumulated counters; synchronises
 * the stream.  Needs a bound scratch buffer. */
rt_status rt_get_stats(rt_ctx *ctx, rt_stats *out);
rt_status rt_reset_stats(rt_ctx *ctx);

/* Photon accounting on (1) or off (0, the default) for rt_step,
 * rt_transport and rt_thermochem.  While on, every step also sums the
 * transported photons and the boundary outflow per block, runs a
 * fixed-order reduction of the photon totals after its chemistry and
 * histograms the substeps (a few percent of extra work); the sums are
 * reproducible run to run.  The batched form does not account. */
rt_status rt_set_accounting(rt_ctx *ctx, int enabled);

/* Photon-group attributes of a blackbody source at temperature T_bb [K]
 * for M groups bounded by edges_eV[0..M] (edges_eV[M] may be +inf):
 * sigN, sigE [cm^2] of eqs. (csn_multi), (cse_multi) with the Verner et
 * al. fits of App. E.4, ebar [erg] of eq. (egy_multi), and frac[g], the
 * photon-number fraction of group g over [edges_eV[0], edges_eV[M]].
 * Host computation by quadrature; output arrays are host [3][3], [3], [3]. */
rt_status rt_group_attributes(double T_bb, int M, const double *edges_eV, double sigN[3][3],
                              double sigE[3][3], double ebar[3], double frac[3]);

/* The context's HLL table (host copy, nf*nth*2 doubles, layout
 * [f][theta][lambda_min, lambda_max], c = 1 units, uniform nodes
 * f = i/(nf-1), theta = pi k/(nth-1)).  The pointer is owned by ctx. */
rt_status rt_hll_table(const rt_ctx *ctx, const double **table, int *nf, int *nth);

/* Build the same table on the host into caller memory out[nf*nth*2]
 * (nf, nth >= 2).  Needs no device. */
rt_status rt_build_hll_table(int nf, int nth, double *out);

/* Kernel timing with HIP events on the bound stream.  While enabled, every
 * launch of the step is bracketed by events; rt_get_timing synchronises the
 * stream and returns the accumulated milliseconds and launch counts per
 * kernel class, then clears them.  Disabled by default. */
#define RT_TIMING_CLASSES 6
typedef struct {
    double ms[RT_TIMING_CLASSES];  /* inject, transport, chemistry head (fused
                                      with transport on the per-cell path; the
                                      whole one-pass chemistry), chemistry
                                      tail, other (adjoint passes), photon
                                      accounting (reductions, ledger) */
    long long launches[RT_TIMING_CLASSES];
} rt_timing;
rt_status rt_set_timing(rt_ctx *ctx, int enabled);
rt_status rt_get_timing(rt_ctx *ctx, rt_timing *out);

const char *rt_last_error(const rt_ctx *ctx);
void rt_free(rt_ctx *ctx);

/* ---------------------------------------------------------------------
 * Batched form: nbox independent grids ("boxes") of any size, each with its
 * own 1..3 photon groups, advanced together with the same time step.  One
 * step is the same method as rt_step on every box; it runs as one HIP graph
 * (injection, a persistent kernel over 64-cell chunks of all boxes doing
 * transport and the first chemistry attempts, a persistent kernel finishing
 * the cells still subcycling).  Each box's result equals rt_step on that box
 * alone, bit for bit.
 * --------------------------------------------------------------------- */
typedef struct rt_batch rt_batch;

/* grids[nbox], groups[nbox] (all with the same c_r), params common to all
 * boxes.  Validation as rt_init.  1 <= nbox <= 65535. */
rt_status rt_batch_init(int nbox, const rt_grid *grids, const rt_groups *groups, const rt_params *params,
                        rt_batch **out);

/* Device scratch the batch needs (chunk counter and the queue of cells still
 * subcycling, with room for every cell). */
size_t rt_batch_scratch_bytes(const rt_batch *b);

/* states[nbox]: caller-owned arrays of every box as for rt_bind (the scratch
 * fields of states[] are ignored); scratch of rt_batch_scratch_bytes() bytes.
 * Sets the current radiation set of all boxes to 0. */
rt_status rt_batch_bind(rt_batch *b, const rt_state *states, void *scratch, size_t scratch_bytes);

/* Stream for all work; graphs are captured on it, so it must not be the
 * null stream when graphs are enabled (otherwise steps launch eagerly). */
rt_status rt_batch_set_stream(rt_batch *b, void *hip_stream);

int rt_batch_current(const rt_batch *b);
rt_status rt_batch_set_current(rt_batch *b, int set);

/* Sources of one box, as rt_set_sources (ndot[s*M_box + g]). */
rt_status rt_batch_set_sources(rt_batch *b, int box, int n, const int32_t *ijk, const double *ndot);

/* Courant-limited step of the batch (Sec. 4.1, eq. dt_courant): courant x
 * dx_min / (3 c_r), the finest box setting the common step (courant > 0). */
rt_status rt_batch_courant_dt(const rt_batch *b, double courant, double *dt);

/* nsteps steps of every box; dt <= 0 uses 0.8 dx_min/(3 c_r).  dt must
 * satisfy the Courant limit of the finest box. */
rt_status rt_batch_step(rt_batch *b, double dt, int nsteps);

/* Launch tuning (results do not depend on it; negative keeps the value):
 * persistent head blocks per compute unit (1..64), chemistry attempts in the
 * head pass (1..1e6), tail blocks (1..65536), graphs on/off. */
rt_status rt_batch_set_tuning(rt_batch *b, int head_blocks_per_cu, int head_attempts, int tail_blocks,
                              int use_graph);

/* Accumulated chemistry counters and flags of all boxes (the photon fields
 * of rt_stats are zero); synchronises the stream. */
rt_status rt_batch_get_stats(rt_batch *b, rt_stats *out);
rt_status rt_batch_reset_stats(rt_batch *b);

const char *rt_batch_last_error(const rt_batch *b);
void rt_batch_free(rt_batch *b);

/* ---------------------------------------------------------------------
 * Differentiation form: the reverse (adjoint) pass of rt_step, giving
 * dL/dln Ndot_s for every source and dL/dln n_H for every cell of a scalar
 * L of the state after some steps.
 *
 * Supported configuration (RT_EUNSUPPORTED otherwise): one photon group,
 * hydrogen-only gas (Y = 0), GLF flux, periodic boundaries on all faces,
 * no smoothing, OTSA, static box.  Isothermal and temperature-evolving gas
 * are both supported, and both precisions: with RT_PREC_FP32_TRANSPORT the forward
 * steps are the mixed form's (FP32 N and F), the tape holds them widened to
 * FP64 and the adjoint runs in FP64, so the result is the gradient of the
 * mixed form's own forward map.
 *
 * Of step k (U_k -> injection -> U_a -> transport -> U_b -> chemistry ->
 * U_k+1) the adjoint applies the transposes of
 *   - the chemistry (App. A): per cell, its accepted substeps in reverse,
 *     each linearised at the state recorded before it, with the substep
 *     lengths held fixed (they are piecewise constant in the state: the
 *     derivative is that of the branch the forward step took);
 *   - the transport (Sec. 3.2, eqs. dUdt_sol, glf): the 7-point stencil,
 *     linearised at U_a with the M1 flux Jacobian (Sec. 2, eqs. edd2,
 *     eddTens) in closed form;
 *   - the injection (Sec. 3.1, eq. injnum).
 * The caller drives the checkpointing: it restores U_k, calls
 * rt_step_record (which advances the bound state by one step exactly as
 * rt_step does, split into kernels, and writes a tape), then, later and in
 * reverse step order, rt_step_adjoint with that tape.
 * --------------------------------------------------------------------- */

/* Per-step tape, caller-owned device memory.
 *   Na      ncell doubles: N after the step's injection (the transport input;
 *           with RT_PREC_FP32_TRANSPORT the FP32 values, widened)
 *   Fa      3*ncell doubles: F after injection, layout [axis][cell]
 *   counts  ncell int32: accepted chemistry substeps of each cell in this
 *           step, as rt_step writes them to rt_state.nacc (input)
 *   off     rt_tape_offsets_len() int64: trace offsets (written by record)
 *   trace   7*cap doubles: per cell, the state {N, Fx, Fy, Fz, x_HII, T_mu
 *           (T when isothermal), h} before each accepted substep, then the
 *           state after the chemistry
 *   cap     trace entries; must be >= ncell + sum(counts) */
typedef struct {
    double *Na, *Fa;
    const int32_t *counts;
    int64_t *off;
    double *trace;
    long long cap;
} rt_tape;

/* Adjoint state (device, caller-owned), updated in place from lambda_k+1 =
 * dL/dU_k+1 to lambda_k = dL/dU_k:
 *   N (ncell), F (3*ncell, [axis][cell]), xHII (ncell), T (ncell);
 *   wN (ncell) and wF (3*ncell) are work arrays. */
typedef struct {
    double *N, *F, *xHII, *T;
    double *wN, *wF;
} rt_adj;

/* int64 entries of rt_tape.off for this grid: ncell + 1 offsets plus one
 * partial sum per 1024 cells. */
size_t rt_tape_offsets_len(const rt_ctx *ctx);

/* One forward step (as rt_step with nsteps = 1, same result) that writes the
 * tape.  tape->counts must hold this step's substep counts (from a previous
 * rt_step of the same state with rt_state.nacc bound); a mismatch or a too
 * small cap sets RT_FLAG_TRACE in rt_stats.flags.  dt as for rt_transport. */
rt_status rt_step_record(rt_ctx *ctx, double dt, const rt_tape *tape);

/* A forward step whose chemistry replays the substep schedule of a recorded
 * step (per cell: the number of accepted substeps and their lengths from
 * tape, applied to the current state without the 10% checks of App. A).
 * Its result is a smooth function of the inputs and parameters, and its
 * derivative is the one rt_step_adjoint computes: finite differences of
 * replayed runs check the adjoint without the jumps that a changed substep
 * schedule puts into finite differences of rt_step.  Reads tape (counts,
 * off, trace as written by rt_step_record); advances the bound state. */
rt_status rt_step_replay(rt_ctx *ctx, double dt, const rt_tape *tape);

/* Reverse of the recorded step: lam from lambda_k+1 to lambda_k; adds the
 * step's contributions to g_lnNdot[s] (device, one per source in the order
 * given to rt_set_sources) and g_lnnH[cell] (device, ncell).  Reads the
 * bound n_H and the tape; does not touch the bound state.  Sources and dt
 * must be those of the recorded step. */
rt_status rt_step_adjoint(rt_ctx *ctx, double dt, const rt_tape *tape, const rt_adj *lam, double *g_lnNdot,
                          double *g_lnnH);

#ifdef __cplusplus
}
#endif
#endif /* RTM1_H */
