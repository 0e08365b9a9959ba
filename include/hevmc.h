/*
 * libhevmc — Metropolis sweeps and local energies of Jastrow variational Monte
 * Carlo for liquid 4He on AMD Instinct MI355X (gfx950).
 *
 * Method: Y. Lutsyshyn, "Fast quantum Monte Carlo on a GPU", arXiv:1312.1282.
 *   - wavefunction psi = exp(sum_{i<j} u(r_ij))                      Sec. 2, Eq. (6)
 *   - u(r) = f(r) + f(L-r) - 2 f(L/2) for r <= L/2, 0 beyond,
 *     f(r) = -(1/2)(b/r)^5   (multiplicative reading of Eq. (8))    Sec. 2, Eqs. (8), (9)
 *   - V(r) = HFD-B(HE) ("Aziz-II"), truncated at L/2               Sec. 2, Sec. 7
 *   - single-particle Gaussian moves, acceptance exp(2 dU) > xi,
 *     dU = sum_{i != s} [u(|r_s'-r_i|) - u(|r_s-r_i|)]              Sec. 2, Eqs. (5), (7)
 *   - local energy E_L = V + T, with T_PB, T_JF, T_F estimators      Sec. 2, Sec. 5.4
 *   - minimum-image periodic cubic box of side L = (N/density)^(1/3) Sec. 5.1, Sec. 7
 *
 * Conventions
 *   - Every function returns an hevmc_status: 0 on success, a negative code on
 *     error (then hevmc_last_error() describes it).  Nothing aborts or exits.
 *   - Units: lengths in Angstrom, energies in Kelvin, density in 1/Angstrom^3.
 *   - "Device" pointers are HIP device memory on the current device (for
 *     example torch CUDA tensors); "host" pointers are ordinary memory.  The
 *     library never keeps a pointer after a call returns, except inside an
 *     hevmc_ensemble created by hevmc_create_on (see there).
 *   - Kernels are launched on the given hipStream_t (passed as void*; NULL is
 *     the null stream) and are asynchronous unless stated otherwise.  Errors a
 *     kernel cannot report are checked by the next synchronising call.
 *   - Coordinates of a walker are structure of arrays: x[0..N-1], y[0..N-1],
 *     z[0..N-1], each in [0, L).  An ensemble of W walkers is [W][3][N].
 *     Element type: double for HEVMC_FP64, float for HEVMC_FP32.
 *   - Random numbers: the moves of micro-step k of sweep t of walker w come from
 *     Philox4x32-10 with counter (k, t, walker_id_base + w, 0|1) and key =
 *     seed, so results depend only on (seed, walker id, sweep index) and not
 *     on how sweeps are split into calls or how walkers are placed.
 *   - Calls that share buffers and overlap on one device race; separate
 *     ensembles on separate buffers may run concurrently on separate streams.
 */
#ifndef HEVMC_H
#define HEVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HEVMC_OK = 0,
    HEVMC_EINVAL = -1,   /* invalid argument                                   */
    HEVMC_ENOMEM = -2,   /* device or host allocation failed                   */
    HEVMC_ENOFIT = -3,   /* walker does not fit in one workgroup's LDS         */
    HEVMC_EDEVICE = -4,  /* HIP runtime error (no device, launch failure, ...) */
    HEVMC_ESTATE = -5,   /* non-finite running state or accumulator detected   */
    HEVMC_EBUSY = -6     /* the ensemble is in use by a call on another thread */
} hevmc_status;

typedef enum {
    HEVMC_FP64 = 0,      /* all arithmetic FP64                                          */
    HEVMC_FP32 = 1       /* FP32 coordinates and pair terms; FP64 sums, decision, energies */
} hevmc_precision;

typedef enum {
    HEVMC_SELECT_RANDOM = 0,     /* s drawn uniformly each micro-step (Sec. 2, Sec. 5.1) */
    HEVMC_SELECT_SEQUENTIAL = 1  /* s = k, the micro-step index                          */
} hevmc_order;

/* How the sweep forms the Eq. (7) sums (same Markov chain either way, up to
 * rounding).  PLAIN evaluates u and V at the old and the new position of the
 * moved atom for every trial move.  ROWS keeps each atom's row sum
 * R_i = sum_{j != i} u(r_ij) (FP64, in LDS; refreshed by every local-energy
 * pass) and evaluates only u at the new position per trial move; the old
 * position's terms, the row updates and dV are formed only for accepted moves.
 * ROWS needs N <= 8 x threads and 8 N more bytes of LDS per walker; in FP32
 * with 512 threads and N <= 22 x 512 it can instead keep the rows in
 * registers (no LDS beyond the coordinates, no refresh at local-energy passes;
 * the rows persist through the rows buffer as in LDS form).  The batched sweep
 * runs such walkers PLAIN. */
typedef enum {
    HEVMC_VARIANT_AUTO = 0,      /* ROWS when it fits, else PLAIN */
    HEVMC_VARIANT_PLAIN = 1,
    HEVMC_VARIANT_ROWS = 2
} hevmc_variant;

/* Parameters of one ensemble of independent walkers (Markov chains). */
typedef struct {
    int32_t n;               /* atoms per walker N, >= 2                                  */
    int32_t n_walkers;       /* walkers W, >= 1                                           */
    int32_t precision;       /* hevmc_precision                                           */
    int32_t order;           /* hevmc_order                                               */
    double density;          /* N / L^3 (1/A^3), > 0                                      */
    double b;                /* Jastrow parameter b of Eq. (9) (A), >= 0                  */
    double hbar2_over_m;     /* hbar^2/m (K A^2), > 0; 12.1194 for 4He                    */
    double step_sigma;       /* std. deviation of each Cartesian move component (A), > 0 */
    uint64_t seed;           /* Philox key: (low 32 bits, high 32 bits)                   */
    uint32_t walker_id_base; /* walker w uses Philox walker id walker_id_base + w         */
    int32_t threads;         /* threads per walker: 0 = library choice, else 64, 128,
                                256, 512 or 1024 (64: one wavefront per walker, four
                                walkers per workgroup)                                     */
    int32_t variant;         /* hevmc_variant                                             */
} hevmc_params;

/* Per-walker running state and accumulators, in device memory ([W] array).
 * Sums are Neumaier-compensated: the value of sum_x is sum_x + c_x.
 * Energies are totals for the walker's N atoms (K), not per atom. */
typedef struct {
    double u_run, v_run;     /* ln psi and V of the current configuration                 */
    double sum_e, c_e;       /* sum of local energies E_L over samples                    */
    double sum_e2, c_e2;     /* sum of E_L^2                                              */
    double sum_v, c_v;       /* sum of V at samples                                       */
    double sum_tpb, c_tpb;   /* sum of T_PB = -kappa sum_i (lap_i ln psi + |grad_i ln psi|^2) */
    double sum_tjf, c_tjf;   /* sum of T_JF = -(kappa/2) sum_i lap_i ln psi               */
    double sum_tf, c_tf;     /* sum of T_F  =  kappa sum_i |grad_i ln psi|^2              */
    double sum_vs, c_vs;     /* sum of v_run at the end of every measured sweep           */
    int64_t n_samples;       /* local-energy samples                                      */
    int64_t n_sweeps_meas;   /* measured sweeps                                           */
    int64_t n_acc;           /* accepted moves in measured sweeps                         */
    int64_t n_try;           /* attempted moves in measured sweeps                        */
} hevmc_walker_acc;

/* How the library will run a sweep of p on the current device (the launch
 * plan; no work is done).  All fields are outputs. */
typedef struct {
    int32_t threads;          /* threads per walker                                       */
    int32_t variant;          /* HEVMC_VARIANT_PLAIN or HEVMC_VARIANT_ROWS                 */
    int32_t spatial_order;    /* 1: atoms are re-sorted by cell (Morton order) in LDS at
                                 every sweep, so a wavefront's atoms are neighbours in
                                 space; results are the same up to summation order       */
    int32_t walkers_per_cu;   /* walkers one compute unit holds at a time                 */
    uint64_t lds_per_walker;  /* LDS bytes of one walker                                  */
    uint64_t lds_per_group;   /* dynamic LDS bytes requested per workgroup                */
    int32_t slices;           /* workgroups per walker: 1, or C > 1 for a spread walker   */
    int32_t reserved;         /* 0                                                        */
} hevmc_plan;

/* Spread walkers.  A walker whose coordinates do not fit in one workgroup's
 * LDS (FP64 beyond about 6800 atoms, FP32 beyond about 13600) is spread over
 * C workgroups of a cooperative launch, workgroup g holding atoms
 * [g S, g S + S): the cooperative kernel that Sec. 3 describes, over several
 * compute units (C <= 14).  Each micro-update's Eq. (7) sums are formed by
 * the C workgroups over their own atoms, published to a mailbox in device
 * memory and added in a fixed order by every workgroup once all C are there,
 * so all take the same Eq. (5) decision; the workgroup holding the next move's
 * atom publishes its position the same way.  Such walkers use the plain form
 * (no rows; a rows argument is ignored) with 512 threads per workgroup (256
 * or 1024 if hevmc_params.threads asks for it); their local
 * energies run in separate kernels that stream the coordinates through LDS,
 * several workgroups per walker.  hevmc_init_walkers, hevmc_sweep, hevmc_sweep_log,
 * hevmc_sweep_gr, hevmc_sweep_trace (histogram and records formed by those
 * local-energy kernels), hevmc_local_energy, hevmc_footprint,
 * hevmc_plan_launch and the ensemble layer accept them; the other entry
 * points return HEVMC_ENOFIT.  For spread
 * walkers hevmc_sweep and hevmc_sweep_log are synchronous: every wait of a
 * workgroup for the others is bounded, and a wait that gives up (a workgroup
 * stopped arriving) ends the call with HEVMC_EDEVICE and the walkers' state
 * not valid.  The library keeps a small device workspace per device for the
 * mailboxes and the local energy's partial sums (grow-only, held until the
 * process ends); calls that overlap on one device race.  */

/* Fills *out with the launch plan of hevmc_sweep for p.  HEVMC_ENOFIT as
 * hevmc_footprint. */
hevmc_status hevmc_plan_launch(const hevmc_params *p, hevmc_plan *out);

/* Box side L = cbrt(n / density) (A), as every kernel uses it. */
hevmc_status hevmc_box(const hevmc_params *p, double *L_out);

/* LDS bytes one walker needs (over all its workgroups) and device bytes an
 * ensemble's state takes (coordinates + accumulators + rows).  HEVMC_ENOFIT if
 * the walker fits neither one workgroup's LDS nor the chip's as a spread
 * walker. */
hevmc_status hevmc_footprint(const hevmc_params *p, size_t *lds_bytes_per_walker,
                             size_t *hbm_bytes);

/* Start walkers.  If fcc_start != 0, first writes the fcc start with a
 * deterministic jitter of 1e-3 lattice constants (device coords [W][3][N]);
 * otherwise coords must already hold valid positions.  Then sets u_run, v_run
 * of every walker from a full O(N^2) evaluation, zeroes all accumulators and,
 * if rows is not NULL, fills rows ([W][N] doubles, device) with each atom's
 * row sum sum_{j != i} u(r_ij) for later hevmc_sweep calls.  A walker with a
 * non-finite coordinate gets u_run = v_run = NaN.
 * coords, acc: device.  Asynchronous on stream. */
hevmc_status hevmc_init_walkers(const hevmc_params *p, void *coords, hevmc_walker_acc *acc,
                                double *rows, int32_t fcc_start, void *stream);

/* The hot path: sweeps t = sweep0 .. sweep0+n_sweeps-1 of all W walkers
 * (Sec. 5.1 workflow; one sweep = N micro-updates, a "macroupdate" of Sec. 4.1).
 * Each micro-update draws (s, xi, delta), forms dU and dV by the O(N) pair loop
 * of Eq. (7), accepts if exp(2 dU) > xi (Eq. (5)), and on acceptance moves atom s
 * and adds dU, dV to u_run, v_run.  Sweeps t >= measure_start are measured:
 * moves are counted, v_run is added to sum_vs after the sweep, and if
 * energy_every = m > 0 and (t - measure_start + 1) % m == 0 the local energy of
 * the configuration is evaluated, added to the accumulators, and u_run, v_run
 * are reset to its fresh totals.  Pass measure_start = 0xFFFFFFFF for
 * equilibration only.  coords, acc: device, updated in place.  rows: NULL or
 * a device [W][N] double buffer that keeps the row sums of the ROWS variant
 * between calls (filled by hevmc_init_walkers or a previous hevmc_sweep on the
 * same walkers); the kernel checks sum_i R_i = 2 u_run and recomputes the rows
 * when the buffer is NULL or disagrees, an O(N^2) pass per walker.  Ignored by
 * the PLAIN variant.  A walker with a non-finite coordinate ends the call with
 * u_run = v_run = NaN (its pairs would otherwise drop out of every sum
 * unnoticed).  Requires sweep0 + n_sweeps <= 0xFFFFFFFF.  Asynchronous on
 * stream. */
hevmc_status hevmc_sweep(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                         uint32_t sweep0, int32_t n_sweeps, uint32_t measure_start,
                         int32_t energy_every, void *stream);

/* ---- Pair distribution function g(r) ---------------------------------------- */

#define HEVMC_MAX_GR_BINS 4096

/* hevmc_sweep that also accumulates the pair distribution histogram, the
 * g(r) of the paper's analysis of sampled configurations (Sec. 5.4, Sec. 7).
 * At every local-energy sample, each unordered pair with minimum-image
 * distance r <= L/2 adds 1 to gr[w][min(gr_bins - 1, floor(r gr_bins / (L/2)))]
 * (gr: device [W][gr_bins] uint64, caller-owned, added to, never cleared).
 * Normalisation: g(r_b) = counts_b / (samples * N/2 * (N/L^3) * shell volume of
 * bin b).  gr = NULL is hevmc_sweep.  The sweep's results are bitwise the same
 * with or without the histogram.  HEVMC_EINVAL for gr_bins outside
 * [1, HEVMC_MAX_GR_BINS]; HEVMC_ENOFIT if the walker fits one workgroup's LDS
 * but not with the bins beside it (a walker that fits no workgroup at all is
 * spread, see below, and its local-energy kernels form the histogram). */
hevmc_status hevmc_sweep_gr(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                            uint64_t *gr, int32_t gr_bins, uint32_t sweep0, int32_t n_sweeps,
                            uint32_t measure_start, int32_t energy_every, void *stream);

/* The pair distribution histogram of each of the W configurations in coords
 * (device [W][3][N] of the precision's type), binned as in hevmc_sweep_gr:
 * counts (device [W][n_bins] uint64) is overwritten.  Asynchronous. */
hevmc_status hevmc_pair_histogram(const hevmc_params *p, const void *coords, int32_t n_bins,
                                  uint64_t *counts, void *stream);

/* ---- Per-sample records (correlated sampling over b) ---------------------- */

/* hevmc_sweep that also writes, at every local-energy sample, the record
 * (E_L, V, T_PB, T_JF, T_F, U) of the sampled configuration (the quantities of
 * hevmc_local_energy) to trace[w][s][0..5], s the sample's index among all of
 * walker w's samples (its n_samples before the sample), for s < trace_cap;
 * later samples are counted in the accumulators but not recorded.
 * trace: device [W][trace_cap][6] doubles, caller-owned.
 * Because f of Eq. (9) scales as b^5, u for another b' is (b'/b)^5 u, and so
 * are ln psi, its gradient and its Laplacian: each record gives E_L and the
 * reweighting factor exp(2 (U_b' - U_b)) at any b' (Sec. 2 variational
 * optimisation), see the host helper observables.reweight_b.  The sweep's
 * results are bitwise the same with or without the trace.  HEVMC_EINVAL for
 * trace_cap < 1. */
hevmc_status hevmc_sweep_trace(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                               double *trace, int32_t trace_cap, uint32_t sweep0, int32_t n_sweeps,
                               uint32_t measure_start, int32_t energy_every, void *stream);

/* ---- Per-move records (parity of the micro-updates) ----------------------- */

/* hevmc_sweep that also records every micro-update of walkers
 * w = 0 .. log_walkers-1 (the micro-update of Eqs. (5) and (7), Sec. 2):
 * log[w][q][0..3] = (s, accepted, dU, dV) for the q-th micro-update of the
 * call, q = (t - sweep0) N + k, for q < log_cap (later ones are not recorded).
 * s is the moved atom's label (its index in the coordinate arrays), accepted
 * is 1.0 or 0.0, dU is the Eq. (7) sum the decision used (for the row-sum
 * forms: sum_i u(|r_s' - r_i|) minus the moved atom's row sum), and dV the
 * potential change: for every micro-update in the PLAIN form, for accepted
 * ones only in the row-sum forms (NaN for rejected ones, whose dV those forms
 * never form).  log: device [log_walkers][log_cap][4] doubles, caller-owned,
 * written only where recorded.  The sweep's results are bitwise the same with
 * or without the records.  HEVMC_EINVAL for log = NULL, log_walkers outside
 * [1, n_walkers] or log_cap < 1. */
hevmc_status hevmc_sweep_log(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                             double *log, int32_t log_walkers, int64_t log_cap, uint32_t sweep0,
                             int32_t n_sweeps, uint32_t measure_start, int32_t energy_every, void *stream);

/* ---- Batched sweeps (serving: walkers of several requests in one launch) ---- */

#define HEVMC_MAX_BATCH 16

/* One request of a batched sweep: its parameters (n_walkers = its walkers)
 * and where its sweep counters stand for this launch. */
typedef struct {
    hevmc_params params;
    uint32_t sweep0;         /* index of the request's first sweep in this launch */
    uint32_t measure_start;  /* as in hevmc_sweep                                  */
    int32_t energy_every;    /* as in hevmc_sweep                                  */
    int32_t reserved;        /* 0                                                  */
} hevmc_request;

/* hevmc_sweep for walker slots of up to HEVMC_MAX_BATCH requests that share
 * N, precision, threads and variant (their density, b, step, seed and sweep
 * counters may differ), n_sweeps sweeps each, in one launch.  Slot w of the
 * device buffers coords [n_slots][3][N], acc [n_slots], rows [n_slots][N]
 * (rows may be NULL) belongs to request map[2w] (an index into requests, or
 * -1 for an unused slot, which the launch leaves untouched) and draws its
 * random numbers as Philox walker id map[2w+1].  map: device int32
 * [n_slots][2].  requests: host array, copied into the launch's arguments.  A
 * request's result does not depend on which slots it occupies or which other
 * requests share the launch.  Asynchronous on stream. */
hevmc_status hevmc_sweep_batch(int32_t n_requests, const hevmc_request *requests, const int32_t *map,
                               int32_t n_slots, void *coords, hevmc_walker_acc *acc, double *rows,
                               int32_t n_sweeps, void *stream);

/* Local energy of each walker's configuration (Sec. 2 local value of H).
 * coords: device [W][3][N]; out: device [W][6] doubles =
 * (E_L, V, T_PB, T_JF, T_F, U) with U = ln psi.  Asynchronous on stream. */
hevmc_status hevmc_local_energy(const hevmc_params *p, const void *coords, double *out,
                                void *stream);

/* Eq. (7) sums of one trial move per walker, without applying it: atom s[w]
 * moved to wrap(r_s + delta[w]).  coords: device [W][3][N]; s: device [W]
 * int32 in [0, N); delta: device [W][3] doubles; out: device [W][2] doubles =
 * (dU, dV).  Asynchronous on stream. */
hevmc_status hevmc_move_delta(const hevmc_params *p, const void *coords, const int32_t *s,
                              const double *delta, double *out, void *stream);

/* The random quantities of the N micro-steps of sweep t for every walker, as
 * the sweep kernel draws them: s_out [W][N] int32, xi_out [W][N] doubles,
 * delta_out [W][N][3] doubles (device).  Asynchronous on stream. */
hevmc_status hevmc_draw_moves(const hevmc_params *p, uint32_t sweep, int32_t *s_out,
                              double *xi_out, double *delta_out, void *stream);

/* ---- Ensemble convenience layer (state kept on the device between calls) ---- */

typedef struct hevmc_ensemble hevmc_ensemble;

/* Create an ensemble that owns its device state (hipMalloc).  init_xyz: host
 * [W][3][N] doubles, or NULL for the fcc start.  stream: the stream all its
 * work runs on.  Blocks until initialised. */
hevmc_status hevmc_create(const hevmc_params *p, const double *init_xyz, void *stream,
                          hevmc_ensemble **out);

/* Create an ensemble on caller-owned device buffers (coords [W][3][N] of the
 * precision's type, already holding valid positions; acc [W]).  The buffers
 * must outlive the ensemble.  Initialises acc from coords; asynchronous.  When
 * the plan uses row sums the ensemble allocates its own row buffer (8 N W
 * bytes), which hevmc_destroy frees. */
hevmc_status hevmc_create_on(const hevmc_params *p, void *dev_coords, hevmc_walker_acc *dev_acc,
                             void *stream, hevmc_ensemble **out);

/* The calls on an ensemble below (run, sync, get_*, destroy) hold it while
 * they run: a call on the same ensemble from another thread meanwhile returns
 * HEVMC_EBUSY and does nothing. */

/* Run n_sweeps more sweeps.  measure != 0 starts (or continues) measuring:
 * the first measured sweep fixes measure_start.  Asynchronous. */
hevmc_status hevmc_run(hevmc_ensemble *e, int32_t n_sweeps, int32_t energy_every, int32_t measure);

/* Wait for the ensemble's stream; checks the running state for NaN/Inf. */
hevmc_status hevmc_sync(hevmc_ensemble *e);

/* Copy accumulators ([W], host) or coordinates ([W][3][N] doubles, host) out;
 * both synchronise first. */
hevmc_status hevmc_get_acc(hevmc_ensemble *e, hevmc_walker_acc *host_out);
hevmc_status hevmc_get_coords(hevmc_ensemble *e, double *host_out);

/* Sweep counter of the ensemble (next sweep index). */
hevmc_status hevmc_get_sweep(hevmc_ensemble *e, uint32_t *sweep_out);

hevmc_status hevmc_destroy(hevmc_ensemble *e);

/* Parity entry on host buffers (synchronous): for one configuration xyz
 * (host [3][N] doubles; rounded to float for HEVMC_FP32) returns the Eq. (7)
 * sums for moving atom s by delta, and out_el[6] = (E_L, V, T_PB, T_JF, T_F, U).
 * Uses p->n, precision, density, b, hbar2_over_m; ignores n_walkers. */
hevmc_status hevmc_eval_config(const hevmc_params *p, const double *xyz, int32_t s,
                               const double delta[3], double *d_u, double *d_v,
                               double out_el[6]);

/* ---- Entry point that allocates nothing ------------------------------------ */

#define HEVMC_NOALLOC_MAX_N 8192

/* hevmc_eval_config for callers that cannot allocate device memory (code that
 * runs under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results, bit for bit, as
 * hevmc_eval_config; the staging buffers (configuration, s, delta, results)
 * are a fixed device array of the library (196.7 KB per device, held until
 * the process ends) instead of hipMalloc'ed memory, and the call makes no
 * hipMalloc, hipFree or other allocating call on the device.  Synchronous, on
 * the null stream.  Requires p->n <= HEVMC_NOALLOC_MAX_N (HEVMC_EINVAL
 * otherwise), and the other limits of hevmc_eval_config.  All calls on one
 * device share that array: calls that overlap on one device (from several
 * host threads) race. */
hevmc_status hevmc_eval_config_noalloc(const hevmc_params *p, const double *xyz, int32_t s,
                                       const double delta[3], double *d_u, double *d_v,
                                       double out_el[6]);

/* Description of the last error on the calling thread (never NULL). */
const char *hevmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
