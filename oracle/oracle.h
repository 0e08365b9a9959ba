/*
 * Plain FP64 CPU oracle for Jastrow variational Monte Carlo of liquid 4He
 * (Lutsyshyn, "Fast quantum Monte Carlo on a GPU", arXiv:1312.1282).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  The product path (libhevmc) never includes, links or calls anything here,
 * and this code includes nothing from the product.
 *
 * Everything is scalar FP64 loops in the order the paper states the method,
 * built with -O2 -ffp-contract=off.  Long sums use Neumaier compensation so that
 * the oracle is the more accurate side of every comparison.
 *
 * Units: lengths in Angstrom, energies in Kelvin.
 * Coordinates are structure-of-arrays: xyz[0..n-1] = x, xyz[n..2n-1] = y,
 * xyz[2n..3n-1] = z, each in [0, L).
 */
#ifndef HE_ORACLE_H
#define HE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One simulated system: N atoms in a cubic periodic box of side L. */
typedef struct {
    int32_t n;             /* number of atoms N                                   */
    int32_t order;         /* 0: random particle index per move, 1: s = k           */
    double L;              /* box side (Angstrom)                                  */
    double b;              /* Jastrow parameter b of Eq. (9) (Angstrom)            */
    double hbar2_over_m;   /* hbar^2 / m_He (K Angstrom^2)                         */
    double step_sigma;     /* std. dev. of each Cartesian component of delta (A)   */
    uint64_t seed;         /* Philox key = (low 32 bits, high 32 bits)             */
    int32_t fp32_coords;   /* 1: every stored position (start, accepted move) is
                              rounded to the nearest FP32 number, as the precision
                              form keeps its coordinates; arithmetic stays FP64    */
} or_system;

/* Per-walker running state and accumulators (all sums Neumaier-compensated;
 * the value of a sum is sum + comp). */
typedef struct {
    double u_run, v_run;     /* ln psi and potential energy of current config   */
    double sum_e, c_e;       /* sum of local energies E_L                       */
    double sum_e2, c_e2;     /* sum of E_L^2                                    */
    double sum_v, c_v;       /* sum of potential energies at E_L samples        */
    double sum_tpb, c_tpb;   /* sum of T_PB (local kinetic energy)              */
    double sum_tjf, c_tjf;   /* sum of T_JF                                     */
    double sum_tf, c_tf;     /* sum of T_F                                      */
    double sum_vs, c_vs;     /* sum of v_run over measured sweeps               */
    int64_t n_samples;       /* number of E_L samples                           */
    int64_t n_sweeps_meas;   /* number of measured sweeps                       */
    int64_t n_acc;           /* accepted moves in measured sweeps               */
    int64_t n_try;           /* attempted moves in measured sweeps              */
} or_walker;

/* Box side L = (N / density)^(1/3); rounded to FP32 if fp32 != 0. */
double or_box_side(int32_t n, double density, int32_t fp32);

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Random quantities of micro-step k of sweep t of walker w: particle index s,
 * Metropolis variable xi in (0,1), Gaussian displacement delta (Sec. 2, Sec. 5.1). */
void or_draw_move(const or_system *sys, uint32_t k, uint32_t t, uint32_t w,
                  int32_t *s, double *xi, double delta[3]);

/* Pair functions of Sec. 2: f of Eq. (9), u of Eq. (8) (as read: multiplicative
 * symmetrization, zero beyond L/2), its first two derivatives, and the HFD-B(HE)
 * potential. */
double or_f(const or_system *sys, double r);
double or_u(const or_system *sys, double r);
void or_u_derivs(const or_system *sys, double r, double *u, double *du, double *d2u);
double or_aziz(double r);                          /* untruncated V(r)      */
double or_aziz_deriv(double r);                    /* its dV/dr             */
double or_min_image(double d, double L);

/* Totals U = sum_{i<j} u(r_ij) = ln psi (Eq. 6) and V = sum_{i<j} V(r_ij). */
void or_totals(const or_system *sys, const double *xyz, double *U, double *V);

/* Single-particle trial move r_s -> wrap(r_s + delta): new position
 * (rounded to FP32 if sys->fp32_coords). */
void or_trial_position(const or_system *sys, const double *xyz, int32_t s,
                       const double delta[3], double rnew[3]);

/* Eq. (7): dU = sum_{i != s} [u(|r_s' - r_i|) - u(|r_s - r_i|)] and the same
 * for V.  scale_u / scale_v = sum of |terms| (tolerance scale). */
void or_delta(const or_system *sys, const double *xyz, int32_t s, const double rnew[3],
              double *du, double *dv, double *scale_u, double *scale_v);

/* Tolerance slopes of the same move: slope_u = sum_{i != s} (|u'(r_i')| +
 * |u'(r_i)|), slope_v likewise with dV/dr (zero beyond L/2). */
void or_delta_slopes(const or_system *sys, const double *xyz, int32_t s, const double rnew[3],
                     double *slope_u, double *slope_v);

/* Local energy of a configuration.  out[0..5] = E_L, V, T_PB, T_JF, T_F, U.
 * scale = sum |V_ij| + kappa * sum_i (|Lap_i| + |G_i|^2).  grad (3N, SoA) and
 * lap (N) receive grad_i ln psi and lap_i ln psi if not NULL. */
void or_local_energy(const or_system *sys, const double *xyz, double out[6], double *scale,
                     double *grad, double *lap);

/* fcc start with deterministic Philox jitter for walker id w. */
/* Pair distribution histogram of one configuration (the g(r) the paper's
 * host analysis computes, Sec. 5.4 and Sec. 7): counts[b], b = 0..nb-1, is the
 * number of unordered pairs whose minimum-image distance r lies in
 * [b h/nb, (b+1) h/nb), h = L/2, with r = h itself in the last bin and pairs
 * beyond h not counted.  edge[b] (may be NULL) counts the pairs whose r/(h/nb)
 * lies within rel_window of the integer b (a bin edge; b = nb is the cutoff),
 * where another rounding of r could put the pair in the neighbouring bin. */
void or_pair_histogram(const or_system *sys, const double *xyz, int32_t nb, uint64_t *counts,
                       uint64_t *edge, double rel_window);

void or_fcc_start(const or_system *sys, uint32_t w, double *xyz);

/* Eq. (5): the Metropolis decision for a move whose Eq. (7) sum is du:
 * 1 if |psi'|^2 / |psi|^2 = exp(2 du) > xi (strict), else 0. */
int or_metropolis_accept(double du, double xi);

/* Fresh running state for a configuration: u_run, v_run from or_totals,
 * accumulators zeroed. */
void or_walker_init(const or_system *sys, const double *xyz, or_walker *acc);

/* Run sweeps t = t0 .. t0+n_sweeps-1 of walker w (Sec. 5.1 workflow).
 * Sweeps t >= measure_start are measured: moves counted, v_run accumulated, and
 * after sweep t the local energy is sampled if m > 0 and
 * (t - measure_start + 1) % m == 0.  If el_out is not NULL, each sample's
 * E_L is appended there (el_out[*n_el] ...).  Returns 0. */
int or_run_walker(const or_system *sys, uint32_t w, double *xyz, or_walker *acc,
                  uint32_t t0, int32_t n_sweeps, uint32_t measure_start, int32_t m,
                  double *el_out, int64_t *n_el);

/* or_run_walker that also records every micro-update q = (t - t0) N + k of
 * the call, for q < log_cap: log[8 q .. 8 q + 7] = (s, accepted, dU, dV,
 * scale_u, scale_v, slope_u, slope_v) with the Eq. (7) sums of or_delta and
 * the slopes of or_delta_slopes at the configuration the move was proposed in.  The chain itself is the same as or_run_walker's. */
int or_run_walker_log(const or_system *sys, uint32_t w, double *xyz, or_walker *acc,
                      uint32_t t0, int32_t n_sweeps, uint32_t measure_start, int32_t m,
                      double *log, int64_t log_cap);

/* Same as or_run_walker for walkers w0 .. w0+nw-1 (xyz: nw blocks of 3N,
 * acc: nw entries), spread over n_threads POSIX threads, one walker at a time
 * per thread.  The per-walker computation is identical to or_run_walker. */
int or_run_walkers(const or_system *sys, uint32_t w0, int32_t nw, double *xyz,
                   or_walker *acc, uint32_t t0, int32_t n_sweeps, uint32_t measure_start,
                   int32_t m, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
