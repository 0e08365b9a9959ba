/*
 * Driver that calls every entry point of the CPU oracle at small sizes, for a
 * build under the host sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer,
 * or ThreadSanitizer for the threaded walker runner).  It checks that the
 * results are finite and that the threaded runner gives the bits of the
 * single-walker one; a sanitizer report ends the program with a non-zero status.
 *
 *   oracle_sanitize_driver N FP32 ORDER THREADS
 * Prints "ok <samples> <accepted>" on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int finite_all(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i]))
            return 0;
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 5)
        return 2;
    const int32_t n = atoi(argv[1]);
    const int32_t fp32 = atoi(argv[2]);
    const int32_t order = atoi(argv[3]);
    const int32_t threads = atoi(argv[4]);
    or_system sys;
    memset(&sys, 0, sizeof sys);
    sys.n = n;
    sys.order = order;
    sys.L = or_box_side(n, 0.021836, fp32);
    sys.b = 3.07;
    sys.hbar2_over_m = 12.1194;
    sys.step_sigma = 0.35;
    sys.seed = 0x1234abcd5678ull;
    sys.fp32_coords = fp32;

    /* pair functions over the whole range, including r = L/2 and beyond */
    for (int q = 1; q <= 400; ++q) {
        const double r = sys.L * q / 400.0;
        double u, du, d2u;
        or_u_derivs(&sys, r, &u, &du, &d2u);
        const double v[7] = {or_f(&sys, r), or_u(&sys, r), u, du, d2u, or_aziz(r), or_aziz_deriv(r)};
        if (!finite_all(v, 7) || !isfinite(or_min_image(r - 0.7 * sys.L, sys.L)))
            return 3;
    }

    const int32_t nw = 3;
    double *xyz = (double *)malloc(sizeof(double) * 3 * (size_t)n * nw);
    double *xyz2 = (double *)malloc(sizeof(double) * 3 * (size_t)n * nw);
    or_walker *acc = (or_walker *)calloc((size_t)nw, sizeof(or_walker));
    or_walker *acc2 = (or_walker *)calloc((size_t)nw, sizeof(or_walker));
    if (!xyz || !xyz2 || !acc || !acc2)
        return 4;
    for (int32_t w = 0; w < nw; ++w) {
        or_fcc_start(&sys, (uint32_t)w, xyz + (size_t)w * 3 * n);
        or_walker_init(&sys, xyz + (size_t)w * 3 * n, &acc[w]);
    }
    memcpy(xyz2, xyz, sizeof(double) * 3 * (size_t)n * nw);
    memcpy(acc2, acc, sizeof(or_walker) * (size_t)nw);

    /* one random move taken apart */
    int32_t s;
    double xi, delta[3], rnew[3], du, dv, su, sv, slu, slv;
    or_draw_move(&sys, 5, 2, 1, &s, &xi, delta);
    if (s < 0 || s >= n || !(xi > 0.0 && xi < 1.0))
        return 5;
    or_trial_position(&sys, xyz, s, delta, rnew);
    or_delta(&sys, xyz, s, rnew, &du, &dv, &su, &sv);
    or_delta_slopes(&sys, xyz, s, rnew, &slu, &slv);
    (void)or_metropolis_accept(du, xi);
    const double mv[11] = {rnew[0], rnew[1], rnew[2], du, dv, su, sv, slu, slv, xi, delta[0]};
    if (!finite_all(mv, 11))
        return 6;

    /* chains: three sweeps of equilibration, four measured with E_L every sweep */
    const int32_t sweeps = 7, m = 1;
    const uint32_t t0 = 0, meas = 3;
    double el[16];
    int64_t n_el = 0;
    for (int32_t w = 0; w < nw; ++w)
        or_run_walker(&sys, (uint32_t)w, xyz + (size_t)w * 3 * n, &acc[w], t0, sweeps, meas, m, el, &n_el);
    if (n_el != 4 * nw || !finite_all(el, (size_t)n_el))
        return 7;
    or_run_walkers(&sys, 0, nw, xyz2, acc2, t0, sweeps, meas, m, threads);
    if (memcmp(xyz, xyz2, sizeof(double) * 3 * (size_t)n * nw) != 0 ||
        memcmp(acc, acc2, sizeof(or_walker) * (size_t)nw) != 0)
        return 8;

    /* the logging runner continues the first walker */
    const int64_t log_cap = 2 * (int64_t)n + 5;
    double *log = (double *)calloc((size_t)(8 * log_cap), sizeof(double));
    if (!log)
        return 4;
    or_run_walker_log(&sys, 0, xyz, &acc[0], t0 + sweeps, 3, meas, m, log, log_cap);
    if (!finite_all(log, (size_t)(8 * log_cap)))
        return 9;

    /* local energy with gradient and Laplacian, and the pair histogram */
    double out[6], scale;
    double *grad = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *lap = (double *)malloc(sizeof(double) * (size_t)n);
    const int32_t nb = 37;
    uint64_t counts[37], edge[38];
    if (!grad || !lap)
        return 4;
    or_local_energy(&sys, xyz, out, &scale, grad, lap);
    or_local_energy(&sys, xyz, out, &scale, NULL, NULL);
    if (!finite_all(out, 6) || !isfinite(scale) || !finite_all(grad, 3 * (size_t)n) || !finite_all(lap, (size_t)n))
        return 10;
    or_pair_histogram(&sys, xyz, nb, counts, edge, 1e-9);
    or_pair_histogram(&sys, xyz, nb, counts, NULL, 0.0);
    uint64_t pairs = 0;
    for (int32_t b = 0; b < nb; ++b)
        pairs += counts[b];
    if (pairs == 0 || pairs > (uint64_t)n * (uint64_t)(n - 1) / 2)
        return 11;

    int64_t n_acc = 0;
    for (int32_t w = 0; w < nw; ++w)
        n_acc += acc[w].n_acc;
    printf("ok %lld %lld\n", (long long)n_el, (long long)n_acc);
    free(xyz);
    free(xyz2);
    free(acc);
    free(acc2);
    free(log);
    free(grad);
    free(lap);
    return 0;
}
