/*
 * Plain FP64 CPU oracle: TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper: Y. Lutsyshyn, "Fast quantum Monte Carlo on a GPU", arXiv:1312.1282.
 * Each function cites the passage it follows.  Readings of garbled or silent
 * passages are marked "Reading:".
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Sec. 7: cubic box at density rho, L = (N / rho)^(1/3).  With fp32 != 0 the
 * side is rounded to single precision: the FP32 form of the GPU library works
 * in the box whose side is representable in FP32. */
double or_box_side(int32_t n, double density, int32_t fp32)
{
    double L = cbrt((double)n / density);
    return fp32 ? (double)(float)L : L;
}

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated summation: the value of the sum is *s + *c.          */
static void nsum(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon et al., SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of two 32x32->64
 * multiplications with multipliers 0xD2511F53 and 0xCD9E8D57, the high halves
 * xor-ed with the other counter words and the round key; the key is bumped by
 * the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0,1) from a 32-bit word: (w + 1/2) 2^-32 */
static double unit32(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Sec. 2 (trial configuration: random index s, Gaussian displacement delta),
 * Eq. (5) (uniform xi), Sec. 5.1 (Box-Muller transform of raw uniforms;
 * s, xi and the three components of delta: five numbers per micro-update).
 * Reading: the raw uniforms come from Philox with counter (k, t, w, tag) and
 * key = seed, two calls per move (tag 0 and 1) instead of a pre-generated
 * stream, so a move's numbers depend only on (walker, sweep, micro-step).
 *   s     = floor(a0 * N / 2^32)             (or s = k in sequential order)
 *   xi    = (m + 1/2) 2^-52, m = top 52 bits of (a1, a2)   -> xi in (0,1)
 *   delta = sigma * (R cos(2 pi u2), R sin(2 pi u2), R' cos(2 pi u4)),
 *           R = sqrt(-2 ln u1), R' = sqrt(-2 ln u3),
 *           u1 = a3, u2 = b0, u3 = b1, u4 = b2 mapped to (0,1). */
void or_draw_move(const or_system *sys, uint32_t k, uint32_t t, uint32_t w,
                  int32_t *s, double *xi, double delta[3])
{
    const uint32_t key[2] = {(uint32_t)sys->seed, (uint32_t)(sys->seed >> 32)};
    uint32_t ca[4] = {k, t, w, 0u}, cb[4] = {k, t, w, 1u};
    uint32_t a[4], bw[4];
    or_philox4x32_10(ca, key, a);
    or_philox4x32_10(cb, key, bw);

    if (sys->order == 1)
        *s = (int32_t)(k % (uint32_t)sys->n);
    else
        *s = (int32_t)(((uint64_t)a[0] * (uint64_t)(uint32_t)sys->n) >> 32);

    uint64_t m52 = ((uint64_t)a[1] << 20) | (uint64_t)(a[2] >> 12);
    *xi = ((double)m52 + 0.5) * 0x1p-52;

    const double two_pi = 6.283185307179586;
    double u1 = unit32(a[3]), u2 = unit32(bw[0]);
    double u3 = unit32(bw[1]), u4 = unit32(bw[2]);
    double R1 = sqrt(-2.0 * log(u1));
    double R2 = sqrt(-2.0 * log(u3));
    delta[0] = sys->step_sigma * (R1 * cos(two_pi * u2));
    delta[1] = sys->step_sigma * (R1 * sin(two_pi * u2));
    delta[2] = sys->step_sigma * (R2 * cos(two_pi * u4));
}

/* ------------------------------------------------------------------------ */
/* Eq. (9): Schiff-Verlet / McMillan pair correlation f(r) = -(1/2)(b/r)^5. */
double or_f(const or_system *sys, double r)
{
    double q = sys->b / r;
    return -0.5 * (q * q * q * q * q);
}

/* Eq. (8), Reading: the printed ratio form is garbled (taken literally it
 * diverges to +infinity at short range, contradicting the statement after
 * Eq. (9) that f prevents core overlap, and its value of one beyond L/2 is
 * that of a pair factor, not of its logarithm).  Read as the symmetrization of the pair
 * factor exp(f):  exp(u(r)) = exp(f(r)) exp(f(L-r)) / exp(f(L/2))^2, i.e.
 *   u(r) = f(r) + f(L - r) - 2 f(L/2)   for r <= L/2,   0 beyond,
 * which gives u(L/2) = u'(L/2) = 0: the continuous first derivative and absent
 * kinetic tail that the text after Eq. (8) describes. */
double or_u(const or_system *sys, double r)
{
    const double h = 0.5 * sys->L;
    if (r > h)
        return 0.0;
    return or_f(sys, r) + or_f(sys, sys->L - r) - 2.0 * or_f(sys, h);
}

/* u and its first two radial derivatives (same reading of Eq. (8)):
 *   f'(r) = (5/2) b^5 r^-6,  f''(r) = -15 b^5 r^-7,
 *   u' = f'(r) - f'(L-r),    u'' = f''(r) + f''(L-r). */
void or_u_derivs(const or_system *sys, double r, double *u, double *du, double *d2u)
{
    const double h = 0.5 * sys->L;
    if (r > h) {
        *u = 0.0; *du = 0.0; *d2u = 0.0;
        return;
    }
    const double b5 = sys->b * sys->b * sys->b * sys->b * sys->b;
    const double rp = sys->L - r;
    *u = or_u(sys, r);
    *du = 2.5 * b5 * (1.0 / pow(r, 6) - 1.0 / pow(rp, 6));
    *d2u = -15.0 * b5 * (1.0 / pow(r, 7) + 1.0 / pow(rp, 7));
}

/* Sec. 2: the pair interaction is HFD-B(HE) ("Aziz-II"), cited there to
 * Aziz, McCourt and Wong, Mol. Phys. 61, 1487 (1987).  The paper does not print
 * the constants; these are that publication's:
 *   V(r) = eps [ A exp(-alpha x + beta x^2) - F(x) (C6/x^6 + C8/x^8 + C10/x^10) ],
 *   x = r / r_m,  F(x) = exp(-(D/x - 1)^2) for x < D, else 1. */
#define AZ_EPS   10.948
#define AZ_RM    2.963
#define AZ_A     184431.01
#define AZ_ALPHA 10.43329537
#define AZ_BETA  (-2.27965105)
#define AZ_C6    1.36745214
#define AZ_C8    0.42123807
#define AZ_C10   0.17473318
#define AZ_D     1.4826

double or_aziz(double r)
{
    double x = r / AZ_RM;
    double F = 1.0;
    if (x < AZ_D) {
        double q = AZ_D / x - 1.0;
        F = exp(-(q * q));
    }
    double x2 = x * x, x6 = x2 * x2 * x2, x8 = x6 * x2, x10 = x8 * x2;
    double rep = AZ_A * exp(-AZ_ALPHA * x + AZ_BETA * x2);
    double disp = AZ_C6 / x6 + AZ_C8 / x8 + AZ_C10 / x10;
    return AZ_EPS * (rep - F * disp);
}

/* dV/dr of the untruncated HFD-B(HE) potential (derivative of or_aziz term
 * by term, x = r / r_m):
 *   dV/dr = (eps / r_m) [ A e^{-alpha x + beta x^2} (2 beta x - alpha)
 *                         - F'(x) P(x) - F(x) P'(x) ],
 *   P = C6 x^-6 + C8 x^-8 + C10 x^-10,  P' = -6 C6 x^-7 - 8 C8 x^-9 - 10 C10 x^-11,
 *   F' = 2 (D/x - 1) (D/x^2) F for x < D, else 0.
 * Used only as a tolerance scale (how far V moves when a pair distance carries
 * a small absolute error). */
double or_aziz_deriv(double r)
{
    double x = r / AZ_RM;
    double F = 1.0, dF = 0.0;
    if (x < AZ_D) {
        double q = AZ_D / x - 1.0;
        F = exp(-(q * q));
        dF = 2.0 * q * (AZ_D / (x * x)) * F;
    }
    double x2 = x * x, x6 = x2 * x2 * x2, x7 = x6 * x, x8 = x6 * x2, x9 = x8 * x, x10 = x8 * x2;
    double x11 = x10 * x;
    double rep = AZ_A * exp(-AZ_ALPHA * x + AZ_BETA * x2);
    double P = AZ_C6 / x6 + AZ_C8 / x8 + AZ_C10 / x10;
    double dP = -6.0 * AZ_C6 / x7 - 8.0 * AZ_C8 / x9 - 10.0 * AZ_C10 / x11;
    return AZ_EPS / AZ_RM * (rep * (2.0 * AZ_BETA * x - AZ_ALPHA) - dF * P - F * dP);
}

/* Sec. 5.1: periodic boundary conditions on all interparticle distances.
 * Reading: the minimum image, d - L * nearest_integer(d / L), ties to even. */
double or_min_image(double d, double L)
{
    return d - L * nearbyint(d / L);
}

/* Sec. 7: the potential and the correlation factor are both cut at half the
 * box.  Reading: V is truncated (not shifted) beyond L/2, cutoff inclusive. */
static double pair_v(const or_system *sys, double r)
{
    return (r <= 0.5 * sys->L) ? or_aziz(r) : 0.0;
}

static double pair_dist(const or_system *sys, const double *xyz, int i, int j, double d[3])
{
    const int n = sys->n;
    for (int a = 0; a < 3; ++a)
        d[a] = or_min_image(xyz[a * n + i] - xyz[a * n + j], sys->L);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

static double point_dist(const or_system *sys, const double p[3], const double *xyz, int i)
{
    const int n = sys->n;
    double d[3];
    for (int a = 0; a < 3; ++a)
        d[a] = or_min_image(p[a] - xyz[a * n + i], sys->L);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Eq. (6): ln psi = U = sum_{i<j} u(r_ij); Hamiltonian of Sec. 2: potential
 * V = sum_{i<j} V(r_ij). */
void or_totals(const or_system *sys, const double *xyz, double *U, double *V)
{
    double su = 0, cu = 0, sv = 0, cv = 0;
    double d[3];
    for (int i = 0; i < sys->n; ++i)
        for (int j = i + 1; j < sys->n; ++j) {
            double r = pair_dist(sys, xyz, i, j, d);
            nsum(&su, &cu, or_u(sys, r));
            nsum(&sv, &cv, pair_v(sys, r));
        }
    *U = su + cu;
    *V = sv + cv;
}

/* How a position in [0, L) is kept.  FP64: as it is.  Reading (precision
 * form, FP32 coordinates with FP64 arithmetic on them): rounded to the nearest
 * FP32 number; the side L is then itself an FP32 number (or_box_side with
 * fp32), and a value that rounds up to L is the same point as 0, kept as 0. */
static double stored_coord(const or_system *sys, double x)
{
    if (!sys->fp32_coords)
        return x;
    const double f = (double)(float)x;
    return f >= sys->L ? 0.0 : f;
}

/* Sec. 2: X' = X with r_s -> r_s + delta; the moved atom is put back into the
 * primary box [0, L) (periodic boundary conditions, Sec. 5.1):
 * x' = y - L floor(y / L) with y = x + delta, and x' = x' - L if rounding left
 * it at L. */
void or_trial_position(const or_system *sys, const double *xyz, int32_t s,
                       const double delta[3], double rnew[3])
{
    const double L = sys->L;
    for (int a = 0; a < 3; ++a) {
        double y = xyz[a * sys->n + s] + delta[a];
        double x = y - L * floor(y / L);
        if (x >= L)
            x -= L;
        rnew[a] = stored_coord(sys, x);
    }
}

/* Eq. (7): the log of the acceptance ratio of a single-particle move is
 * 2 * sum_{i != s} [u(|r_s + delta - r_i|) - u(|r_s - r_i|)]; this returns
 * dU = that sum (without the factor 2) and the matching change of the
 * potential energy dV. */
void or_delta(const or_system *sys, const double *xyz, int32_t s, const double rnew[3],
              double *du, double *dv, double *scale_u, double *scale_v)
{
    const int n = sys->n;
    double rold[3] = {xyz[s], xyz[n + s], xyz[2 * n + s]};
    double su = 0, cu = 0, sv = 0, cv = 0, au = 0, av = 0;
    for (int i = 0; i < n; ++i) {
        if (i == s)
            continue;
        double r1 = point_dist(sys, rnew, xyz, i);
        double r0 = point_dist(sys, rold, xyz, i);
        double u1 = or_u(sys, r1), u0 = or_u(sys, r0);
        double v1 = pair_v(sys, r1), v0 = pair_v(sys, r0);
        nsum(&su, &cu, u1 - u0);
        nsum(&sv, &cv, v1 - v0);
        au += fabs(u1) + fabs(u0);
        av += fabs(v1) + fabs(v0);
    }
    *du = su + cu;
    *dv = sv + cv;
    if (scale_u) *scale_u = au;
    if (scale_v) *scale_v = av;
}

/* Slopes of the Eq. (7) terms: slope_u = sum_{i != s} (|u'(r_i')| + |u'(r_i)|),
 * slope_v the same with dV/dr (zero beyond L/2), r_i' and r_i the distances of
 * atom i from the trial and the old position.  A tolerance scale: the change
 * of dU and dV when every pair distance moves by at most one unit (to first
 * order). */
void or_delta_slopes(const or_system *sys, const double *xyz, int32_t s, const double rnew[3],
                     double *slope_u, double *slope_v)
{
    const int n = sys->n;
    const double h = 0.5 * sys->L;
    double rold[3] = {xyz[s], xyz[n + s], xyz[2 * n + s]};
    double au = 0, av = 0;
    for (int i = 0; i < n; ++i) {
        if (i == s)
            continue;
        double r[2] = {point_dist(sys, rnew, xyz, i), point_dist(sys, rold, xyz, i)};
        for (int c = 0; c < 2; ++c) {
            double u, du, d2u;
            or_u_derivs(sys, r[c], &u, &du, &d2u);
            au += fabs(du);
            av += r[c] <= h ? fabs(or_aziz_deriv(r[c])) : 0.0;
        }
    }
    *slope_u = au;
    *slope_v = av;
}

/* Local energy E_L = H psi / psi (Sec. 2, local value A_L) with the Hamiltonian
 * of Sec. 2.  For psi = exp(U):
 *   grad_i ln psi = G_i = sum_{j != i} u'(r_ij) (r_i - r_j) / r_ij,
 *   lap_i  ln psi = L_i = sum_{j != i} [u''(r_ij) + 2 u'(r_ij) / r_ij],
 *   (lap_i psi)/psi = L_i + |G_i|^2.
 * With kappa = hbar^2 / (2 m):
 *   T_PB = -kappa sum_i (L_i + |G_i|^2)      (local kinetic energy),
 *   T_JF = -(kappa/2) sum_i L_i,  T_F = kappa sum_i |G_i|^2.
 * Reading: the text after Eq. (8) says the symmetrized u allows alternative
 * kinetic estimators, and Sec. 5.4 lists two kinetic estimates that must agree
 * statistically; these are taken to be T_PB and T_JF, with T_F as a third.
 * All three have the same expectation over |psi|^2.  E_L = V + T_PB. */
/* Pair distribution histogram (Sec. 5.4: the host analysis accumulates the
 * pair distribution function of the sampled configurations; Sec. 7 cuts every
 * pair term at half the box).  Bins of equal width in r over [0, L/2]. */
void or_pair_histogram(const or_system *sys, const double *xyz, int32_t nb, uint64_t *counts,
                       uint64_t *edge, double rel_window)
{
    const int n = sys->n;
    const double h = 0.5 * sys->L;
    const double width = h / nb;
    double d[3];
    for (int b = 0; b < nb; ++b)
        counts[b] = 0;
    if (edge)
        for (int b = 0; b <= nb; ++b)
            edge[b] = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double r = pair_dist(sys, xyz, i, j, d);
            const double x = r / width;
            if (edge) {
                const double e = floor(x + 0.5);
                if (e <= nb && fabs(x - e) <= rel_window * (e > 1.0 ? e : 1.0))
                    edge[(int)e] += 1;
            }
            if (r > h)
                continue;
            int b = (int)floor(x);
            if (b >= nb)
                b = nb - 1;
            counts[b] += 1;
        }
}

void or_local_energy(const or_system *sys, const double *xyz, double out[6], double *scale,
                     double *grad, double *lap)
{
    const int n = sys->n;
    const double kappa = 0.5 * sys->hbar2_over_m;
    double *G = (double *)calloc((size_t)3 * n, sizeof(double));
    double *Lp = (double *)calloc((size_t)n, sizeof(double));
    double *cG = (double *)calloc((size_t)3 * n, sizeof(double));
    double *cL = (double *)calloc((size_t)n, sizeof(double));
    double sv = 0, cv = 0, su = 0, cu = 0, av = 0;
    double d[3];
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double r = pair_dist(sys, xyz, i, j, d);
            if (r > 0.5 * sys->L)
                continue;
            double u, du, d2u;
            or_u_derivs(sys, r, &u, &du, &d2u);
            double v = or_aziz(r);
            nsum(&sv, &cv, v);
            nsum(&su, &cu, u);
            av += fabs(v);
            for (int a = 0; a < 3; ++a) {
                double g = du * d[a] / r;
                nsum(&G[a * n + i], &cG[a * n + i], g);
                nsum(&G[a * n + j], &cG[a * n + j], -g);
            }
            double l = d2u + 2.0 * du / r;
            nsum(&Lp[i], &cL[i], l);
            nsum(&Lp[j], &cL[j], l);
        }
    double sl = 0, cl = 0, sg = 0, cg = 0, al = 0;
    for (int i = 0; i < n; ++i) {
        double gx = G[i] + cG[i], gy = G[n + i] + cG[n + i], gz = G[2 * n + i] + cG[2 * n + i];
        double li = Lp[i] + cL[i];
        double g2 = gx * gx + gy * gy + gz * gz;
        nsum(&sl, &cl, li);
        nsum(&sg, &cg, g2);
        al += fabs(li) + g2;
        if (grad) {
            grad[i] = gx; grad[n + i] = gy; grad[2 * n + i] = gz;
        }
        if (lap)
            lap[i] = li;
    }
    double V = sv + cv, sumL = sl + cl, sumG2 = sg + cg;
    double tpb = -kappa * (sumL + sumG2);
    double tjf = -0.5 * kappa * sumL;
    double tf = kappa * sumG2;
    out[0] = V + tpb;
    out[1] = V;
    out[2] = tpb;
    out[3] = tjf;
    out[4] = tf;
    out[5] = su + cu;
    if (scale)
        *scale = av + kappa * al;
    free(G); free(Lp); free(cG); free(cL);
}

/* Start configuration.  The paper reads starting coordinates from an input file
 * (Sec. 5.1).  Reading: an fcc lattice filling the box, n^3 cells with
 * N = 4 n^3 (for other N the first N sites of the smallest enclosing lattice),
 * site p = 4 ((ix n + iy) n + iz) + beta at a ((ix,iy,iz) + basis_beta + 1/4),
 * then each coordinate moved by 1e-3 a (U - 1/2), with U from Philox counter
 * (p, 0xFFFFFFFF, w, 2), word 0/1/2 for x/y/z, so that no pair sits exactly on
 * the cutoff distance L/2. */
void or_fcc_start(const or_system *sys, uint32_t w, double *xyz)
{
    const int n = sys->n;
    int nc = 1;
    while (4 * nc * nc * nc < n)
        ++nc;
    const double a = sys->L / nc;
    static const double basis[4][3] = {{0, 0, 0}, {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};
    const uint32_t key[2] = {(uint32_t)sys->seed, (uint32_t)(sys->seed >> 32)};
    for (int p = 0; p < n; ++p) {
        int beta = p % 4, cell = p / 4;
        int iz = cell % nc, iy = (cell / nc) % nc, ix = cell / (nc * nc);
        int idx[3] = {ix, iy, iz};
        uint32_t ctr[4] = {(uint32_t)p, 0xFFFFFFFFu, w, 2u}, r[4];
        or_philox4x32_10(ctr, key, r);
        for (int c = 0; c < 3; ++c) {
            double x = a * ((double)idx[c] + basis[beta][c] + 0.25);
            xyz[c * n + p] = stored_coord(sys, x + 1e-3 * a * (unit32(r[c]) - 0.5));
        }
    }
}

void or_walker_init(const or_system *sys, const double *xyz, or_walker *acc)
{
    memset(acc, 0, sizeof(*acc));
    or_totals(sys, xyz, &acc->u_run, &acc->v_run);
}

/* Eq. (5): accept the trial configuration if the ratio of the squared
 * wavefunctions, exp(2 dU) by Eq. (7), exceeds the uniform xi (strict ">"). */
int or_metropolis_accept(double du, double xi)
{
    return exp(2.0 * du) > xi;
}

/* Sec. 5.1 workflow for one walker (one Markov chain): N micro-updates per
 * sweep ("macroupdate", Sec. 4.1); each draws s, xi, delta, forms dU by Eq. (7),
 * accepts by Eq. (5) (strict ">"), and on acceptance moves r_s.  Analysis
 * (local energy) every m sweeps (Sec. 4.1).  log: see or_run_walker_log. */
static int run_walker(const or_system *sys, uint32_t w, double *xyz, or_walker *acc,
                      uint32_t t0, int32_t n_sweeps, uint32_t measure_start, int32_t m,
                      double *el_out, int64_t *n_el, double *log, int64_t log_cap)
{
    const int n = sys->n;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        const uint32_t t = t0 + (uint32_t)it;
        const int measured = t >= measure_start;
        for (int k = 0; k < n; ++k) {
            int32_t s;
            double xi, delta[3], rnew[3], du, dv, scu, scv;
            or_draw_move(sys, (uint32_t)k, t, w, &s, &xi, delta);
            or_trial_position(sys, xyz, s, delta, rnew);
            or_delta(sys, xyz, s, rnew, &du, &dv, &scu, &scv);
            int accept = or_metropolis_accept(du, xi);
            const int64_t q = (int64_t)it * n + k;
            if (log && q < log_cap) {
                double *rec = log + 8 * q;
                rec[0] = (double)s;
                rec[1] = (double)accept;
                rec[2] = du;
                rec[3] = dv;
                rec[4] = scu;
                rec[5] = scv;
                or_delta_slopes(sys, xyz, s, rnew, &rec[6], &rec[7]);
            }
            if (measured) {
                acc->n_try += 1;
                acc->n_acc += accept;
            }
            if (accept) {
                xyz[s] = rnew[0];
                xyz[n + s] = rnew[1];
                xyz[2 * n + s] = rnew[2];
                acc->u_run += du;
                acc->v_run += dv;
            }
        }
        if (!measured)
            continue;
        if (m > 0 && (t - measure_start + 1) % (uint32_t)m == 0) {
            double el[6];
            or_local_energy(sys, xyz, el, NULL, NULL, NULL);
            nsum(&acc->sum_e, &acc->c_e, el[0]);
            nsum(&acc->sum_e2, &acc->c_e2, el[0] * el[0]);
            nsum(&acc->sum_v, &acc->c_v, el[1]);
            nsum(&acc->sum_tpb, &acc->c_tpb, el[2]);
            nsum(&acc->sum_tjf, &acc->c_tjf, el[3]);
            nsum(&acc->sum_tf, &acc->c_tf, el[4]);
            acc->n_samples += 1;
            /* the running totals restart from the fresh evaluation */
            acc->u_run = el[5];
            acc->v_run = el[1];
            if (el_out)
                el_out[(*n_el)++] = el[0];
        }
        nsum(&acc->sum_vs, &acc->c_vs, acc->v_run);
        acc->n_sweeps_meas += 1;
    }
    return 0;
}

int or_run_walker(const or_system *sys, uint32_t w, double *xyz, or_walker *acc,
                  uint32_t t0, int32_t n_sweeps, uint32_t measure_start, int32_t m,
                  double *el_out, int64_t *n_el)
{
    return run_walker(sys, w, xyz, acc, t0, n_sweeps, measure_start, m, el_out, n_el, NULL, 0);
}

int or_run_walker_log(const or_system *sys, uint32_t w, double *xyz, or_walker *acc,
                      uint32_t t0, int32_t n_sweeps, uint32_t measure_start, int32_t m,
                      double *log, int64_t log_cap)
{
    return run_walker(sys, w, xyz, acc, t0, n_sweeps, measure_start, m, NULL, NULL, log, log_cap);
}

/* ------------------------------------------------------------------------ */
typedef struct {
    const or_system *sys;
    uint32_t w0;
    int32_t nw, stride, first;
    double *xyz;
    or_walker *acc;
    uint32_t t0, measure_start;
    int32_t n_sweeps, m;
} or_job;

static void *run_job(void *arg)
{
    or_job *j = (or_job *)arg;
    const size_t blk = (size_t)3 * j->sys->n;
    for (int32_t i = j->first; i < j->nw; i += j->stride)
        or_run_walker(j->sys, j->w0 + (uint32_t)i, j->xyz + blk * i, &j->acc[i], j->t0,
                      j->n_sweeps, j->measure_start, j->m, NULL, NULL);
    return NULL;
}

int or_run_walkers(const or_system *sys, uint32_t w0, int32_t nw, double *xyz,
                   or_walker *acc, uint32_t t0, int32_t n_sweeps, uint32_t measure_start,
                   int32_t m, int32_t n_threads)
{
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > nw)
        n_threads = nw;
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    or_job *jobs = (or_job *)calloc((size_t)n_threads, sizeof(or_job));
    for (int i = 0; i < n_threads; ++i) {
        jobs[i] = (or_job){sys, w0, nw, n_threads, i, xyz, acc, t0, measure_start, n_sweeps, m};
        pthread_create(&th[i], NULL, run_job, &jobs[i]);
    }
    for (int i = 0; i < n_threads; ++i)
        pthread_join(th[i], NULL);
    free(th);
    free(jobs);
    return 0;
}
