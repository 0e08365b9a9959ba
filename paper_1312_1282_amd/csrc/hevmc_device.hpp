// Device-side building blocks of libhevmc (gfx950): counter-based random
// numbers, pair terms of the Jastrow wavefunction and the HFD-B(HE) potential,
// and wave64 / workgroup reductions.
//
// Method: Lutsyshyn, "Fast quantum Monte Carlo on a GPU" (arXiv:1312.1282),
// Sec. 2 (Eqs. (5)-(9)), Sec. 5.1, Sec. 7.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hevmc.h"

namespace hevmc {

// Kernel-side constants of one ensemble, derived once on the host.
struct KParams {
    int32_t n;           // atoms per walker
    int32_t order;       // hevmc_order
    uint32_t wid_base;   // Philox walker id of walker 0
    uint32_t key0, key1; // Philox key (seed)
    double L, invL;      // box side and its reciprocal
    double h2;           // (L/2)^2: pair cutoff, inclusive
    double step;         // Gaussian step, per component
    double c5;           // -b^5 / 2, so f(r) = c5 r^-5 (Eq. (9))
    double u0;           // -2 f(L/2): u(r) = f(r) + f(L-r) + u0 (Eq. (8), as read)
    double kappa;        // hbar^2 / 2m
    float Lf, invLf, h2f, c5f, u0f;
    // FP32 form of V with the constants folded (set on the host): eps A e^a =
    // 2^(r (vb r - va) + vl) with a = -alpha x + beta x^2, x = r / r_m;
    // F = 2^-((vd / r - vs)^2) for r < vdr = D r_m; dispersion coefficients
    // vc6, vc8, vc10 on powers of 1/r^2 (eps and r_m folded in)
    float vb, va, vl, vd, vs, vdr, vc6, vc8, vc10;
    int32_t sorted;      // sweep keeps the atoms in LDS in spatial (Morton) order
    int32_t gr_bins;     // bins of the pair histogram accumulated at each sample (0: none)
    uint64_t *gr;        // [W][gr_bins] histogram counts (device), or null
    double *trace;       // [W][trace_cap][6] per-sample local-energy records, or null
    int32_t trace_cap;   // samples per walker the trace holds
    uint32_t share_tag;  // nonzero: this launch's tag for balancing walkers that share a CU (0: off)
    double *movelog;     // [log_walkers][log_cap][4] per-move records (s, accepted, dU, dV), or null
    int64_t log_cap;     // records per logged walker
    int32_t log_walkers; // walkers 0 .. log_walkers-1 of the launch are logged
};

// HFD-B(HE) pair potential (Aziz, McCourt, Wong 1987), the interaction named
// in Sec. 2:  V = eps [A exp(-alpha x + beta x^2) - F(x)(C6 x^-6 + C8 x^-8 + C10 x^-10)],
// x = r / r_m, F(x) = exp(-(D/x - 1)^2) for x < D, else 1.
namespace az {
constexpr double eps = 10.948;
constexpr double rm = 2.963;
constexpr double A = 184431.01;
constexpr double alpha = 10.43329537;
constexpr double beta = -2.27965105;
constexpr double C6 = 1.36745214;
constexpr double C8 = 0.42123807;
constexpr double C10 = 0.17473318;
constexpr double D = 1.4826;
constexpr double inv_rm = 1.0 / rm;
constexpr double rm2 = rm * rm;
constexpr double Drm = D * rm;        // D / x = Drm / r
constexpr double beta_rm2 = beta / (rm * rm);   // -alpha x + beta x^2 = beta_rm2 r^2 - alpha_rm r
constexpr double alpha_rm = alpha / rm;
// eps folded into the amplitudes and r_m into the dispersion coefficients
// (the FP32 form's constants): eps C_k x^-k = eC_k w^(k/2), w = r^-2,
// eC_k = eps C_k r_m^k
constexpr double epsA = eps * A;
constexpr double eC6 = eps * C6 * rm2 * rm2 * rm2;
constexpr double eC8 = eC6 / C6 * C8 * rm2;
constexpr double eC10 = eC6 / C6 * C10 * rm2 * rm2;
// The repulsive exponential is skipped where its exponent is below rep_min:
// there eps A e^a < 2.7e-18 K, under half an ulp of V itself at the distance
// where that happens (9.27 A, V = -0.016 K).
constexpr double rep_min = -55.0;
}  // namespace az

// 1/k! for k = 12, 11, ..., 3: the Taylor coefficients of exp_neg, in
// constant memory.  Not declared const, so the compiler cannot fold them into
// the code: it loads them once into scalar registers, where each Horner step
// takes its coefficient as the addend of one FMA.  As compile-time constants
// they would be held in vector registers and copied before every step (the
// addend of the two-operand FMA form is also its result).
// (Defined in the kernels' translation unit only; external linkage keeps the
// optimiser from treating the initial values as the final ones.)
#ifdef HEVMC_KERNELS_TU
__constant__ double exp_taylor[10] = {
    2.08767569878680989792e-09, 2.50521083854417187751e-08, 2.75573192239858906526e-07,
    2.75573192239858906526e-06, 2.48015873015873015873e-05, 1.98412698412698412698e-04,
    1.38888888888888888889e-03, 8.33333333333333333333e-03, 4.16666666666666666667e-02,
    1.66666666666666666667e-01};
#else
extern __constant__ double exp_taylor[10];
#endif

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ double unit32(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// The five random numbers of micro-step k of sweep t (Sec. 2: random atom s and
// Gaussian displacement; Eq. (5): uniform xi; Sec. 5.1: Box-Muller).  Two
// Philox blocks with counters (k, t, wid, 0) and (k, t, wid, 1):
//   s = floor(a0 N / 2^32) (or k), xi = (top 52 bits of a1:a2 + 1/2) 2^-52,
//   delta = step (R cos 2pi u2, R sin 2pi u2, R' cos 2pi u4),
//   R = sqrt(-2 ln u1), R' = sqrt(-2 ln u3), (u1,u2,u3,u4) from (a3, b0, b1, b2).
__device__ __forceinline__ void draw_move(const KParams &p, uint32_t k, uint32_t t, uint32_t wid,
                                          int &s, double &xi, double &dx, double &dy, double &dz)
{
    uint32_t a[4], b[4];
    philox4x32_10(k, t, wid, 0u, p.key0, p.key1, a);
    philox4x32_10(k, t, wid, 1u, p.key0, p.key1, b);
    s = (p.order == HEVMC_SELECT_SEQUENTIAL) ? (int)(k % (uint32_t)p.n)
                                             : (int)__umulhi(a[0], (uint32_t)p.n);
    const uint64_t m52 = ((uint64_t)a[1] << 20) | (uint64_t)(a[2] >> 12);
    xi = ((double)m52 + 0.5) * 0x1p-52;
    const double two_pi = 6.283185307179586;
    const double R1 = sqrt(-2.0 * log(unit32(a[3])));
    const double R2 = sqrt(-2.0 * log(unit32(b[1])));
    double sn, cs;
    sincos(two_pi * unit32(b[0]), &sn, &cs);
    dx = p.step * (R1 * cs);
    dy = p.step * (R1 * sn);
    dz = p.step * (R2 * cos(two_pi * unit32(b[2])));
}

// Periodic wrap of a moved coordinate into [0, L) (Sec. 5.1): y - L floor(y/L),
// with y/L formed as y * (1/L) and the two results rounding can leave outside
// [0, L) moved back in.
__device__ __forceinline__ double wrap_box(double y, double L, double invL)
{
    double x = y - L * floor(y * invL);
    x = (x >= L) ? x - L : x;
    return (x < 0.0) ? x + L : x;
}

// A wrapped trial coordinate as the walker stores it.  In FP32 a value just
// below L can round up to L itself, the same point as 0 of the periodic box:
// it is stored as 0, so every stored coordinate lies in [0, L).
__device__ __forceinline__ double stored_coord(double y, const KParams &p) { return wrap_box(y, p.L, p.invL); }
__device__ __forceinline__ float stored_coord_f(double y, const KParams &p)
{
    const float v = (float)wrap_box(y, p.L, p.invL);
    return v >= p.Lf ? 0.0f : v;
}
template <typename T>
__device__ __forceinline__ T trial_coord(double y, const KParams &p)
{
    if constexpr (sizeof(T) == 4)
        return stored_coord_f(y, p);
    else
        return stored_coord(y, p);
}

// Minimum image of one coordinate difference (Sec. 5.1), signed (the local
// energy's gradient needs the direction).
__device__ __forceinline__ double min_image(double d, const KParams &p) { return d - p.L * rint(d * p.invL); }
__device__ __forceinline__ float min_image(float d, const KParams &p) { return d - p.Lf * rintf(d * p.invLf); }

// Length of the minimum image of d = a - b for coordinates a, b in [0, L): the
// shorter of |d| and L - |d|.  For |d| >= L/2, L - |d| is exact (Sterbenz), so
// the result equals the signed form's magnitude wherever that form rounds
// d / L away from 1/2, and it takes three instructions instead of four.  Used
// where only squares of the components matter.
__device__ __forceinline__ double image_len(double d, const KParams &p)
{
    const double a = fabs(d);
    return fmin(a, p.L - a);
}
__device__ __forceinline__ float image_len(float d, const KParams &p)
{
    const float a = fabsf(d);
    return fminf(a, p.Lf - a);
}

// --------------------------------------------------------------------------
// FP64 elementary functions for the pair loop.  Division, sqrt and exp from the
// device math library are correctly rounded or within an ulp but expand to long
// instruction sequences; these use the hardware estimates with Newton steps.

// 1/x: hardware reciprocal estimate refined by one Newton step
// (y <- y + y (1 - x y)).  On gfx950 the estimate's relative error is below
// 5e-8 and one step brings it below 3e-15 (measured over 1e-2 <= x <= 1e4),
// three orders inside the 1e-12 tolerance the sums are held to.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// 1/sqrt(x): hardware estimate refined by one Newton step
// (y <- y + (y/2)(1 - x y^2)); below 5e-15 relative after the step.
__device__ __forceinline__ double rsq_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// e^a for a <= 0 (both exponentials of the potential have non-positive
// arguments).  Cody-Waite reduction a = k ln2 + f, |f| <= ln2/2, with the
// two-part ln2 of fdlibm (its high part has trailing zero bits, so k*ln2_hi is
// exact), e^f by its Taylor series to degree 12 (truncation < 2e-16 relative),
// scaled by 2^k.  For a below about -745 the scaling underflows to zero, the
// value of e^a in FP64 (a = -inf, the distance-zero pair of an atom with
// itself, gives NaN, which the callers' masks discard).  The coefficients of
// degrees 12 .. 3 come from exp_taylor.
__device__ __forceinline__ double exp_neg(const KParams &, double a)
{
    const double k = rint(a * 1.4426950408889634);
    double f = fma(-k, 6.93147180369123816490e-01, a);
    f = fma(-k, 1.90821492927058770002e-10, f);
    double q = exp_taylor[0];
#pragma unroll
    for (int j = 1; j < 10; ++j)
        q = fma(q, f, exp_taylor[j]);
    q = fma(q, f, 0.5);
    q = fma(q, f, 1.0);
    q = fma(q, f, 1.0);
    return ldexp(q, (int)k);
}

// v if keep, else v with its high word cleared: a number below 2^-1022 in
// magnitude, which no sum it enters can feel (one 32-bit select instead of
// two; a masked NaN also becomes such a number).
__device__ __forceinline__ double keep_or_tiny(bool keep, double v)
{
    return __hiloint2double(keep ? __double2hiint(v) : 0, __double2loint(v));
}

// --------------------------------------------------------------------------
// Pair terms at squared min-image distance r2 (Eqs. (8), (9); HFD-B(HE)).
// u and V are zero beyond the inclusive cutoff L/2 (in the FP64 terms of the
// row-sum sweep, keep_or_tiny's numerical zero); callers mask i == s
// (r2 = 0 gives non-finite terms that the mask discards).

// FP64: u(r) and V(r).
__device__ __forceinline__ void pair_uv(const KParams &p, double r2, double &u, double &v)
{
    const double ri = rsq_nr(r2);
    const double r = r2 * ri;
    const double rpi = rcp_nr(p.L - r);
    const double ri2 = ri * ri, rpi2 = rpi * rpi;
    const double uu = fma(p.c5, fma(ri2 * ri2, ri, rpi2 * rpi2 * rpi), p.u0);
    const double ea = fma(az::beta_rm2, r2, -(az::alpha_rm * r));
    double rep = 0.0;
    if (ea > az::rep_min)
        rep = az::A * exp_neg(p, ea);
    const double y = az::rm2 * ri2;                   // x^-2
    const double y2 = y * y;
    const double disp = y2 * y * fma(y, fma(y, az::C10, az::C8), az::C6);
    double F = 1.0;
    if (r < az::Drm) {
        const double q = fma(az::Drm, ri, -1.0);
        F = exp_neg(p, -(q * q));
    }
    const double vv = az::eps * fma(-F, disp, rep);
    const bool in = r2 <= p.h2;
    u = in ? uu : 0.0;
    v = in ? vv : 0.0;
}

// FP64: pair_uv at two distances (a moved atom's old and new position against
// one partner), each bitwise equal to pair_uv; the exponentials of both are
// formed in shared branches so that their Horner chains interleave.
__device__ __forceinline__ void pair_uv2(const KParams &p, double r2a, double r2b, double &ua, double &va,
                                         double &ub, double &vb)
{
    const double ria = rsq_nr(r2a), rib = rsq_nr(r2b);
    const double ra = r2a * ria, rb = r2b * rib;
    const double rpa = rcp_nr(p.L - ra), rpb = rcp_nr(p.L - rb);
    const double ria2 = ria * ria, rpa2 = rpa * rpa, rib2 = rib * rib, rpb2 = rpb * rpb;
    const double uua = fma(p.c5, fma(ria2 * ria2, ria, rpa2 * rpa2 * rpa), p.u0);
    const double uub = fma(p.c5, fma(rib2 * rib2, rib, rpb2 * rpb2 * rpb), p.u0);
    const double eaa = fma(az::beta_rm2, r2a, -(az::alpha_rm * ra));
    const double eab = fma(az::beta_rm2, r2b, -(az::alpha_rm * rb));
    const bool ka = eaa > az::rep_min, kb = eab > az::rep_min;
    double repa = 0.0, repb = 0.0;
    if (ka || kb) {
        const double xa = exp_neg(p, eaa), xb = exp_neg(p, eab);
        repa = ka ? az::A * xa : 0.0;
        repb = kb ? az::A * xb : 0.0;
    }
    const double ya = az::rm2 * ria2, yb = az::rm2 * rib2;
    const double ya2 = ya * ya, yb2 = yb * yb;
    const double dispa = ya2 * ya * fma(ya, fma(ya, az::C10, az::C8), az::C6);
    const double dispb = yb2 * yb * fma(yb, fma(yb, az::C10, az::C8), az::C6);
    const bool da = ra < az::Drm, db = rb < az::Drm;
    double Fa = 1.0, Fb = 1.0;
    if (da || db) {
        const double qa = fma(az::Drm, ria, -1.0), qb = fma(az::Drm, rib, -1.0);
        const double xa = exp_neg(p, -(qa * qa)), xb = exp_neg(p, -(qb * qb));
        Fa = da ? xa : 1.0;
        Fb = db ? xb : 1.0;
    }
    const double vva = az::eps * fma(-Fa, dispa, repa), vvb = az::eps * fma(-Fb, dispb, repb);
    const bool ina = r2a <= p.h2, inb = r2b <= p.h2;
    ua = ina ? uua : 0.0;
    va = ina ? vva : 0.0;
    ub = inb ? uub : 0.0;
    vb = inb ? vvb : 0.0;
}

// Whether a pair at squared distance r2 is inside the (inclusive) cutoff.
__device__ __forceinline__ bool pair_inside(const KParams &p, double r2) { return r2 <= p.h2; }
__device__ __forceinline__ bool pair_inside(const KParams &p, float r2) { return r2 <= p.h2f; }

// Reciprocal distance from r^2 in the pair's precision.
__device__ __forceinline__ double inv_sqrt(double r2) { return rsq_nr(r2); }
__device__ __forceinline__ float inv_sqrt(float r2) { return __builtin_amdgcn_rsqf(r2); }

// FP64: u(r) alone, given r^2 and 1/r (the forward half of a micro-update
// needs only ln psi).
__device__ __forceinline__ double pair_u_ri(const KParams &p, double r2, double ri)
{
    const double r = r2 * ri;
    const double rpi = rcp_nr(p.L - r);
    const double ri2 = ri * ri, rpi2 = rpi * rpi;
    const double uu = fma(p.c5, fma(ri2 * ri2, ri, rpi2 * rpi2 * rpi), p.u0);
    return keep_or_tiny(r2 <= p.h2, uu);
}

// u(r) for a pair that counts if `keep` (the moved atom itself does not):
// (numerically) zero beyond the cutoff or when !keep, with one select for both.
__device__ __forceinline__ double pair_u_in(const KParams &p, double r2, double ri, bool keep)
{
    const double r = r2 * ri;
    const double rpi = rcp_nr(p.L - r);
    const double ri2 = ri * ri, rpi2 = rpi * rpi;
    const double uu = fma(p.c5, fma(ri2 * ri2, ri, rpi2 * rpi2 * rpi), p.u0);
    return keep_or_tiny(keep && r2 <= p.h2, uu);
}

// FP64: V(r) alone, given r^2 and 1/r.
__device__ __forceinline__ double pair_v_ri(const KParams &p, double r2, double ri)
{
    const double r = r2 * ri;
    const double ea = fma(az::beta_rm2, r2, -(az::alpha_rm * r));
    double rep = 0.0;
    if (ea > az::rep_min)
        rep = az::A * exp_neg(p, ea);
    const double y = az::rm2 * (ri * ri);
    const double y2 = y * y;
    const double disp = y2 * y * fma(y, fma(y, az::C10, az::C8), az::C6);
    double F = 1.0;
    if (r < az::Drm) {
        const double q = fma(az::Drm, ri, -1.0);
        F = exp_neg(p, -(q * q));
    }
    const double vv = az::eps * fma(-F, disp, rep);
    return keep_or_tiny(r2 <= p.h2, vv);
}

// FP64: V at two distances (a moved atom's old and new position against one
// partner), each bitwise equal to pair_v_ri, in three phases: vp_pre forms
// everything but the exponentials, vp_exp the exponentials, vp_post the two
// values.  An exponential is formed for both distances when either needs it
// (the other's value is discarded), so the two dependent Horner chains run
// interleaved in one branch instead of one after the other in two.  A caller
// holding several such pairs runs every pair's vp_pre, then every vp_exp, then
// every vp_post, so that the pairs' arithmetic also interleaves outside the
// branches; pair_v_ri2 is the three phases for one pair.
struct VPair {
    double disa, disb, eaa, eab, qa, qb, repa, repb, Fa, Fb;
    bool ka, kb, da, db, ina, inb;
};

__device__ __forceinline__ void vp_pre(const KParams &p, double r2a, double ria, double r2b, double rib, VPair &v)
{
    const double ra = r2a * ria, rb = r2b * rib;
    v.eaa = fma(az::beta_rm2, r2a, -(az::alpha_rm * ra));
    v.eab = fma(az::beta_rm2, r2b, -(az::alpha_rm * rb));
    v.ka = v.eaa > az::rep_min;
    v.kb = v.eab > az::rep_min;
    const double ya = az::rm2 * (ria * ria), yb = az::rm2 * (rib * rib);
    const double ya2 = ya * ya, yb2 = yb * yb;
    v.disa = ya2 * ya * fma(ya, fma(ya, az::C10, az::C8), az::C6);
    v.disb = yb2 * yb * fma(yb, fma(yb, az::C10, az::C8), az::C6);
    v.da = ra < az::Drm;
    v.db = rb < az::Drm;
    v.qa = fma(az::Drm, ria, -1.0);
    v.qb = fma(az::Drm, rib, -1.0);
    v.ina = r2a <= p.h2;
    v.inb = r2b <= p.h2;
}

__device__ __forceinline__ void vp_exp(const KParams &p, VPair &v)
{
    v.repa = 0.0;
    v.repb = 0.0;
    if (v.ka || v.kb) {
        const double xa = exp_neg(p, v.eaa), xb = exp_neg(p, v.eab);
        v.repa = v.ka ? az::A * xa : 0.0;
        v.repb = v.kb ? az::A * xb : 0.0;
    }
    v.Fa = 1.0;
    v.Fb = 1.0;
    if (v.da || v.db) {
        const double xa = exp_neg(p, -(v.qa * v.qa)), xb = exp_neg(p, -(v.qb * v.qb));
        v.Fa = v.da ? xa : 1.0;
        v.Fb = v.db ? xb : 1.0;
    }
}

__device__ __forceinline__ void vp_post(const VPair &v, double &va, double &vb)
{
    va = keep_or_tiny(v.ina, az::eps * fma(-v.Fa, v.disa, v.repa));
    vb = keep_or_tiny(v.inb, az::eps * fma(-v.Fb, v.disb, v.repb));
}

__device__ __forceinline__ void pair_v_ri2(const KParams &p, double r2a, double ria, double r2b, double rib,
                                           double &va, double &vb)
{
    VPair v;
    vp_pre(p, r2a, ria, r2b, rib, v);
    vp_exp(p, v);
    vp_post(v, va, vb);
}

// FP32 form: same terms in single precision with the hardware reciprocal,
// reciprocal square root and base-2 exponential.

// FP32 V(r) from r, 1/r and 1/r^2 with the host-folded constants of KParams
// (no cutoff): the same terms as the FP64 form, each exponential one exp2.
__device__ __forceinline__ float aziz_f(const KParams &p, float r, float ri, float w)
{
    const float rep = __builtin_amdgcn_exp2f(fmaf(r, fmaf(p.vb, r, -p.va), p.vl));
    const float disp = w * w * w * fmaf(w, fmaf(w, p.vc10, p.vc8), p.vc6);
    const float q = fmaf(p.vd, ri, -p.vs);
    const float F = r < p.vdr ? __builtin_amdgcn_exp2f(-(q * q)) : 1.0f;
    return fmaf(-F, disp, rep);
}

__device__ __forceinline__ void pair_uv(const KParams &p, float r2, float &u, float &v)
{
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float rpi = __builtin_amdgcn_rcpf(p.Lf - r);
    const float ri2 = ri * ri, rpi2 = rpi * rpi;
    const float uu = p.c5f * (ri2 * ri2 * ri + rpi2 * rpi2 * rpi) + p.u0f;
    const float vv = aziz_f(p, r, ri, ri2);
    const bool in = r2 <= p.h2f;
    u = in ? uu : 0.0f;
    v = in ? vv : 0.0f;
}

__device__ __forceinline__ void pair_uv2(const KParams &p, float r2a, float r2b, float &ua, float &va, float &ub,
                                         float &vb)
{
    pair_uv(p, r2a, ua, va);
    pair_uv(p, r2b, ub, vb);
}

__device__ __forceinline__ float pair_u_ri(const KParams &p, float r2, float ri)
{
    const float r = r2 * ri;
    const float rpi = __builtin_amdgcn_rcpf(p.Lf - r);
    const float ri2 = ri * ri, rpi2 = rpi * rpi;
    const float uu = p.c5f * (ri2 * ri2 * ri + rpi2 * rpi2 * rpi) + p.u0f;
    return r2 <= p.h2f ? uu : 0.0f;
}

__device__ __forceinline__ float pair_u_in(const KParams &p, float r2, float ri, bool keep)
{
    const float r = r2 * ri;
    const float rpi = __builtin_amdgcn_rcpf(p.Lf - r);
    const float ri2 = ri * ri, rpi2 = rpi * rpi;
    const float uu = p.c5f * (ri2 * ri2 * ri + rpi2 * rpi2 * rpi) + p.u0f;
    return (keep && r2 <= p.h2f) ? uu : 0.0f;
}

__device__ __forceinline__ float pair_v_ri(const KParams &p, float r2, float ri)
{
    const float vv = aziz_f(p, r2 * ri, ri, ri * ri);
    return r2 <= p.h2f ? vv : 0.0f;
}

__device__ __forceinline__ void pair_v_ri2(const KParams &p, float r2a, float ria, float r2b, float rib, float &va,
                                           float &vb)
{
    va = pair_v_ri(p, r2a, ria);
    vb = pair_v_ri(p, r2b, rib);
}

// Terms of the local energy of one ordered pair: u, V, u'/r (the gradient of
// ln psi is sum u'/r d) and u'' + 2u'/r (the Laplacian term), zero beyond L/2.
// u' = -5 c5 (r^-6 - (L-r)^-6), u'' = 30 c5 (r^-7 + (L-r)^-7).
struct ETerms {
    double u, v, dur, lap;
    double r;   // the pair distance (for the pair histogram)
};

__device__ __forceinline__ void pair_energy(const KParams &p, double r2, ETerms &e)
{
    const double ri = rsq_nr(r2);
    const double r = r2 * ri;
    const double rpi = rcp_nr(p.L - r);
    const double ri2 = ri * ri, rpi2 = rpi * rpi;
    const double ri5 = ri2 * ri2 * ri, rpi5 = rpi2 * rpi2 * rpi;
    const double ri6 = ri5 * ri, rpi6 = rpi5 * rpi;
    const double uu = fma(p.c5, ri5 + rpi5, p.u0);
    const double du = -5.0 * p.c5 * (ri6 - rpi6);
    const double d2u = 30.0 * p.c5 * fma(ri6, ri, rpi6 * rpi);
    const double ea = fma(az::beta_rm2, r2, -(az::alpha_rm * r));
    double rep = 0.0;
    if (ea > az::rep_min)
        rep = az::A * exp_neg(p, ea);
    const double y = az::rm2 * ri2;
    const double y2 = y * y;
    const double disp = y2 * y * fma(y, fma(y, az::C10, az::C8), az::C6);
    double F = 1.0;
    if (r < az::Drm) {
        const double q = fma(az::Drm, ri, -1.0);
        F = exp_neg(p, -(q * q));
    }
    const double vv = az::eps * fma(-F, disp, rep);
    const double dur = du * ri;
    const bool in = r2 <= p.h2;
    e.r = r;
    e.u = in ? uu : 0.0;
    e.v = in ? vv : 0.0;
    e.dur = in ? dur : 0.0;
    e.lap = in ? fma(2.0, dur, d2u) : 0.0;
}

// The gradient and row terms of an ordered pair alone: u and u'/r, zero beyond
// L/2 (the symmetric terms V and the Laplacian are formed once per unordered
// pair by the caller).
__device__ __forceinline__ void pair_grad_u(const KParams &p, double r2, double &u, double &dur)
{
    const double ri = rsq_nr(r2);
    const double r = r2 * ri;
    const double rpi = rcp_nr(p.L - r);
    const double ri2 = ri * ri, rpi2 = rpi * rpi;
    const double ri5 = ri2 * ri2 * ri, rpi5 = rpi2 * rpi2 * rpi;
    const double ri6 = ri5 * ri, rpi6 = rpi5 * rpi;
    const double uu = fma(p.c5, ri5 + rpi5, p.u0);
    const double du = -5.0 * p.c5 * (ri6 - rpi6);
    const bool in = r2 <= p.h2;
    u = in ? uu : 0.0;
    dur = in ? du * ri : 0.0;
}

__device__ __forceinline__ void pair_grad_u(const KParams &p, float r2, double &u, double &dur)
{
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float rpi = __builtin_amdgcn_rcpf(p.Lf - r);
    const float ri2 = ri * ri, rpi2 = rpi * rpi;
    const float ri5 = ri2 * ri2 * ri, rpi5 = rpi2 * rpi2 * rpi;
    const float ri6 = ri5 * ri, rpi6 = rpi5 * rpi;
    const float uu = p.c5f * (ri5 + rpi5) + p.u0f;
    const float du = -5.0f * p.c5f * (ri6 - rpi6);
    const bool in = r2 <= p.h2f;
    u = in ? (double)uu : 0.0;
    dur = in ? (double)(du * ri) : 0.0;
}

__device__ __forceinline__ void pair_energy(const KParams &p, float r2, ETerms &e)
{
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float rpi = __builtin_amdgcn_rcpf(p.Lf - r);
    const float ri2 = ri * ri, rpi2 = rpi * rpi;
    const float ri5 = ri2 * ri2 * ri, rpi5 = rpi2 * rpi2 * rpi;
    const float ri6 = ri5 * ri, rpi6 = rpi5 * rpi;
    const float uu = p.c5f * (ri5 + rpi5) + p.u0f;
    const float du = -5.0f * p.c5f * (ri6 - rpi6);
    const float d2u = 30.0f * p.c5f * (ri6 * ri + rpi6 * rpi);
    const float vv = aziz_f(p, r, ri, ri2);
    const float dur = du * ri;
    const bool in = r2 <= p.h2f;
    e.r = (double)r;
    e.u = in ? (double)uu : 0.0;
    e.v = in ? (double)vv : 0.0;
    e.dur = in ? (double)dur : 0.0;
    e.lap = in ? (double)(d2u + 2.0f * dur) : 0.0;
}

// Metropolis decision of Eq. (5): accept if |psi'|^2/|psi|^2 = exp(2 dU) > xi,
// xi in (0, 1), taken with the logarithm on the uniform: 2 dU > ln xi (the
// same decision up to rounding; ln xi is formed ahead of the move, off the
// decision's critical path).  For dU >= 0 the ratio is >= 1 > xi.
__device__ __forceinline__ bool metropolis_accept_log(double du, double log_xi)
{
    return du >= 0.0 || 2.0 * du > log_xi;
}

// --------------------------------------------------------------------------
// Reductions.  Within each 16-lane row, four DPP steps (swap neighbours, swap
// pairs, mirror halves, mirror the row) add each lane's value to a partner's,
// so every lane of the row ends with the bitwise-identical row sum (both
// partners add the same two operands).  The four row sums are then read as
// scalars and added in a fixed order.  The total depends only on the data and
// the lane layout, and every lane holds the same value.  All 64 lanes must be
// active.
// Every lane has a valid source under the four controls used here, so the
// moves need no prior value in their destination (no zeroing moves).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_double<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_double<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_double<0x141>(v);   // row_half_mirror
    v += dpp_double<0x140>(v);   // row_mirror
    return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// Neumaier-compensated accumulation: value = s + c.
__device__ __forceinline__ void nsum(double &s, double &c, double x)
{
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

}  // namespace hevmc
