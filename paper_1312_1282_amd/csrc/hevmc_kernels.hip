// libhevmc kernels for gfx950: the Metropolis sweep with its fused local-energy
// pass, and the standalone entry kernels used for start-up and parity checks.
//
// One workgroup advances one walker (one Markov chain, Sec. 3).  The walker's
// coordinates live in LDS for the whole launch (Sec. 3: shared-memory
// persistence) as structure of arrays x[N], y[N], z[N]; HBM is touched only to
// load the walker at the start and store it at the end.  Each micro-update's
// O(N) pair loop of Eq. (7) is spread over the workgroup's lanes (lane tid owns
// atoms i = tid + j*NT), reduced per wave with DPP row sums and lane reads and
// across waves through a small double-buffered LDS array, so one barrier per
// micro-update suffices.  Every lane then takes the same Metropolis decision (Eq. (5)).
//
// Two variants of the micro-update:
//  * plain: the pair loop forms u and V at the old and the new position of the
//    moved atom for every trial move, as Eq. (7) is written;
//  * row sums (ROWS): each atom's row R_i = sum_{j != i} u(r_ij) is kept in LDS
//    (FP64), so the forward half of a micro-update evaluates u only at the new
//    position and dU = sum_i u(|r_s' - r_i|) - R_s.  Only an accepted move needs
//    the old-position terms: it updates the rows of all atoms and forms dV
//    (the potential change enters no result for a rejected move).  dV's
//    workgroup sum rides on the next micro-update's reduction.  Rows kept in
//    LDS are refreshed exactly by every local-energy pass; rows kept in
//    registers (walkers whose rows do not fit in LDS) are only updated move by
//    move within a launch.  Either way they can be kept in HBM between
//    launches and are checked against u_run (sum_i R_i = 2 U) on load.
//
// Walkers of at most 512 atoms can run one wave each, four to a workgroup,
// synchronised by wavefront fences only.  Larger walkers re-sort their atoms
// in LDS by cell at every sweep (spatial order), so that a wave's atoms are
// neighbours and whole waves skip the short-range exponentials.  The
// local-energy pass can also count a pair-distance histogram (g(r)) and the
// sweep can record every sample's local-energy terms; both leave the chain's
// bits unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#define HEVMC_KERNELS_TU 1
#include "hevmc_device.hpp"
#include "hevmc_internal.hpp"

namespace hevmc {

__device__ __forceinline__ int readlane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Synchronise the NT threads of one walker: the workgroup, or, when a walker
// is a single wave (NT = 64, several walkers per workgroup), the wave, whose
// LDS accesses are ordered by wavefront-scope fences.
template <int NT>
__device__ __forceinline__ void walker_sync()
{
    if constexpr (NT == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Thread index within a walker's NT threads.
template <int NT>
__device__ __forceinline__ int walker_tid() { return (int)(threadIdx.x & (NT - 1)); }

// Sum of NV doubles over a walker's NT threads; every thread gets the same
// totals.  For NT > 64, buf must hold NW*NV doubles (free again on return).
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *buf)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = walker_tid<NT>() >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q)
        v[q] = wave_sum(v[q]);
    if constexpr (NW == 1)
        return;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            buf[wave * NV + q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w)
            t += buf[w * NV + q];
        v[q] = t;
    }
    __syncthreads();
}

// True on every thread of a walker if pred holds on any of them (the walker's
// threads must all arrive; acts as walker_sync).  For NT > 64, buf as in
// block_sum (the runtime's workgroup vote would take LDS of its own, beyond
// the launch plan's budget).
template <int NT>
__device__ __forceinline__ bool walker_any(bool pred, double *buf)
{
    if constexpr (NT == 64) {
        walker_sync<64>();
        return __builtin_amdgcn_ballot_w64(pred) != 0;
    } else {
        double f[1] = {pred ? 1.0 : 0.0};
        block_sum<NT, 1>(f, buf);
        // decided here as one wave-uniform word, so that the partial sums are
        // not kept alive until the flag's use at the end of a launch
        return __builtin_amdgcn_readfirstlane(f[0] > 0.0 ? 1 : 0) != 0;
    }
}

// Local energy of the walker in LDS (Sec. 2 local value of H): out =
// (E_L, V, T_PB, T_JF, T_F, U).  Each lane owns atoms i = tid + c*NT and visits
// every other atom once, as j = i + k (mod N) for k = 1 .. N-1, so no atomics
// are needed.  The gradient of ln psi and the row sum of atom i need all N-1
// partners, but V and the Laplacian terms are symmetric in the pair: they are
// formed only for offsets k < N/2 (weight 2 for the Laplacian sum over atoms,
// which counts every pair twice) and k = N/2 (each such pair is met from both
// of its atoms: weight 1 and 1/2), halving the costliest pair terms.  If rows
// is not null, the row sums sum_{j != i} u(r_ij) of the lane's atoms are
// stored there (LDS or global memory).  If hist is not null, every unordered
// pair inside the cutoff is also counted in hist[min(nb - 1, floor(r nb / h))]
// (the pair distribution histogram, LDS, integer adds in any order).
template <typename T, int NT, bool HIST = false>
__device__ void local_energy_pass(const KParams &p, const T *sx, const T *sy, const T *sz, double *buf,
                                  double out[6], double *rows, uint32_t *hist = nullptr, int nb = 0)
{
    const double bin_scale = (double)nb * 2.0 * p.invL;   // bins per Angstrom
    const int n = p.n;
    const int half = (n - 1) / 2;   // offsets 1 .. half: all pair terms
    const bool mid = (n & 1) == 0;  // offset n/2: the antipodal pair, met twice
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // sum |G_i|^2, sum L_i, V, sum U_i
    for (int i = walker_tid<NT>(); i < n; i += NT) {
        const T xi = sx[i], yi = sy[i], zi = sz[i];
        double gx = 0, gy = 0, gz = 0, ui = 0;
        double lh = 0, vh = 0;   // offsets below n/2
        double lm = 0, vm = 0;   // offset n/2
        // partner j = i + k (mod n); its coordinates are loaded one step ahead
        int j = (i + 1 == n) ? 0 : i + 1;
        T xj = sx[j], yj = sy[j], zj = sz[j];
#pragma unroll 2
        for (int k = 1; k <= half; ++k) {
            const int jn = (j + 1 == n) ? 0 : j + 1;
            const T xq = sx[jn], yq = sy[jn], zq = sz[jn];
            const T dx = min_image(xi - xj, p);
            const T dy = min_image(yi - yj, p);
            const T dz = min_image(zi - zj, p);
            ETerms e;
            pair_energy(p, dx * dx + dy * dy + dz * dz, e);
            gx += e.dur * (double)dx;
            gy += e.dur * (double)dy;
            gz += e.dur * (double)dz;
            ui += e.u;
            lh += e.lap;
            vh += e.v;
            if (HIST && pair_inside(p, dx * dx + dy * dy + dz * dz))
                atomicAdd(&hist[min(nb - 1, (int)(e.r * bin_scale))], 1u);
            j = jn;
            xj = xq;
            yj = yq;
            zj = zq;
        }
        if (mid) {
            const int jn = (j + 1 == n) ? 0 : j + 1;
            const T dx = min_image(xi - xj, p);
            const T dy = min_image(yi - yj, p);
            const T dz = min_image(zi - zj, p);
            ETerms e;
            pair_energy(p, dx * dx + dy * dy + dz * dz, e);
            gx += e.dur * (double)dx;
            gy += e.dur * (double)dy;
            gz += e.dur * (double)dz;
            ui += e.u;
            lm = e.lap;
            vm = e.v;
            // the antipodal pair is met from both atoms: count it from the lower slot
            if (HIST && i < j && pair_inside(p, dx * dx + dy * dy + dz * dz))
                atomicAdd(&hist[min(nb - 1, (int)(e.r * bin_scale))], 1u);
            j = jn;
            xj = sx[j];
            yj = sy[j];
            zj = sz[j];
        }
#pragma unroll 2
        for (int k = half + 1 + (mid ? 1 : 0); k < n; ++k) {
            const int jn = (j + 1 == n) ? 0 : j + 1;
            const T xq = sx[jn], yq = sy[jn], zq = sz[jn];
            const T dx = min_image(xi - xj, p);
            const T dy = min_image(yi - yj, p);
            const T dz = min_image(zi - zj, p);
            double u, dur;
            pair_grad_u(p, dx * dx + dy * dy + dz * dz, u, dur);
            gx += dur * (double)dx;
            gy += dur * (double)dy;
            gz += dur * (double)dz;
            ui += u;
            j = jn;
            xj = xq;
            yj = yq;
            zj = zq;
        }
        acc[0] += gx * gx + gy * gy + gz * gz;
        acc[1] += fma(2.0, lh, lm);
        acc[2] += fma(0.5, vm, vh);
        acc[3] += ui;
        if (rows)
            rows[i] = ui;
    }
    block_sum<NT, 4>(acc, buf);
    const double V = acc[2], U = 0.5 * acc[3];
    const double tpb = -p.kappa * (acc[1] + acc[0]);
    out[0] = V + tpb;
    out[1] = V;
    out[2] = tpb;
    out[3] = -0.5 * p.kappa * acc[1];
    out[4] = p.kappa * acc[0];
    out[5] = U;
}

// Row sums rows[i] = sum_{j != i} u(r_ij) of the lane's atoms.
// Row sum R_i = sum over j != i of u(r_ij), from the coordinates in LDS.
template <typename T>
__device__ double row_of(const KParams &p, const T *sx, const T *sy, const T *sz, int i)
{
    const int n = p.n;
    const T xi = sx[i], yi = sy[i], zi = sz[i];
    double ui = 0.0;
    for (int j = 0; j < n; ++j) {
        const T dx = image_len(xi - sx[j], p);
        const T dy = image_len(yi - sy[j], p);
        const T dz = image_len(zi - sz[j], p);
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T u = pair_u_ri(p, r2, inv_sqrt(r2));
        ui += (j == i) ? 0.0 : (double)u;
    }
    return ui;
}

template <typename T, int NT>
__device__ void row_pass(const KParams &p, const T *sx, const T *sy, const T *sz, double *rows)
{
    for (int i = walker_tid<NT>(); i < p.n; i += NT)
        rows[i] = row_of(p, sx, sy, sz, i);
}

// Element q of a register array, q wave-uniform: a chain of uniform branches
// (the empty volatile asm keeps each one a branch rather than a select), so
// one element moves instead of every element being selected over.
template <int Q, int K>
__device__ __forceinline__ double reg_get(const double (&a)[K], int q)
{
    if constexpr (Q == K) {
        return 0.0;
    } else {
        if (q == Q) {
            asm volatile("");
            return a[Q];
        }
        return reg_get<Q + 1, K>(a, q);
    }
}

template <int Q, int K>
__device__ __forceinline__ void reg_set(double (&a)[K], int q, double v)
{
    if constexpr (Q < K) {
        if (q == Q) {
            asm volatile("");
            a[Q] = v;
            return;
        }
        reg_set<Q + 1, K>(a, q, v);
    }
}

// Lane partial of the Eq. (7) sums for moving atom s from (ox,oy,oz) to
// (nx,ny,nz): sum over this lane's atoms i != s of u(new) - u(old), V(new) - V(old).
template <typename T, int NT>
__device__ __forceinline__ void move_partial(const KParams &p, const T *sx, const T *sy, const T *sz,
                                             int s, T ox, T oy, T oz, T nx, T ny, T nz,
                                             double &du, double &dv)
{
    const int n = p.n;
    for (int i = walker_tid<NT>(); i < n; i += NT) {
        const T xi = sx[i], yi = sy[i], zi = sz[i];
        const T ax = image_len(ox - xi, p), ay = image_len(oy - yi, p), az_ = image_len(oz - zi, p);
        const T bx = image_len(nx - xi, p), by = image_len(ny - yi, p), bz = image_len(nz - zi, p);
        const T r2o = ax * ax + ay * ay + az_ * az_;
        const T r2n = bx * bx + by * by + bz * bz;
        T uo, vo, un, vn;
        pair_uv2(p, r2o, r2n, uo, vo, un, vn);
        const bool self = (i == s);
        du += self ? 0.0 : (double)(un - uo);
        dv += self ? 0.0 : (double)(vn - vo);
    }
}

template <typename T>
__device__ __forceinline__ T dist2(const KParams &p, T ax, T ay, T az_, T bx, T by, T bz)
{
    const T dx = image_len(ax - bx, p), dy = image_len(ay - by, p), dz = image_len(az_ - bz, p);
    return dx * dx + dy * dy + dz * dz;
}

// fcc start of walker wid with deterministic jitter (see hevmc_init_walkers).
template <typename T>
__device__ void fcc_site(const KParams &p, uint32_t wid, int pidx, int nc, double a, T *x, T *y, T *z)
{
    const int beta = pidx & 3, cell = pidx >> 2;
    const int iz = cell % nc, iy = (cell / nc) % nc, ix = cell / (nc * nc);
    const double bx = (beta == 2 || beta == 3) ? 0.5 : 0.0;
    const double by = (beta == 1 || beta == 3) ? 0.5 : 0.0;
    const double bz = (beta == 1 || beta == 2) ? 0.5 : 0.0;
    uint32_t r[4];
    philox4x32_10((uint32_t)pidx, 0xFFFFFFFFu, wid, 2u, p.key0, p.key1, r);
    const double px = a * ((double)ix + bx + 0.25) + 1e-3 * a * (unit32(r[0]) - 0.5);
    const double py = a * ((double)iy + by + 0.25) + 1e-3 * a * (unit32(r[1]) - 0.5);
    const double pz = a * ((double)iz + bz + 0.25) + 1e-3 * a * (unit32(r[2]) - 0.5);
    *x = (T)px; *y = (T)py; *z = (T)pz;
}

// --------------------------------------------------------------------------
// Morton code of the cell (kSortCells per side) that holds a position in [0, L).
template <typename T>
__device__ __forceinline__ uint32_t morton_cell(const KParams &p, T x, T y, T z)
{
    const double s = (double)kSortCells * p.invL;
    const uint32_t cx = (uint32_t)min(kSortCells - 1, max(0, (int)((double)x * s)));
    const uint32_t cy = (uint32_t)min(kSortCells - 1, max(0, (int)((double)y * s)));
    const uint32_t cz = (uint32_t)min(kSortCells - 1, max(0, (int)((double)z * s)));
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        m |= (((cx >> b) & 1u) << (3 * b)) | (((cy >> b) & 1u) << (3 * b + 1)) | (((cz >> b) & 1u) << (3 * b + 2));
    return m;
}

// Puts a walker's atoms in LDS into the spatial order of their cells' Morton
// codes, ties by label: keys are rebuilt from the current positions, sorted by
// a bitonic network (pk keys, a power of two) and the coordinates (and rows)
// are permuted through registers.  The order depends only on the positions,
// so a run gives the same bits however it is split into launches.  Requires
// n <= 8 NT.  Walker-wide: every thread of the walker must call it.
template <typename T, int NT, bool ROWS>
__device__ void walker_resort(const KParams &p, T *sx, T *sy, T *sz, double *ru, uint32_t *key,
                              uint16_t *slot_of)
{
    const int n = p.n, pk = sort_keys(n), tid = walker_tid<NT>();
    walker_sync<NT>();
    for (int q = tid; q < pk; q += NT)
        key[q] = q < n ? (morton_cell(p, sx[q], sy[q], sz[q]) << 16) | (key[q] & 0xFFFFu) : 0xFFFFFFFFu;
    walker_sync<NT>();
    for (int k = 2; k <= pk; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < (pk >> 1); i += NT) {
                const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1)), hi = lo + j;
                const uint32_t a = key[lo], b = key[hi];
                if ((a > b) == ((lo & k) == 0)) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            walker_sync<NT>();
        }
    }
    T gx[kRowsPerLane], gy[kRowsPerLane], gz[kRowsPerLane];
    double gr[kRowsPerLane];
#pragma unroll
    for (int c = 0; c < kRowsPerLane; ++c) {
        const int q = tid + c * NT;
        if (q < n) {
            const int o = slot_of[key[q] & 0xFFFFu];
            gx[c] = sx[o];
            gy[c] = sy[o];
            gz[c] = sz[o];
            gr[c] = ROWS ? ru[o] : 0.0;
        }
    }
    walker_sync<NT>();
#pragma unroll
    for (int c = 0; c < kRowsPerLane; ++c) {
        const int q = tid + c * NT;
        if (q < n) {
            sx[q] = gx[c];
            sy[q] = gy[c];
            sz[q] = gz[c];
            if (ROWS)
                ru[q] = gr[c];
            slot_of[key[q] & 0xFFFFu] = (uint16_t)q;
        }
    }
    walker_sync<NT>();
}

// One walker's sweeps (the body of the sweep kernels).  Dynamic LDS: x, y, z
// (T) and, for ROWS, the row sums (double) at rows_lds_offset(n, sizeof(T)).
// g: the walker's coordinates [3][N]; accp: its accumulators; rg: its row sums
// in HBM ([N] doubles) or null; grw: its pair histogram ([gr_bins], HIST
// only); trw: its per-sample records ([trace_cap][6]) or null; mlw: its
// per-move records ([log_cap][4]: atom label, accepted, dU, dV) or null.  For NT = 64 the walker is one wave and red, rsl, ebuf are not used.
// Two walkers that share a compute unit compete for its four SIMDs, and the
// hardware issues from the oldest ready wave first.  Left to that, the walker
// dispatched first finishes in about two thirds of the launch and its partner
// runs the rest alone, with no second wave per SIMD to cover its barrier and
// reduction latencies.  So every 64 moves thread 0 swaps its progress into its
// compute unit's word of cu_progress and reads back what was there.  If that
// came from the partner (same launch tag, other walker) and the partner is
// ahead, the walker raises its waves' issue priority for the next 64 moves;
// otherwise it lowers it.  Only the order in which waves issue changes, so
// every result is bitwise the same.
//   word: launch tag (24 bits) | walker id (16 bits) | 64-move blocks done (24 bits)
__device__ unsigned long long cu_progress[1024];

__device__ __forceinline__ int share_turn(uint32_t tag, uint32_t wid, uint32_t blk, uint32_t cu, int prev)
{
    const unsigned long long mine = ((unsigned long long)(tag & 0xFFFFFFu) << 40) |
                                    ((unsigned long long)(wid & 0xFFFFu) << 24) | (blk & 0xFFFFFFu);
    const unsigned long long seen = atomicExch(&cu_progress[cu & 1023u], mine);
    if ((uint32_t)(seen >> 40) == (tag & 0xFFFFFFu) && (uint32_t)((seen >> 24) & 0xFFFFu) != (wid & 0xFFFFu))
        return (uint32_t)(seen & 0xFFFFFFu) > (blk & 0xFFFFFFu) ? 1 : 0;
    return prev;
}

// Rows in registers (RREG): the row-sum sweep for walkers whose rows do not
// fit in LDS beside the coordinates (N = 10976 in FP32 takes 131.7 KB of
// coordinates; its rows would need 87.8 KB more).  Lane tid keeps the rows of
// its atoms tid + q NT, q < kRegChunks, in registers; they are loaded from and
// stored to the HBM rows buffer at the launch's ends, and the moved atom's row
// reaches the other lanes through the same LDS slot as in the LDS form.  The
// passes read each partner's coordinates from LDS and keep no per-pair terms
// between the forward and the accept pass (they are recomputed, bitwise the
// same), so the registers go to the rows.
// (kRegChunks: hevmc_internal.hpp)
// the (precision, threads) instantiated with rows in registers
template <typename T, int NT>
constexpr bool kRregForm = std::is_same<T, float>::value && NT == 512;

template <typename T, int NT, bool ROWS, bool HIST = false, bool RREG = false>
__device__ __forceinline__ void sweep_walker(const KParams &p, uint32_t wid, T *__restrict__ g,
                                             hevmc_walker_acc *__restrict__ accp, double *__restrict__ rg,
                                             uint64_t *__restrict__ grw, double *__restrict__ trw,
                                             double *__restrict__ mlw,
                                             uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t m,
                                             unsigned char *smem_raw, double (*red)[NT / 64][2], double *rsl,
                                             double *ebuf, int *prio)
{
    constexpr int NW = NT / 64;
    T *sx = reinterpret_cast<T *>(smem_raw);
    const int n = p.n;
    T *sy = sx + n, *sz = sy + n;
    double *ru = reinterpret_cast<double *>(smem_raw + rows_lds_offset(n, sizeof(T)));
    const int tid = walker_tid<NT>(), lane = tid & 63, wave = tid >> 6;
    // spatial order (p.sorted): LDS slot q holds the atom labelled key[q] & 0xFFFF
    const bool sorted = NT > 64 && p.sorted != 0;
    static_assert(!RREG || ROWS, "rows in registers is a form of the row-sum sweep");
    constexpr bool LROWS = ROWS && !RREG;   // rows in LDS
    uint32_t *key = reinterpret_cast<uint32_t *>(smem_raw + sort_lds_offset(n, sizeof(T), LROWS));
    uint16_t *slot_of = reinterpret_cast<uint16_t *>(smem_raw + slot_of_lds_offset(n, sizeof(T), LROWS));
    if (sorted) {
        for (int q = tid; q < n; q += NT) {
            key[q] = (uint32_t)q;
            slot_of[q] = (uint16_t)q;
        }
    }
    // pair histogram of the samples (grw: this walker's [gr_bins] counts)
    const int nb = HIST ? p.gr_bins : 0;
    uint32_t *hist =
        HIST ? reinterpret_cast<uint32_t *>(smem_raw + hist_lds_offset(n, sizeof(T), LROWS, sorted)) : nullptr;

    bool bad = false;
    for (int i = tid; i < 3 * n; i += NT) {
        const T v = g[i];
        sx[i] = v;
        bad |= !isfinite((double)v);
    }
    // the accumulators stay in HBM: thread 0 adds to them at samples and at
    // the end of measured sweeps, so the move loop holds only the running
    // totals in registers
    double u_run = accp->u_run, v_run = accp->v_run;
    const int64_t samples0 = accp->n_samples;
    // a walker with a non-finite coordinate (whose pairs would silently drop
    // out of every sum) leaves the launch with NaN running totals, which the
    // caller detects
    const bool bad_walker = walker_any<NT>(bad, ebuf);
    int64_t n_acc = 0, n_try = 0, n_samp = 0, n_swm = 0;
    const int nch_all = (n + NT - 1) / NT;
    double rr[RREG ? kRegChunks : 1];
    if constexpr (RREG) {
        // rows from HBM if they agree with u_run (the same sum rule), else
        // recomputed; atoms past N in the last chunk hold zero
        bool valid = false;
        if (rg) {
            double c[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < kRegChunks; ++q) {
                const int i = tid + q * NT;
                rr[q] = (q < nch_all && i < n) ? rg[i] : 0.0;
                c[0] += rr[q];
                c[1] += fabs(rr[q]);
            }
            block_sum<NT, 2>(c, ebuf);
            valid = fabs(0.5 * c[0] - u_run) <= 1e-9 * (0.5 * c[1] + 1.0);
        }
        walker_sync<NT>();
        if (!valid) {
#pragma unroll
            for (int q = 0; q < kRegChunks; ++q) {
                const int i = tid + q * NT;
                rr[q] = (q < nch_all && i < n) ? row_of(p, sx, sy, sz, i) : 0.0;
            }
        }
    } else if constexpr (ROWS) {
        bool valid = false;
        if (rg) {
            double c[2] = {0.0, 0.0};
            for (int i = tid; i < n; i += NT) {
                const double r = rg[i];
                ru[i] = r;
                c[0] += r;
                c[1] += fabs(r);
            }
            block_sum<NT, 2>(c, ebuf);
            valid = fabs(0.5 * c[0] - u_run) <= 1e-9 * (0.5 * c[1] + 1.0);
        }
        walker_sync<NT>();
        if (!valid)
            row_pass<T, NT>(p, sx, sy, sz, ru);
    } else {
        walker_sync<NT>();
    }

    // row-sum passes: kRowsPerLane when every lane owns that many atoms; 1, 2
    // or 4 when at most that many chunks of NT atoms cover N (the last one
    // partial: its idle lanes re-read atom N-1 and count nothing); 0 otherwise.
    // The first four have no per-lane branch, so their LDS loads issue up front.
    // The few-chunk forms are compiled only for walkers of at most 128 threads
    // (small N): in the large-walker kernels their registers would crowd the
    // eight-chunk form, which then spills.
    constexpr bool kFewChunkModes = NT <= 128;
    // atoms per group of the FP64 row-sum accept pass (1: no grouping); more
    // than these make the kernels spill
    constexpr int kAcceptGroup = NT == 256 ? 4 : NT == 512 ? 2 : 1;
    const int nchunks = (n + NT - 1) / NT;
    const int lane_mode = n == kRowsPerLane * NT ? kRowsPerLane
                          : nchunks <= 1       ? 1
                          : nchunks <= 2       ? 2
                          : nchunks <= 4       ? 4
                                               : 0;
    // Register copies of the lane's own atoms (FULL lanes of multi-wave row-sum
    // walkers): atom tid + jj NT's coordinates and row.  Only this thread ever
    // writes them in LDS between re-sorts and samples (it owns the atoms), so
    // the copies are refilled from LDS after each of those and kept in step
    // with every write in between; the pair passes then read no LDS.
    constexpr bool kCache = ROWS && NT >= 128 && sizeof(T) == 4;
    constexpr bool kCacheRow = kCache;
    const bool cached = kCache && lane_mode == kRowsPerLane;
    T cx[kRowsPerLane], cy[kRowsPerLane], cz[kRowsPerLane];
    double cr[kRowsPerLane];
    auto refill = [&]() {
#pragma unroll
        for (int jj = 0; jj < kRowsPerLane; ++jj) {
            const int i = tid + jj * NT;
            cx[jj] = sx[i];
            cy[jj] = sy[i];
            cz[jj] = sz[i];
            if constexpr (kCacheRow)
                cr[jj] = ru[i];
        }
    };
    int last_s = -1;          // atom accepted in the previous micro-update
    T lx = 0, ly = 0, lz = 0; // its new position (LDS copy not yet visible to all waves)
    double dv_pend = 0.0;     // ROWS: lane partial of dV of the last accepted move

    // issue priority against the walker sharing this compute unit (prio: two
    // flags in LDS, written by thread 0 for blocks of alternating parity)
    const bool share = NT > 64 && prio != nullptr && p.share_tag != 0;
    const uint32_t cu = share ? __smid() : 0u;
    const uint32_t nblk = (uint32_t)((n + 63) / 64);
    // micro-updates done in this launch: picks the reduction buffer, so that
    // consecutive micro-updates use different buffers across sweep ends too
    uint32_t mv = 0;
    // per-move record awaiting its dV (row-sum forms reduce an accepted move's
    // dV with the next micro-update), or -1
    int64_t log_pend = -1;
    for (int it = 0; it < nsw; ++it) {
        const uint32_t t = sweep0 + (uint32_t)it;
        const bool measured = t >= mstart;
        if (sorted) {
            walker_resort<T, NT, LROWS>(p, sx, sy, sz, ru, key, slot_of);
            last_s = -1;
        }
        if (kCache && cached && (sorted || it == 0))
            refill();
        for (int k0 = 0; k0 < n; k0 += 64) {
            if (share) {
                // a barrier of every move lies between a flag's write (block
                // blk - 1) and its reads here, and the next write to the same
                // flag (block blk + 1)
                const uint32_t blk = (uint32_t)it * nblk + (uint32_t)(k0 >> 6);
                const int mine = blk > 0 ? __builtin_amdgcn_readfirstlane(prio[(blk & 1u) ^ 1u]) : 0;
                if (mine)
                    __builtin_amdgcn_s_setprio(1);
                else
                    __builtin_amdgcn_s_setprio(0);
                if (tid == 0)
                    prio[blk & 1u] = share_turn(p.share_tag, wid, blk, cu, mine);
            }
            // lane l draws the random numbers of micro-step k0 + l; the atom's
            // label becomes its LDS slot
            int bs;
            double bxi, bdx, bdy, bdz;
            draw_move(p, (uint32_t)(k0 + lane), t, wid, bs, bxi, bdx, bdy, bdz);
            const double blx = log(bxi);   // ln xi of micro-step k0 + lane
            const int blab = bs;           // the atom's label (bs becomes its slot)
            if (sorted)
                bs = slot_of[bs];
            // Old and trial position of micro-step k0 + lane, taken here from
            // the positions in LDS, off the moves' critical path.  A lane's
            // pair goes stale when its atom is moved by an accepted earlier
            // micro-update of the batch (bit `lane` of `stale`), or is the
            // atom accepted just before the batch, whose new LDS copy other
            // waves may not see yet; a stale micro-step forms both positions
            // again when it runs, from the forwarded copy or from LDS.
            const T box = sx[bs], boy = sy[bs], boz = sz[bs];
            const T bnx = trial_coord<T>((double)box + bdx, p);
            const T bny = trial_coord<T>((double)boy + bdy, p);
            const T bnz = trial_coord<T>((double)boz + bdz, p);
            uint64_t stale = last_s >= 0 ? __builtin_amdgcn_ballot_w64(bs == last_s) : 0ull;
            const int kend = min(64, n - k0);
            for (int j = 0; j < kend; ++j) {
                const int k = k0 + j;
                const uint32_t par = mv & 1u;
                ++mv;
                const int64_t q_log = (int64_t)it * n + k;   // this micro-update's record
                const int s = readlane_i(bs, j);
                const double lxi = lane_value(blx, j);
                T ox, oy, oz, nx, ny, nz;
                if ((stale >> j) & 1ull) {
                    if (s == last_s) {
                        ox = lx; oy = ly; oz = lz;
                    } else {
                        ox = sx[s]; oy = sy[s]; oz = sz[s];
                    }
                    nx = trial_coord<T>((double)ox + lane_value(bdx, j), p);
                    ny = trial_coord<T>((double)oy + lane_value(bdy, j), p);
                    nz = trial_coord<T>((double)oz + lane_value(bdz, j), p);
                } else {
                    ox = lane_value(box, j); oy = lane_value(boy, j); oz = lane_value(boz, j);
                    nx = lane_value(bnx, j); ny = lane_value(bny, j); nz = lane_value(bnz, j);
                }
                // the later micro-steps of the batch that move atom s (called
                // after an accepted micro-update of atom s)
                auto mark_stale = [&]() {
                    const uint64_t later = j >= 63 ? 0ull : (~0ull << (j + 1));
                    stale |= __builtin_amdgcn_ballot_w64(bs == s) & later;
                };
                const bool owner = (tid == s % NT);
                // the record of this micro-update (label, decision, dU; dV when known)
                auto log_move = [&](bool acc_, double du_, double dv_) {
                    if (mlw && tid == 0 && q_log < p.log_cap) {
                        double *rec = mlw + 4 * q_log;
                        rec[0] = (double)readlane_i(blab, j);
                        rec[1] = acc_ ? 1.0 : 0.0;
                        rec[2] = du_;
                        rec[3] = dv_;
                    }
                };
                // the dV of the previous accepted micro-update (row-sum forms)
                auto log_pending_dv = [&](double dv_) {
                    if (mlw && tid == 0 && log_pend >= 0)
                        mlw[4 * log_pend + 3] = dv_;
                    log_pend = -1;
                };
                if constexpr (RREG) {
                    // forward half: u at the new position over the lane's atoms
                    // (the rows are not touched, so this loop needs no unrolling)
                    double su = 0.0;
#pragma unroll 2
                    for (int i = tid; i < n; i += NT) {
                        const T r2 = dist2(p, nx, ny, nz, sx[i], sy[i], sz[i]);
                        su += (double)pair_u_in(p, r2, inv_sqrt(r2), i != s);
                    }
                    const double w0 = wave_sum(su);
                    const double w1 = (last_s >= 0) ? wave_sum(dv_pend) : 0.0;
                    const int js = s / NT;
                    const double rs_own = reg_get<0, kRegChunks>(rr, js);
                    double SU = 0.0, DVP = 0.0;
                    if (lane == 0) {
                        red[par][wave][0] = w0;
                        red[par][wave][1] = w1;
                    }
                    if (owner)
                        rsl[par] = rs_own;
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        SU += red[par][q][0];
                        DVP += red[par][q][1];
                    }
                    const double RS = rsl[par];
                    v_run += DVP;
                    dv_pend = 0.0;
                    const double DU = SU - RS;
                    const bool accept = metropolis_accept_log(DU, lxi);
                    log_pending_dv(DVP);
                    log_move(accept, DU, __builtin_nan(""));
                    if (accept && q_log < p.log_cap)
                        log_pend = q_log;
                    if (measured) {
                        n_try += 1;
                        n_acc += accept ? 1 : 0;
                    }
                    if (accept) {
                        u_run += DU;
                        // old- and new-position terms (the new ones recomputed
                        // from the same operands as the forward half): rows, dV
                        double dvl = 0.0;
#pragma unroll
                        for (int q = 0; q < kRegChunks; ++q) {
                            if (q < nch_all) {
                                // keeps the next chunk's loads from being hoisted
                                // over this one (their registers would spill)
                                asm volatile("" ::: "memory");
                                const int i = tid + q * NT;
                                const bool live = i < n;
                                const int ic = live ? i : n - 1;
                                const T xi = sx[ic], yi = sy[ic], zi = sz[ic];
                                const T r2o = dist2(p, ox, oy, oz, xi, yi, zi);
                                const T r2n = dist2(p, nx, ny, nz, xi, yi, zi);
                                const T rio = inv_sqrt(r2o), rin = inv_sqrt(r2n);
                                const T uo = pair_u_ri(p, r2o, rio), un = pair_u_ri(p, r2n, rin);
                                T vo, vn;
                                pair_v_ri2(p, r2o, rio, r2n, rin, vo, vn);
                                const bool other = live && i != s;
                                rr[q] += other ? (double)un - (double)uo : 0.0;
                                dvl += other ? (double)vn - (double)vo : 0.0;
                            }
                        }
                        dv_pend = dvl;
                        if (owner) {
                            sx[s] = nx; sy[s] = ny; sz[s] = nz;
                            reg_set<0, kRegChunks>(rr, js, SU);
                        }
                        last_s = s;
                        mark_stale();
                        lx = nx; ly = ny; lz = nz;
                    } else {
                        last_s = -1;
                    }
                } else if constexpr (ROWS) {
                    // forward half: u at the new position only; r^2 and 1/r are
                    // kept for the potential if the move is accepted
                    double su = 0.0;
                    T un_[kRowsPerLane], r2n_[kRowsPerLane], rin_[kRowsPerLane];
                    // FULL: every lane owns kRowsPerLane atoms, so the unrolled
                    // body has no per-lane branch and its loads issue up front
                    auto forward = [&](auto mode_c) {
                        constexpr int MODE = decltype(mode_c)::value;
                        constexpr int CH = MODE == 0 ? kRowsPerLane : MODE;
#pragma unroll
                        for (int jj = 0; jj < CH; ++jj) {
                            const int i = tid + jj * NT;
                            T uu = T(0), r2 = T(1), ri = T(1);
                            if constexpr (MODE == 0) {
                                if (i < n) {
                                    r2 = dist2(p, nx, ny, nz, sx[i], sy[i], sz[i]);
                                    ri = inv_sqrt(r2);
                                    uu = pair_u_in(p, r2, ri, i != s);
                                }
                            } else if constexpr (kCache && MODE == kRowsPerLane) {
                                r2 = dist2(p, nx, ny, nz, cx[jj], cy[jj], cz[jj]);
                                ri = inv_sqrt(r2);
                                uu = pair_u_in(p, r2, ri, i != s);
                            } else {
                                const bool live = MODE == kRowsPerLane || i < n;
                                const int ic = MODE == kRowsPerLane ? i : min(i, n - 1);
                                r2 = dist2(p, nx, ny, nz, sx[ic], sy[ic], sz[ic]);
                                ri = inv_sqrt(r2);
                                uu = pair_u_in(p, r2, ri, live && i != s);
                            }
                            un_[jj] = uu;
                            r2n_[jj] = r2;
                            rin_[jj] = ri;
                            su += (double)uu;
                        }
                    };
                    if constexpr (kFewChunkModes) {
                        switch (lane_mode) {
                        case kRowsPerLane: forward(std::integral_constant<int, kRowsPerLane>{}); break;
                        case 4: forward(std::integral_constant<int, 4>{}); break;
                        case 2: forward(std::integral_constant<int, 2>{}); break;
                        case 1: forward(std::integral_constant<int, 1>{}); break;
                        default: forward(std::integral_constant<int, 0>{}); break;
                        }
                    } else {
                        if (lane_mode == kRowsPerLane)
                            forward(std::integral_constant<int, kRowsPerLane>{});
                        else
                            forward(std::integral_constant<int, 0>{});
                    }
                    const double w0 = wave_sum(su);
                    const double w1 = (last_s >= 0) ? wave_sum(dv_pend) : 0.0;
                    double SU = 0.0, DVP = 0.0, RS;
                    if constexpr (NW == 1) {
                        // one wave per walker: the butterfly already gave every
                        // lane the totals, and the owner's row is visible in-wave
                        SU = w0;
                        DVP = w1;
                        RS = ru[s];
                    } else {
                        if (lane == 0) {
                            red[par][wave][0] = w0;
                            red[par][wave][1] = w1;
                        }
                        if (owner)
                            rsl[par] = ru[s];
                        __syncthreads();
#pragma unroll
                        for (int q = 0; q < NW; ++q) {
                            SU += red[par][q][0];
                            DVP += red[par][q][1];
                        }
                        RS = rsl[par];
                    }
                    v_run += DVP;
                    dv_pend = 0.0;
                    const double DU = SU - RS;
                    const bool accept = metropolis_accept_log(DU, lxi);
                    log_pending_dv(DVP);
                    log_move(accept, DU, __builtin_nan(""));
                    if (accept && q_log < p.log_cap)
                        log_pend = q_log;
                    if (measured) {
                        n_try += 1;
                        n_acc += accept ? 1 : 0;
                    }
                    if (accept) {
                        u_run += DU;
                        // old-position terms: update the rows, form dV
                        double dvl = 0.0;
                        auto accept_pass = [&](auto mode_c) {
                            constexpr int MODE = decltype(mode_c)::value;
                            constexpr int CH = MODE == 0 ? kRowsPerLane : MODE;
                            if constexpr (sizeof(T) == 8 && kAcceptGroup > 1 && MODE == kRowsPerLane && CH % kAcceptGroup == 0) {
                                // FP64, every lane owning CH atoms: kAcceptGroup atoms at
                                // a time, their branch-free arithmetic interleaved around
                                // the exponentials' branches (same values, same order)
#pragma unroll
                                for (int j0 = 0; j0 < CH; j0 += kAcceptGroup) {
                                    double r2o[kAcceptGroup], uo[kAcceptGroup];
                                    VPair vp[kAcceptGroup];
#pragma unroll
                                    for (int g = 0; g < kAcceptGroup; ++g) {
                                        const int i = tid + (j0 + g) * NT;
                                        r2o[g] = dist2(p, ox, oy, oz, sx[i], sy[i], sz[i]);
                                        const double rio = inv_sqrt(r2o[g]);
                                        uo[g] = pair_u_ri(p, r2o[g], rio);
                                        vp_pre(p, r2o[g], rio, r2n_[j0 + g], rin_[j0 + g], vp[g]);
                                    }
#pragma unroll
                                    for (int g = 0; g < kAcceptGroup; ++g)
                                        vp_exp(p, vp[g]);
#pragma unroll
                                    for (int g = 0; g < kAcceptGroup; ++g) {
                                        const int i = tid + (j0 + g) * NT;
                                        double vo, vn;
                                        vp_post(vp[g], vo, vn);
                                        const bool other = i != s;
                                        ru[i] += keep_or_tiny(other, (double)un_[j0 + g] - uo[g]);
                                        dvl += keep_or_tiny(other, vn - vo);
                                    }
                                }
                                return;
                            }
#pragma unroll
                            for (int jj = 0; jj < CH; ++jj) {
                                const int i = tid + jj * NT;
                                const bool live = MODE == kRowsPerLane || i < n;
                                if (MODE != 0 || live) {
                                    const int ic = (MODE == 0 || MODE == kRowsPerLane) ? i : min(i, n - 1);
                                    constexpr bool kReg = kCache && MODE == kRowsPerLane;
                                    const T r2o = kReg ? dist2(p, ox, oy, oz, cx[jj], cy[jj], cz[jj])
                                                       : dist2(p, ox, oy, oz, sx[ic], sy[ic], sz[ic]);
                                    const T rio = inv_sqrt(r2o);
                                    const T uo = pair_u_ri(p, r2o, rio);
                                    T vo, vn;
                                    pair_v_ri2(p, r2o, rio, r2n_[jj], rin_[jj], vo, vn);
                                    const bool other = live && (i != s);
                                    const double dr = keep_or_tiny(other, (double)un_[jj] - (double)uo);
                                    if constexpr (kReg && kCacheRow) {
                                        cr[jj] += dr;
                                        ru[i] = cr[jj];
                                    } else if (live) {
                                        ru[i] += dr;
                                    }
                                    dvl += keep_or_tiny(other, (double)vn - (double)vo);
                                }
                            }
                        };
                        if constexpr (kFewChunkModes) {
                            switch (lane_mode) {
                            case kRowsPerLane: accept_pass(std::integral_constant<int, kRowsPerLane>{}); break;
                            case 4: accept_pass(std::integral_constant<int, 4>{}); break;
                            case 2: accept_pass(std::integral_constant<int, 2>{}); break;
                            case 1: accept_pass(std::integral_constant<int, 1>{}); break;
                            default: accept_pass(std::integral_constant<int, 0>{}); break;
                            }
                        } else {
                            if (lane_mode == kRowsPerLane)
                                accept_pass(std::integral_constant<int, kRowsPerLane>{});
                            else
                                accept_pass(std::integral_constant<int, 0>{});
                        }
                        dv_pend = dvl;
                        if (owner) {
                            sx[s] = nx; sy[s] = ny; sz[s] = nz;
                            ru[s] = SU;
                            if (kCache && cached) {
                                const int js = s / NT;
#pragma unroll
                                for (int jj = 0; jj < kRowsPerLane; ++jj)
                                    if (jj == js) {
                                        cx[jj] = nx; cy[jj] = ny; cz[jj] = nz;
                                        if constexpr (kCacheRow)
                                            cr[jj] = SU;
                                    }
                            }
                        }
                        last_s = s;
                        mark_stale();
                        lx = nx; ly = ny; lz = nz;
                    } else {
                        last_s = -1;
                    }
                } else {
                    double du = 0.0, dv = 0.0;
                    move_partial<T, NT>(p, sx, sy, sz, s, ox, oy, oz, nx, ny, nz, du, dv);
                    du = wave_sum(du);
                    dv = wave_sum(dv);
                    double DU = 0.0, DV = 0.0;
                    if constexpr (NW == 1) {
                        DU = du;
                        DV = dv;
                    } else {
                        if (lane == 0) {
                            red[par][wave][0] = du;
                            red[par][wave][1] = dv;
                        }
                        __syncthreads();
#pragma unroll
                        for (int q = 0; q < NW; ++q) {
                            DU += red[par][q][0];
                            DV += red[par][q][1];
                        }
                    }
                    const bool accept = metropolis_accept_log(DU, lxi);
                    log_move(accept, DU, DV);
                    if (measured) {
                        n_try += 1;
                        n_acc += accept ? 1 : 0;
                    }
                    if (accept) {
                        u_run += DU;
                        v_run += DV;
                        if (owner) {
                            sx[s] = nx; sy[s] = ny; sz[s] = nz;
                        }
                        last_s = s;
                        mark_stale();
                        lx = nx; ly = ny; lz = nz;
                    } else {
                        last_s = -1;
                    }
                }
            }
        }
        if constexpr (ROWS) {
            // the last accepted move's dV has not been reduced yet
            double f[1] = {dv_pend};
            block_sum<NT, 1>(f, ebuf);
            v_run += f[0];
            dv_pend = 0.0;
            if (mlw && tid == 0 && log_pend >= 0)
                mlw[4 * log_pend + 3] = f[0];
            log_pend = -1;
        }
        if (measured) {
            if (m > 0 && (t - mstart + 1) % (uint32_t)m == 0) {
                if constexpr (HIST)
                    for (int b = tid; b < nb; b += NT)
                        hist[b] = 0u;
                walker_sync<NT>();
                double el[6];
                local_energy_pass<T, NT, HIST>(p, sx, sy, sz, ebuf, el, LROWS ? ru : nullptr, hist, nb);
                if (kCache && cached)
                    refill();   // the pass rewrote this thread's rows
                if constexpr (HIST) {
                    walker_sync<NT>();
                    for (int b = tid; b < nb; b += NT)
                        grw[b] += hist[b];
                }
                if (trw && tid < 6) {
                    // the sample's record: (E_L, V, T_PB, T_JF, T_F, U), at its
                    // index among all of the walker's samples
                    const int64_t idx = samples0 + n_samp;
                    if (idx < (int64_t)p.trace_cap)
                        trw[(size_t)idx * 6 + tid] = el[tid];
                }
                if (tid == 0) {
                    nsum(accp->sum_e, accp->c_e, el[0]);
                    nsum(accp->sum_e2, accp->c_e2, el[0] * el[0]);
                    nsum(accp->sum_v, accp->c_v, el[1]);
                    nsum(accp->sum_tpb, accp->c_tpb, el[2]);
                    nsum(accp->sum_tjf, accp->c_tjf, el[3]);
                    nsum(accp->sum_tf, accp->c_tf, el[4]);
                }
                n_samp += 1;
                u_run = el[5];
                v_run = el[1];
                last_s = -1;
            }
            if (tid == 0)
                nsum(accp->sum_vs, accp->c_vs, v_run);
            n_swm += 1;
        }
    }
    walker_sync<NT>();
    if (sorted) {
        for (int q = tid; q < n; q += NT) {
            const int l = (int)(key[q] & 0xFFFFu);
            g[l] = sx[q];
            g[n + l] = sy[q];
            g[2 * n + l] = sz[q];
            if (LROWS && rg)
                rg[l] = ru[q];
        }
    } else {
        for (int i = tid; i < 3 * n; i += NT)
            g[i] = sx[i];
        if constexpr (RREG) {
            if (rg) {
#pragma unroll
                for (int q = 0; q < kRegChunks; ++q) {
                    const int i = tid + q * NT;
                    if (q < nch_all && i < n)
                        rg[i] = rr[q];
                }
            }
        } else if constexpr (ROWS) {
            if (rg)
                for (int i = tid; i < n; i += NT)
                    rg[i] = ru[i];
        }
    }
    if (tid == 0) {
        accp->u_run = bad_walker ? __builtin_nan("") : u_run;
        accp->v_run = bad_walker ? __builtin_nan("") : v_run;
        accp->n_samples += n_samp;
        accp->n_sweeps_meas += n_swm;
        accp->n_acc += n_acc;
        accp->n_try += n_try;
    }
}

// The sweep kernel (hevmc_sweep; HIST: hevmc_sweep_gr).  Grid: one workgroup of
// NT threads per walker.
template <typename T, int NT, bool ROWS, bool HIST, bool RREG = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_sweep(KParams p, T *__restrict__ coords,
                                              hevmc_walker_acc *__restrict__ accs,
                                              double *__restrict__ rows_hbm, uint32_t sweep0, int32_t nsw,
                                              uint32_t mstart, int32_t m)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][NT / 64][2];
    __shared__ double rsl[2];
    __shared__ double ebuf[NT / 64 * 4];
    __shared__ int prio[2];
    const int w = blockIdx.x;
    const size_t n = (size_t)p.n;
    sweep_walker<T, NT, ROWS, HIST, RREG>(p, p.wid_base + (uint32_t)w, coords + (size_t)w * 3 * n, accs + w,
                                          rows_hbm ? rows_hbm + (size_t)w * n : nullptr,
                                          HIST ? p.gr + (size_t)w * (size_t)p.gr_bins : nullptr,
                                          p.trace ? p.trace + (size_t)w * (size_t)p.trace_cap * 6 : nullptr,
                                          (p.movelog && w < p.log_walkers)
                                              ? p.movelog + (size_t)w * (size_t)p.log_cap * 4
                                              : nullptr,
                                          sweep0, nsw, mstart, m, smem_raw, red, rsl, ebuf, prio);
}

// The batched sweep kernel (hevmc_sweep_batch): walker slots of several
// requests with the same N and precision in one grid.  map[2w] is the slot's
// request (or -1 for a free slot, which does nothing), map[2w+1] its Philox
// walker id; each request's constants and sweep counters come from the
// kernel arguments.
template <typename T, int NT, bool ROWS>
__global__ __launch_bounds__(NT) void k_sweep_batch(BatchArgs b, const int32_t *__restrict__ map,
                                                    T *__restrict__ coords, hevmc_walker_acc *__restrict__ accs,
                                                    double *__restrict__ rows_hbm, int32_t nsw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][NT / 64][2];
    __shared__ double rsl[2];
    __shared__ double ebuf[NT / 64 * 4];
    __shared__ int prio[2];
    const int w = blockIdx.x;
    const int r = map[2 * w];
    if (r < 0 || r >= b.count)
        return;
    const uint32_t wid = (uint32_t)map[2 * w + 1];
    const size_t n = (size_t)b.k[r].n;
    sweep_walker<T, NT, ROWS>(b.k[r], wid, coords + (size_t)w * 3 * n, accs + w,
                              rows_hbm ? rows_hbm + (size_t)w * n : nullptr, nullptr, nullptr, nullptr, b.sweep0[r],
                              nsw, b.mstart[r], b.m[r], smem_raw, red, rsl, ebuf, prio);
}

// One wave per walker, kWalkersPerGroup walkers per workgroup (small N): the
// walkers of a workgroup share nothing but the compute unit; each has its own
// LDS region of walker_lds bytes and never waits for the others.
template <typename T, bool ROWS, bool HIST>
__global__ __launch_bounds__(64 * kWalkersPerGroup) __attribute__((amdgpu_waves_per_eu(2))) void k_sweep_wave(KParams p, T *__restrict__ coords,
                                                                      hevmc_walker_acc *__restrict__ accs,
                                                                      double *__restrict__ rows_hbm, int32_t W,
                                                                      uint32_t walker_lds, uint32_t sweep0,
                                                                      int32_t nsw, uint32_t mstart, int32_t m)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = threadIdx.x >> 6;
    const int w = blockIdx.x * kWalkersPerGroup + wv;
    if (w >= W)
        return;
    const size_t n = (size_t)p.n;
    sweep_walker<T, 64, ROWS, HIST>(p, p.wid_base + (uint32_t)w, coords + (size_t)w * 3 * n, accs + w,
                                    rows_hbm ? rows_hbm + (size_t)w * n : nullptr,
                                    HIST ? p.gr + (size_t)w * (size_t)p.gr_bins : nullptr,
                                    p.trace ? p.trace + (size_t)w * (size_t)p.trace_cap * 6 : nullptr,
                                    (p.movelog && w < p.log_walkers)
                                        ? p.movelog + (size_t)w * (size_t)p.log_cap * 4
                                        : nullptr,
                                    sweep0, nsw, mstart, m, smem_raw + (size_t)wv * walker_lds, nullptr, nullptr,
                                    nullptr, nullptr);
}

template <typename T, bool ROWS>
__global__ __launch_bounds__(64 * kWalkersPerGroup) __attribute__((amdgpu_waves_per_eu(2))) void k_sweep_batch_wave(
    BatchArgs b, const int32_t *__restrict__ map, T *__restrict__ coords, hevmc_walker_acc *__restrict__ accs,
    double *__restrict__ rows_hbm, int32_t n_slots, uint32_t walker_lds, int32_t nsw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wv = threadIdx.x >> 6;
    const int w = blockIdx.x * kWalkersPerGroup + wv;
    if (w >= n_slots)
        return;
    const int r = map[2 * w];
    if (r < 0 || r >= b.count)
        return;
    const uint32_t wid = (uint32_t)map[2 * w + 1];
    const size_t n = (size_t)b.k[r].n;
    sweep_walker<T, 64, ROWS>(b.k[r], wid, coords + (size_t)w * 3 * n, accs + w,
                              rows_hbm ? rows_hbm + (size_t)w * n : nullptr, nullptr, nullptr, nullptr, b.sweep0[r],
                              nsw, b.mstart[r], b.m[r], smem_raw + (size_t)wv * walker_lds, nullptr, nullptr,
                              nullptr, nullptr);
}

// Pair distribution histograms of the W configurations (hevmc_pair_histogram):
// counts[w][b] for p.gr_bins bins over [0, L/2], through the local-energy pass
// that the sweep's samples use.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pair_hist(KParams p, const T *__restrict__ coords,
                                                  uint64_t *__restrict__ counts)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double ebuf[NW * 4];
    T *sx = reinterpret_cast<T *>(smem_raw);
    const int n = p.n, nb = p.gr_bins;
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem_raw + hist_lds_offset(n, sizeof(T), false, false));
    const T *g = coords + (size_t)blockIdx.x * 3 * (size_t)n;
    for (int i = threadIdx.x; i < 3 * n; i += NT)
        sx[i] = g[i];
    for (int b = threadIdx.x; b < nb; b += NT)
        hist[b] = 0u;
    __syncthreads();
    double el[6];
    local_energy_pass<T, NT, true>(p, sx, sx + n, sx + 2 * n, ebuf, el, nullptr, hist, nb);
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += NT)
        counts[(size_t)blockIdx.x * nb + b] = hist[b];
}

// Local energies of the W configurations (hevmc_local_energy).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_local_energy(KParams p, const T *__restrict__ coords,
                                                     double *__restrict__ out)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double ebuf[NW * 4];
    T *sx = reinterpret_cast<T *>(smem_raw);
    const int n = p.n;
    const T *g = coords + (size_t)blockIdx.x * 3 * (size_t)n;
    for (int i = threadIdx.x; i < 3 * n; i += NT)
        sx[i] = g[i];
    __syncthreads();
    double el[6];
    local_energy_pass<T, NT>(p, sx, sx + n, sx + 2 * n, ebuf, el, nullptr);
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q)
            out[(size_t)blockIdx.x * 6 + q] = el[q];
}

// Start walkers (hevmc_init_walkers): optional fcc start, then running totals
// (and row sums, if rows is not null) from a full evaluation, zeroed accumulators.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_init(KParams p, T *__restrict__ coords,
                                             hevmc_walker_acc *__restrict__ accs, double *__restrict__ rows,
                                             int fcc, int nc, double a_lat)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double ebuf[NW * 4];
    T *sx = reinterpret_cast<T *>(smem_raw);
    const int n = p.n;
    T *g = coords + (size_t)blockIdx.x * 3 * (size_t)n;
    const uint32_t wid = p.wid_base + blockIdx.x;
    // each thread checks the coordinates it stores itself (the others' stores
    // are visible only after the vote's barrier)
    bool bad = false;
    if (fcc) {
        for (int i = threadIdx.x; i < n; i += NT) {
            T x, y, z;
            fcc_site<T>(p, wid, i, nc, a_lat, &x, &y, &z);
            sx[i] = x; sx[n + i] = y; sx[2 * n + i] = z;
            g[i] = x; g[n + i] = y; g[2 * n + i] = z;
        }
    } else {
        for (int i = threadIdx.x; i < 3 * n; i += NT) {
            const T v = g[i];
            sx[i] = v;
            bad |= !isfinite((double)v);
        }
    }
    bad = walker_any<NT>(bad, ebuf);
    double el[6];
    local_energy_pass<T, NT>(p, sx, sx + n, sx + 2 * n, ebuf, el,
                             rows ? rows + (size_t)blockIdx.x * (size_t)n : nullptr);
    if (threadIdx.x == 0) {
        hevmc_walker_acc a = {};
        a.u_run = bad ? __builtin_nan("") : el[5];
        a.v_run = bad ? __builtin_nan("") : el[1];
        accs[blockIdx.x] = a;
    }
}

// Eq. (7) sums of one given trial move per walker (hevmc_move_delta).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_move_delta(KParams p, const T *__restrict__ coords,
                                                   const int32_t *__restrict__ s_in,
                                                   const double *__restrict__ delta,
                                                   double *__restrict__ out)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double ebuf[NW * 2];
    T *sx = reinterpret_cast<T *>(smem_raw);
    const int n = p.n;
    const int w = blockIdx.x;
    const T *g = coords + (size_t)w * 3 * (size_t)n;
    for (int i = threadIdx.x; i < 3 * n; i += NT)
        sx[i] = g[i];
    __syncthreads();
    const int s = s_in[w];
    if (s < 0 || s >= n) {   // invalid atom index: report NaN rather than read outside LDS
        if (threadIdx.x == 0) {
            out[2 * w + 0] = __builtin_nan("");
            out[2 * w + 1] = __builtin_nan("");
        }
        return;
    }
    const T ox = sx[s], oy = sx[n + s], oz = sx[2 * n + s];
    const T nx = trial_coord<T>((double)ox + delta[3 * w + 0], p);
    const T ny = trial_coord<T>((double)oy + delta[3 * w + 1], p);
    const T nz = trial_coord<T>((double)oz + delta[3 * w + 2], p);
    double v[2] = {0.0, 0.0};
    move_partial<T, NT>(p, sx, sx + n, sx + 2 * n, s, ox, oy, oz, nx, ny, nz, v[0], v[1]);
    // same reduction order as the plain sweep: wave butterfly, then waves in order
    block_sum<NT, 2>(v, ebuf);
    if (threadIdx.x == 0) {
        out[2 * w + 0] = v[0];
        out[2 * w + 1] = v[1];
    }
}

// Random numbers of sweep t (hevmc_draw_moves): one thread per (walker, k).
__global__ void k_draw_moves(KParams p, uint32_t t, int32_t *__restrict__ s_out,
                             double *__restrict__ xi_out, double *__restrict__ d_out, int total)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total)
        return;
    const int w = gid / p.n, k = gid % p.n;
    int s;
    double xi, dx, dy, dz;
    draw_move(p, (uint32_t)k, t, p.wid_base + (uint32_t)w, s, xi, dx, dy, dz);
    s_out[gid] = s;
    xi_out[gid] = xi;
    d_out[3 * (size_t)gid + 0] = dx;
    d_out[3 * (size_t)gid + 1] = dy;
    d_out[3 * (size_t)gid + 2] = dz;
}

// --------------------------------------------------------------------------
// Launchers.  The C ABI validated the arguments and planned the launch.

template <typename K>
static hipError_t allow_lds(K kern, size_t bytes)
{
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int NT, bool ROWS, bool HIST, bool RREG = false>
static hipError_t launch_sweep_v(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows,
                                 uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t m)
{
    if constexpr (NT == 64) {
        const int groups = (L.p.n_walkers_grid + kWalkersPerGroup - 1) / kWalkersPerGroup;
        auto kern = k_sweep_wave<T, ROWS, HIST>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(groups), dim3(64 * kWalkersPerGroup), L.lds_bytes, L.stream, L.k,
                           (T *)coords, acc, ROWS ? rows : (double *)nullptr, L.p.n_walkers_grid,
                           (uint32_t)L.walker_lds, sweep0, nsw, mstart, m);
    } else {
        auto kern = k_sweep<T, NT, ROWS, HIST, RREG>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(L.p.n_walkers_grid), dim3(NT), L.lds_bytes, L.stream, L.k, (T *)coords,
                           acc, ROWS ? rows : (double *)nullptr, sweep0, nsw, mstart, m);
    }
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_sweep_t(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows,
                                 uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t m)
{
    const bool hist = L.k.gr != nullptr && L.k.gr_bins > 0;
    if (L.rreg) {
        if constexpr (kRregForm<T, NT>)
            return hist ? launch_sweep_v<T, NT, true, true, true>(L, coords, acc, rows, sweep0, nsw, mstart, m)
                        : launch_sweep_v<T, NT, true, false, true>(L, coords, acc, rows, sweep0, nsw, mstart, m);
        return hipErrorInvalidValue;
    }
    if (L.rows)
        return hist ? launch_sweep_v<T, NT, true, true>(L, coords, acc, rows, sweep0, nsw, mstart, m)
                    : launch_sweep_v<T, NT, true, false>(L, coords, acc, rows, sweep0, nsw, mstart, m);
    return hist ? launch_sweep_v<T, NT, false, true>(L, coords, acc, rows, sweep0, nsw, mstart, m)
                : launch_sweep_v<T, NT, false, false>(L, coords, acc, rows, sweep0, nsw, mstart, m);
}

template <typename T, int NT>
static hipError_t launch_batch_t(const Launch &L, const BatchArgs &b, const int32_t *map, int32_t n_slots,
                                 void *coords, hevmc_walker_acc *acc, double *rows, int32_t nsw)
{
    if constexpr (NT == 64) {
        const int groups = (n_slots + kWalkersPerGroup - 1) / kWalkersPerGroup;
        const uint32_t wl = (uint32_t)L.walker_lds;
        if (L.rows) {
            auto kern = k_sweep_batch_wave<T, true>;
            hipError_t e = allow_lds(kern, L.lds_bytes);
            if (e != hipSuccess)
                return e;
            hipLaunchKernelGGL(kern, dim3(groups), dim3(64 * kWalkersPerGroup), L.lds_bytes, L.stream, b, map,
                               (T *)coords, acc, rows, n_slots, wl, nsw);
        } else {
            auto kern = k_sweep_batch_wave<T, false>;
            hipError_t e = allow_lds(kern, L.lds_bytes);
            if (e != hipSuccess)
                return e;
            hipLaunchKernelGGL(kern, dim3(groups), dim3(64 * kWalkersPerGroup), L.lds_bytes, L.stream, b, map,
                               (T *)coords, acc, (double *)nullptr, n_slots, wl, nsw);
        }
        return hipGetLastError();
    }
    if (L.rows) {
        auto kern = k_sweep_batch<T, NT, true>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(n_slots), dim3(NT), L.lds_bytes, L.stream, b, map, (T *)coords, acc, rows,
                           nsw);
    } else {
        auto kern = k_sweep_batch<T, NT, false>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(n_slots), dim3(NT), L.lds_bytes, L.stream, b, map, (T *)coords, acc,
                           (double *)nullptr, nsw);
    }
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_energy_t(const Launch &L, const void *coords, double *out)
{
    auto kern = k_local_energy<T, NT>;
    hipError_t e = allow_lds(kern, L.walker_lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(L.p.n_walkers_grid), dim3(NT), L.walker_lds, L.stream, L.k,
                       (const T *)coords, out);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_hist_t(const Launch &L, const void *coords, uint64_t *counts)
{
    auto kern = k_pair_hist<T, NT>;
    const size_t bytes = hist_lds_offset(L.k.n, sizeof(T), false, false) + (size_t)L.k.gr_bins * sizeof(uint32_t);
    hipError_t e = allow_lds(kern, bytes);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(L.p.n_walkers_grid), dim3(NT), bytes, L.stream, L.k, (const T *)coords, counts);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_init_t(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, int fcc,
                                int nc, double a_lat)
{
    auto kern = k_init<T, NT>;
    hipError_t e = allow_lds(kern, L.walker_lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(L.p.n_walkers_grid), dim3(NT), L.walker_lds, L.stream, L.k, (T *)coords, acc,
                       rows, fcc, nc, a_lat);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_delta_t(const Launch &L, const void *coords, const int32_t *s, const double *d,
                                 double *out)
{
    auto kern = k_move_delta<T, NT>;
    hipError_t e = allow_lds(kern, L.walker_lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(L.p.n_walkers_grid), dim3(NT), L.walker_lds, L.stream, L.k,
                       (const T *)coords, s, d, out);
    return hipGetLastError();
}

// Dispatch on (precision, threads per walker).
#define HEVMC_DISPATCH(FN, ...)                                                        \
    do {                                                                               \
        if (L.fp32) {                                                                  \
            switch (L.threads) {                                                       \
            case 64: return FN<float, 64>(L, __VA_ARGS__);                            \
            case 128: return FN<float, 128>(L, __VA_ARGS__);                          \
            case 256: return FN<float, 256>(L, __VA_ARGS__);                          \
            case 512: return FN<float, 512>(L, __VA_ARGS__);                          \
            case 1024: return FN<float, 1024>(L, __VA_ARGS__);                        \
            }                                                                          \
        } else {                                                                       \
            switch (L.threads) {                                                       \
            case 64: return FN<double, 64>(L, __VA_ARGS__);                           \
            case 128: return FN<double, 128>(L, __VA_ARGS__);                         \
            case 256: return FN<double, 256>(L, __VA_ARGS__);                         \
            case 512: return FN<double, 512>(L, __VA_ARGS__);                         \
            case 1024: return FN<double, 1024>(L, __VA_ARGS__);                       \
            }                                                                          \
        }                                                                              \
        return hipErrorInvalidValue;                                                   \
    } while (0)

template <typename T, int NT>
static const void *sweep_fn(bool rows, bool rreg)
{
    if constexpr (kRregForm<T, NT>)
        if (rreg)
            return (const void *)k_sweep<T, NT, true, false, true>;
    return rows ? (const void *)k_sweep<T, NT, true, false> : (const void *)k_sweep<T, NT, false, false>;
}

// Registers per thread and static LDS of the sweep kernel a launch would use
// (zeros if unknown).
static SweepAttrs sweep_attrs_query(bool fp32, int threads, bool rows, bool rreg);

SweepAttrs sweep_attrs(bool fp32, int threads, bool rows, bool rreg)
{
    // kernel attributes do not change: query each (precision, threads, form) once
    static std::atomic<int> vgprs[2][6][3], lds[2][6][3];
    static std::atomic<bool> have[2][6][3];
    const int t = threads == 64 ? 0 : threads == 128 ? 1 : threads == 256 ? 2 : threads == 512 ? 3 : threads == 1024 ? 4 : 5;
    const int v = rreg ? 2 : rows ? 1 : 0;
    if (have[fp32][t][v].load(std::memory_order_acquire))
        return SweepAttrs{vgprs[fp32][t][v].load(std::memory_order_relaxed),
                          lds[fp32][t][v].load(std::memory_order_relaxed)};
    const SweepAttrs a = sweep_attrs_query(fp32, threads, rows, rreg);
    vgprs[fp32][t][v].store(a.vgprs, std::memory_order_relaxed);
    lds[fp32][t][v].store(a.static_lds, std::memory_order_relaxed);
    have[fp32][t][v].store(true, std::memory_order_release);
    return a;
}

bool rreg_form(bool fp32, int threads) { return fp32 ? kRregForm<float, 512> && threads == 512 : false; }

static SweepAttrs sweep_attrs_query(bool fp32, int threads, bool rows, bool rreg)
{
    const void *f = nullptr;
    switch (threads) {
    case 64:
        f = fp32 ? (rows ? (const void *)k_sweep_wave<float, true, false> : (const void *)k_sweep_wave<float, false, false>)
                 : (rows ? (const void *)k_sweep_wave<double, true, false>
                         : (const void *)k_sweep_wave<double, false, false>);
        break;
    case 128: f = fp32 ? sweep_fn<float, 128>(rows, rreg) : sweep_fn<double, 128>(rows, rreg); break;
    case 256: f = fp32 ? sweep_fn<float, 256>(rows, rreg) : sweep_fn<double, 256>(rows, rreg); break;
    case 512: f = fp32 ? sweep_fn<float, 512>(rows, rreg) : sweep_fn<double, 512>(rows, rreg); break;
    case 1024: f = fp32 ? sweep_fn<float, 1024>(rows, rreg) : sweep_fn<double, 1024>(rows, rreg); break;
    default: return SweepAttrs{0, 0};
    }
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, f) != hipSuccess)
        return SweepAttrs{0, 0};
    return SweepAttrs{a.numRegs, (int)a.sharedSizeBytes};
}

hipError_t launch_sweep(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, uint32_t sweep0,
                        int32_t nsw, uint32_t mstart, int32_t m)
{
    HEVMC_DISPATCH(launch_sweep_t, coords, acc, rows, sweep0, nsw, mstart, m);
}

hipError_t launch_sweep_batch(const Launch &L, const BatchArgs &b, const int32_t *map, int32_t n_slots,
                              void *coords, hevmc_walker_acc *acc, double *rows, int32_t nsw)
{
    HEVMC_DISPATCH(launch_batch_t, b, map, n_slots, coords, acc, rows, nsw);
}

hipError_t launch_local_energy(const Launch &L, const void *coords, double *out)
{
    HEVMC_DISPATCH(launch_energy_t, coords, out);
}

hipError_t launch_pair_hist(const Launch &L, const void *coords, uint64_t *counts)
{
    HEVMC_DISPATCH(launch_hist_t, coords, counts);
}

hipError_t launch_init(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, int fcc, int nc,
                       double a_lat)
{
    HEVMC_DISPATCH(launch_init_t, coords, acc, rows, fcc, nc, a_lat);
}

hipError_t launch_move_delta(const Launch &L, const void *coords, const int32_t *s, const double *d,
                             double *out)
{
    HEVMC_DISPATCH(launch_delta_t, coords, s, d, out);
}

// ---------------------------------------------------------------------------
// Walkers beyond one workgroup's LDS ("spread" walkers).  Sec. 3 describes a
// cooperative kernel in which several blocks serve one walker; here one
// walker is spread over C workgroups of a cooperative launch (every
// workgroup resident at once), workgroup g holding atoms [g S, g S + S) of
// the walker in its LDS.  Every micro-update is decided by all C workgroups
// together: each forms the Eq. (7) sums over its own atoms (the plain form:
// u and V at the old and the new position), publishes them to a mailbox in
// device memory, and waits until all C have published; every workgroup then
// adds the C partial sums in the same order and takes the same decision.
// The workgroup holding the next move's atom publishes its position in the
// same way.  Every wait is bounded: after spin_cap polls the workgroup gives
// up, records the timeout in *status and leaves; the others then time out in
// turn, so the grid always drains.  Local energies of such walkers come from
// separate kernels that stream the partners through LDS tiles: partial sums
// over blocks of atoms (several workgroups per walker), then a per-walker
// finish that adds them in block order.

// Local energy of spread walkers in two steps, so that every compute unit
// works even when there are fewer walkers than compute units.
// k_energy_part: workgroup blockIdx.x = w * B + b forms, for the atoms i of
// its block b (a run of whole NT-atom chunks) and all their partners j
// (streamed from device memory through LDS tiles of `tile` atoms), the sums
// (|G_i|^2, L_i, ordered V, ordered U) and a non-finite flag, into
// part[blockIdx.x][5].  Every ordered pair is formed.  HIST: each unordered
// pair (i < j) inside the cutoff is also counted in the pair-distance
// histogram of walker w (p.gr, p.gr_bins bins of [0, L/2], the binning of
// the one-workgroup sweep), through an LDS copy and integer atomics.
template <typename T, int NT, bool HIST>
__global__ __launch_bounds__(NT) void k_energy_part(KParams p, const T *__restrict__ coords,
                                                    double *__restrict__ part, int B, int tile)
{
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double ebuf[NW * 4];
    T *tx = reinterpret_cast<T *>(smem_raw);
    T *ty = tx + tile, *tz = ty + tile;
    const int n = p.n, tid = threadIdx.x;
    const int w = (int)(blockIdx.x / (uint32_t)B), b = (int)(blockIdx.x % (uint32_t)B);
    const int nch = (n + NT - 1) / NT, cpb = (nch + B - 1) / B;
    const int i_begin = b * cpb * NT, i_end = min(n, (b + 1) * cpb * NT);
    const T *gx = coords + (size_t)w * 3 * (size_t)n;
    const T *gy = gx + n, *gz = gy + n;
    const int nb = HIST ? p.gr_bins : 0;
    const double bin_scale = (double)nb * 2.0 * p.invL;   // bins per Angstrom
    uint32_t *hist = HIST ? reinterpret_cast<uint32_t *>(smem_raw + 3 * (size_t)tile * sizeof(T)) : nullptr;
    if constexpr (HIST)
        for (int q = tid; q < nb; q += NT)
            hist[q] = 0u;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // sum |G_i|^2, sum L_i, ordered V, ordered U
    bool bad = false;
    for (int c0 = i_begin; c0 < i_end; c0 += NT) {
        const int i = c0 + tid;
        const bool live = i < i_end;
        const T xi = live ? gx[i] : T(0), yi = live ? gy[i] : T(0), zi = live ? gz[i] : T(0);
        bad |= live && !(isfinite((double)xi) && isfinite((double)yi) && isfinite((double)zi));
        double sgx = 0.0, sgy = 0.0, sgz = 0.0, sl = 0.0, sv = 0.0, su = 0.0;
        for (int j0 = 0; j0 < n; j0 += tile) {
            const int m = min(tile, n - j0);
            __syncthreads();
            for (int q = tid; q < m; q += NT) {
                tx[q] = gx[j0 + q];
                ty[q] = gy[j0 + q];
                tz[q] = gz[j0 + q];
            }
            __syncthreads();
            for (int q = 0; q < m; ++q) {
                if (!live || j0 + q == i)
                    continue;
                const T dx = min_image(xi - tx[q], p);
                const T dy = min_image(yi - ty[q], p);
                const T dz = min_image(zi - tz[q], p);
                const T r2 = dx * dx + dy * dy + dz * dz;
                ETerms e;
                pair_energy(p, r2, e);
                sgx += e.dur * (double)dx;
                sgy += e.dur * (double)dy;
                sgz += e.dur * (double)dz;
                sl += e.lap;
                sv += e.v;
                su += e.u;
                if constexpr (HIST)
                    if (i < j0 + q && pair_inside(p, r2))
                        atomicAdd(&hist[min(nb - 1, (int)(e.r * bin_scale))], 1u);
            }
        }
        acc[0] += sgx * sgx + sgy * sgy + sgz * sgz;
        acc[1] += sl;
        acc[2] += sv;
        acc[3] += su;
    }
    const bool any_bad = walker_any<NT>(bad, ebuf);
    block_sum<NT, 4>(acc, ebuf);
    if constexpr (HIST) {
        __syncthreads();
        uint64_t *grw = p.gr + (size_t)w * (size_t)nb;
        for (int q = tid; q < nb; q += NT)
            if (hist[q])
                atomicAdd(reinterpret_cast<unsigned long long *>(&grw[q]), (unsigned long long)hist[q]);
    }
    if (tid == 0) {
        double *o = part + (size_t)blockIdx.x * 5;
        for (int q = 0; q < 4; ++q)
            o[q] = acc[q];
        o[4] = any_bad ? 1.0 : 0.0;
    }
}

// k_energy_finish: thread w adds walker w's B partial sums in block order and
// forms (E_L, V, T_PB, T_JF, T_F, U) (V and U halved: ordered pairs).
// mode 0: start (u_run, v_run of the configuration; accumulators zeroed);
// mode 1: a sample (accumulators, u_run, v_run reset to the fresh totals);
// mode 2: write the six values to out[w][6].
__global__ void k_energy_finish(KParams p, const double *__restrict__ part, int B, int n_walkers,
                                hevmc_walker_acc *__restrict__ accs, double *__restrict__ out, int mode)
{
    const int w = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (w >= n_walkers)
        return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bool any_bad = false;
    for (int b = 0; b < B; ++b) {
        const double *o = part + ((size_t)w * B + b) * 5;
        for (int q = 0; q < 4; ++q)
            acc[q] += o[q];
        any_bad |= o[4] != 0.0;
    }
    const double V = 0.5 * acc[2], U = 0.5 * acc[3];
    const double tpb = -p.kappa * (acc[1] + acc[0]);
    const double el[6] = {V + tpb, V, tpb, -0.5 * p.kappa * acc[1], p.kappa * acc[0], U};
    if (mode == 2) {
        for (int q = 0; q < 6; ++q)
            out[(size_t)w * 6 + q] = el[q];
        return;
    }
    hevmc_walker_acc *a = accs + w;
    if (mode == 0) {
        hevmc_walker_acc z = {};
        *a = z;
    } else {
        // the sample's record, at its index among the walker's samples
        if (p.trace && a->n_samples < (int64_t)p.trace_cap)
            for (int q = 0; q < 6; ++q)
                p.trace[((size_t)w * (size_t)p.trace_cap + (size_t)a->n_samples) * 6 + q] = el[q];
        nsum(a->sum_e, a->c_e, el[0]);
        nsum(a->sum_e2, a->c_e2, el[0] * el[0]);
        nsum(a->sum_v, a->c_v, el[1]);
        nsum(a->sum_tpb, a->c_tpb, el[2]);
        nsum(a->sum_tjf, a->c_tjf, el[3]);
        nsum(a->sum_tf, a->c_tf, el[4]);
        a->n_samples += 1;
    }
    a->u_run = any_bad ? __builtin_nan("") : U;
    a->v_run = any_bad ? __builtin_nan("") : V;
}

// fcc start of spread walkers, one thread per atom (as k_init's fcc start).
template <typename T>
__global__ void k_fcc_global(KParams p, T *__restrict__ coords, int n_walkers, int nc, double a_lat)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = p.n;
    if (q >= (int64_t)n_walkers * n)
        return;
    const int w = (int)(q / n), i = (int)(q % n);
    T *g = coords + (size_t)w * 3 * (size_t)n;
    fcc_site<T>(p, p.wid_base + (uint32_t)w, i, nc, a_lat, &g[i], &g[n + i], &g[2 * n + i]);
}

// Mailbox words of the cooperative sweep: 32 bits of sequence number (the
// launch's micro-update count plus one) over 32 bits of payload.  A word is
// read with one relaxed device-scope atomic load and is valid when its
// sequence matches, so no fence orders it against any other word.
__device__ __forceinline__ void mail_put(uint64_t *w, uint32_t seq, uint32_t payload)
{
    __hip_atomic_store(w, ((uint64_t)seq << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Payload word q (0 or 1: high or low half) of a double.
__device__ __forceinline__ uint32_t half_of(double v, int q)
{
    return (uint32_t)(q == 0 ? __double2hiint(v) : __double2loint(v));
}

// Publishes an atom's position in PW words (FP64: high and low halves of x,
// y, z; FP32: the bits of x, y, z).
__device__ __forceinline__ void put_position(uint64_t *w, uint32_t seq, double x, double y, double z)
{
    mail_put(w + 0, seq, half_of(x, 0));
    mail_put(w + 1, seq, half_of(x, 1));
    mail_put(w + 2, seq, half_of(y, 0));
    mail_put(w + 3, seq, half_of(y, 1));
    mail_put(w + 4, seq, half_of(z, 0));
    mail_put(w + 5, seq, half_of(z, 1));
}
__device__ __forceinline__ void put_position(uint64_t *w, uint32_t seq, float x, float y, float z)
{
    mail_put(w + 0, seq, __float_as_uint(x));
    mail_put(w + 1, seq, __float_as_uint(y));
    mail_put(w + 2, seq, __float_as_uint(z));
}

// The position published in words lo .. lo + PW - 1 held by the lanes of
// the same index (wave-uniform result).
__device__ __forceinline__ void get_position(uint32_t word, int lo, double &x, double &y, double &z)
{
    x = __hiloint2double(readlane_i((int)word, lo), readlane_i((int)word, lo + 1));
    y = __hiloint2double(readlane_i((int)word, lo + 2), readlane_i((int)word, lo + 3));
    z = __hiloint2double(readlane_i((int)word, lo + 4), readlane_i((int)word, lo + 5));
}
__device__ __forceinline__ void get_position(uint32_t word, int lo, float &x, float &y, float &z)
{
    x = __uint_as_float((uint32_t)readlane_i((int)word, lo));
    y = __uint_as_float((uint32_t)readlane_i((int)word, lo + 1));
    z = __uint_as_float((uint32_t)readlane_i((int)word, lo + 2));
}

// The cooperative sweep of spread walkers: workgroup blockIdx.x serves slice
// g = blockIdx.x % c.C of walker blockIdx.x / c.C.  Sweeps t = sweep0 ..
// sweep0 + nsw - 1, the plain form of Eq. (7) (u and V at both positions),
// no local-energy samples (the caller runs them between launches); measured
// sweeps count moves and add v_run to sum_vs.  Movelog as in k_sweep.
//
// Per micro-update mv (parity par = mv & 1 picks one of two mailbox rows of
// the walker, 4C + 8 words each):
//  * every workgroup knows the moved atom's old position (see below) and
//    forms the trial position;
//  * the lane holding the next micro-update's atom in its slice (if that
//    atom is another one) publishes the atom's position in words 4C ..;
//  * each workgroup forms its partial Eq. (7) sums over its slice and lanes
//    0..3 of wave 0 publish them in words 4g .. 4g + 3 (FP64 halves);
//  * wave 0 polls all words it needs until every one carries this move's
//    sequence (bounded by spin_cap polls), adds the C partials in slice
//    order and hands the totals and the next old position to the other
//    waves through LDS; every workgroup takes the same decision.
// A row is written again two moves later, only after its writer has seen
// every workgroup's words of the move in between, which each wrote after
// reading this row.  The next move's old position is the published one, or,
// for the same atom again, the trial position if accepted and the old one if
// not; the first move of a launch reads it from device memory, which the
// launch writes only at its end (each workgroup its slice).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_sweep_coop(KParams p, CoopArgs c, T *__restrict__ coords,
                                                   hevmc_walker_acc *__restrict__ accs, uint32_t sweep0,
                                                   int32_t nsw, uint32_t mstart)
{
    constexpr int NW = NT / 64;
    constexpr int PW = sizeof(T) == 8 ? 6 : 3;   // words of a published position
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[NW][2];
    __shared__ double tot[5];   // dU, dV, the next old position
    __shared__ int fail_flag;
    const int w = (int)(blockIdx.x / (uint32_t)c.C), g = (int)(blockIdx.x % (uint32_t)c.C);
    const int n = p.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int C = c.C;
    const int i0 = g * c.S, ns = min(c.S, n - i0);   // this workgroup's atoms [i0, i0 + ns)
    T *gx = coords + (size_t)w * 3 * (size_t)n;
    T *gy = gx + n, *gz = gy + n;
    T *sx = reinterpret_cast<T *>(smem_raw);
    T *sy = sx + c.S, *sz = sy + c.S;
    // thread q % NT owns slice atom q: it loads it, writes its moves and
    // stores it back, so its LDS entry needs no barrier
    for (int i = tid; i < ns; i += NT) {
        sx[i] = gx[i0 + i];
        sy[i] = gy[i0 + i];
        sz[i] = gz[i0 + i];
    }
    if (tid == 0)
        fail_flag = 0;
    __syncthreads();
    hevmc_walker_acc *accp = accs + w;
    double u_run = accp->u_run, v_run = accp->v_run;
    int64_t n_acc = 0, n_try = 0, n_swm = 0;
    const uint32_t wid = p.wid_base + (uint32_t)w;
    const int row_words = 4 * C + 8;
    uint64_t *mail = c.mail + (size_t)w * 2 * (size_t)row_words;
    double *mlw = (p.movelog && w < p.log_walkers && g == 0) ? p.movelog + (size_t)w * (size_t)p.log_cap * 4
                                                             : nullptr;
    uint32_t mv = 0;   // micro-updates of this launch
    bool failed = false;
    // this batch's moves (lane l: micro-step k0 + l) and the next batch's
    int bs, nbs = 0;
    double bxi, bdx, bdy, bdz, nbxi = 0.5, nbdx = 0.0, nbdy = 0.0, nbdz = 0.0;
    draw_move(p, (uint32_t)lane, sweep0, wid, bs, bxi, bdx, bdy, bdz);
    double blx = log(bxi);
    T ox = 0, oy = 0, oz = 0;   // old position of the current micro-update's atom
    {
        const int s0 = readlane_i(bs, 0);
        ox = gx[s0];
        oy = gy[s0];
        oz = gz[s0];
    }
    for (int it = 0; it < nsw && !failed; ++it) {
        const uint32_t t = sweep0 + (uint32_t)it;
        const bool measured = t >= mstart;
        for (int k0 = 0; k0 < n && !failed; k0 += 64) {
            // the batch after this one (in the next sweep after the last batch)
            const bool next_in_sweep = k0 + 64 < n;
            const bool has_next = next_in_sweep || it + 1 < nsw;
            if (has_next)
                draw_move(p, (uint32_t)((next_in_sweep ? k0 + 64 : 0) + lane), next_in_sweep ? t : t + 1u, wid,
                          nbs, nbxi, nbdx, nbdy, nbdz);
            const int kend = min(64, n - k0);
            for (int j = 0; j < kend; ++j) {
                const int s = readlane_i(bs, j);
                const double lxi = lane_value(blx, j);
                const int s_next = j + 1 < kend ? readlane_i(bs, j + 1) : has_next ? readlane_i(nbs, 0) : -1;
                const bool pub = s_next >= 0 && s_next != s;
                const uint32_t par = mv & 1u, seq = mv + 1u;
                uint64_t *row = mail + (size_t)par * (size_t)row_words;
                const T nx = trial_coord<T>((double)ox + lane_value(bdx, j), p);
                const T ny = trial_coord<T>((double)oy + lane_value(bdy, j), p);
                const T nz = trial_coord<T>((double)oz + lane_value(bdz, j), p);
                if (pub && s_next >= i0 && s_next < i0 + ns && tid == (s_next - i0) % NT) {
                    const int q = s_next - i0;
                    put_position(row + 4 * C, seq, sx[q], sy[q], sz[q]);
                }
                // this workgroup's part of the Eq. (7) sums
                double du = 0.0, dv = 0.0;
                for (int q = tid; q < ns; q += NT) {
                    const T xi = sx[q], yi = sy[q], zi = sz[q];
                    const T r2o = dist2(p, ox, oy, oz, xi, yi, zi);
                    const T r2n = dist2(p, nx, ny, nz, xi, yi, zi);
                    T uo, vo, un, vn;
                    pair_uv2(p, r2o, r2n, uo, vo, un, vn);
                    const bool self = (i0 + q == s);
                    du += self ? 0.0 : (double)(un - uo);
                    dv += self ? 0.0 : (double)(vn - vo);
                }
                du = wave_sum(du);
                dv = wave_sum(dv);
                if (lane == 0) {
                    red[wave][0] = du;
                    red[wave][1] = dv;
                }
                __syncthreads();
                if (wave == 0) {
                    double pu = 0.0, pv = 0.0;
                    for (int q = 0; q < NW; ++q) {
                        pu += red[q][0];
                        pv += red[q][1];
                    }
                    if (lane < 4)
                        mail_put(row + 4 * g + lane, seq, half_of(lane < 2 ? pu : pv, lane & 1));
                    // every word of this move: the C partials and the published position
                    const int nw = 4 * C + (pub ? PW : 0);
                    uint64_t word = 0;
                    bool have = lane >= nw;
                    uint32_t spins = 0;
                    int f = 0;
                    while (true) {
                        if (!have) {
                            word = __hip_atomic_load(row + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            have = (uint32_t)(word >> 32) == seq;
                        }
                        if (__builtin_amdgcn_ballot_w64(!have) == 0ull)
                            break;
                        if (++spins > c.spin_cap) {
                            f = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    const uint32_t pay = (uint32_t)word;
                    double DU = 0.0, DV = 0.0;
                    for (int q = 0; q < C; ++q) {
                        DU += __hiloint2double(readlane_i((int)pay, 4 * q), readlane_i((int)pay, 4 * q + 1));
                        DV += __hiloint2double(readlane_i((int)pay, 4 * q + 2), readlane_i((int)pay, 4 * q + 3));
                    }
                    T px = 0, py = 0, pz = 0;
                    if (pub)
                        get_position(pay, 4 * C, px, py, pz);
                    if (lane == 0) {
                        tot[0] = DU;
                        tot[1] = DV;
                        tot[2] = (double)px;
                        tot[3] = (double)py;
                        tot[4] = (double)pz;
                        fail_flag = f;
                    }
                }
                __syncthreads();
                if (fail_flag) {
                    failed = true;
                    break;
                }
                const double DU = tot[0], DV = tot[1];
                ++mv;
                const bool accept = metropolis_accept_log(DU, lxi);
                const int64_t q_log = c.log_base + (int64_t)it * n + k0 + j;
                if (mlw && tid == 0 && q_log < p.log_cap) {
                    double *rec = mlw + 4 * q_log;
                    rec[0] = (double)s;
                    rec[1] = accept ? 1.0 : 0.0;
                    rec[2] = DU;
                    rec[3] = DV;
                }
                if (measured) {
                    n_try += 1;
                    n_acc += accept ? 1 : 0;
                }
                if (accept) {
                    u_run += DU;
                    v_run += DV;
                    if (s >= i0 && s < i0 + ns && tid == (s - i0) % NT) {
                        sx[s - i0] = nx;
                        sy[s - i0] = ny;
                        sz[s - i0] = nz;
                    }
                }
                // the next micro-update's old position
                if (!pub) {
                    if (accept) {
                        ox = nx;
                        oy = ny;
                        oz = nz;
                    }
                } else {
                    ox = (T)tot[2];
                    oy = (T)tot[3];
                    oz = (T)tot[4];
                }
                // tot is written again only after the next move's first barrier
            }
            if (has_next) {
                bs = nbs;
                bxi = nbxi;
                bdx = nbdx;
                bdy = nbdy;
                bdz = nbdz;
                blx = log(bxi);
            }
        }
        if (measured && !failed) {
            if (g == 0 && tid == 0)
                nsum(accp->sum_vs, accp->c_vs, v_run);
            n_swm += 1;
        }
    }
    if (failed) {
        if (tid == 0)
            atomicOr(c.status, 1u);
        return;
    }
    for (int i = tid; i < ns; i += NT) {
        gx[i0 + i] = sx[i];
        gy[i0 + i] = sy[i];
        gz[i0 + i] = sz[i];
    }
    if (g == 0 && tid == 0) {
        accp->u_run = u_run;
        accp->v_run = v_run;
        accp->n_sweeps_meas += n_swm;
        accp->n_acc += n_acc;
        accp->n_try += n_try;
    }
}

// workgroup sizes of the cooperative sweep (the plan picks one of them)
template <int NT>
constexpr bool kCoopThreads = NT == 256 || NT == 512 || NT == 1024;

template <typename T, int NT>
static hipError_t launch_coop_t(const Launch &L, const CoopArgs &c, void *coords, hevmc_walker_acc *acc,
                                uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t walkers)
{
    if constexpr (!kCoopThreads<NT>) {
        return hipErrorInvalidValue;
    } else {
        auto kern = k_sweep_coop<T, NT>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        KParams k = L.k;
        CoopArgs ca = c;
        T *cp = (T *)coords;
        void *args[] = {&k, &ca, &cp, &acc, &sweep0, &nsw, &mstart};
        return hipLaunchCooperativeKernel((const void *)kern, dim3((unsigned)(walkers * c.C)), dim3(NT), args,
                                          (unsigned)L.lds_bytes, L.stream);
    }
}

template <typename T, int NT>
static hipError_t coop_capacity_t(const Launch &L, int *blocks_per_cu)
{
    if constexpr (!kCoopThreads<NT>) {
        return hipErrorInvalidValue;
    } else {
        auto kern = k_sweep_coop<T, NT>;
        hipError_t e = allow_lds(kern, L.lds_bytes);
        if (e != hipSuccess)
            return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)kern, NT, L.lds_bytes);
    }
}

template <typename T, int NT>
static hipError_t launch_energy_global_t(const Launch &L, const void *coords, hevmc_walker_acc *acc, double *out,
                                         int mode, int tile, double *part, int B)
{
    // the pair histogram at samples (mode 1) when the sweep asks for one
    const bool hist = mode == 1 && L.k.gr && L.k.gr_bins > 0;
    auto kern = hist ? k_energy_part<T, NT, true> : k_energy_part<T, NT, false>;
    const size_t lds = 3 * (size_t)tile * sizeof(T) + (hist ? (size_t)L.k.gr_bins * sizeof(uint32_t) : 0);
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess)
        return e;
    const int W = L.p.n_walkers_grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)(W * B)), dim3(NT), lds, L.stream, L.k, (const T *)coords, part, B, tile);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    KParams kf = L.k;
    if (mode != 1)
        kf.trace = nullptr;   // records are written at samples only
    hipLaunchKernelGGL(k_energy_finish, dim3((unsigned)((W + 63) / 64)), dim3(64), 0, L.stream, kf,
                       (const double *)part, B, W, acc, out, mode);
    return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_fcc_global_t(const Launch &L, void *coords, int nc, double a_lat)
{
    const int64_t total = (int64_t)L.p.n_walkers_grid * L.k.n;
    const int bs = 256;
    hipLaunchKernelGGL(k_fcc_global<T>, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, L.stream, L.k,
                       (T *)coords, L.p.n_walkers_grid, nc, a_lat);
    return hipGetLastError();
}

hipError_t launch_sweep_coop(const Launch &L, const CoopArgs &c, void *coords, hevmc_walker_acc *acc,
                             uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t walkers)
{
    HEVMC_DISPATCH(launch_coop_t, c, coords, acc, sweep0, nsw, mstart, walkers);
}

hipError_t coop_blocks_per_cu(const Launch &L, int *blocks_per_cu)
{
    HEVMC_DISPATCH(coop_capacity_t, blocks_per_cu);
}

int energy_blocks(int n_walkers, int n)
{
    // about 2048 workgroups in all (several per compute unit), each at least
    // one 256-atom chunk of its walker
    const int nch = (n + 255) / 256;
    const int want = (2048 + n_walkers - 1) / n_walkers;
    return std::max(1, std::min(nch, want));
}

hipError_t launch_energy_global(const Launch &Ls, const void *coords, hevmc_walker_acc *acc, double *out, int mode,
                                double *part)
{
    // 256 threads whatever the sweep's workgroup size (no spills at this size);
    // 24 KB tiles, so several workgroups share a compute unit
    Launch L = Ls;
    L.threads = 256;
    const int tile = L.fp32 ? 2048 : 1024;
    const int B = energy_blocks(L.p.n_walkers_grid, L.k.n);
    HEVMC_DISPATCH(launch_energy_global_t, coords, acc, out, mode, tile, part, B);
}

hipError_t launch_fcc_global(const Launch &L, void *coords, int nc, double a_lat)
{
    HEVMC_DISPATCH(launch_fcc_global_t, coords, nc, a_lat);
}

hipError_t launch_draw_moves(const Launch &L, uint32_t t, int32_t *s, double *xi, double *d)
{
    const int total = L.p.n_walkers_grid * L.k.n;
    const int bs = 256;
    hipLaunchKernelGGL(k_draw_moves, dim3((total + bs - 1) / bs), dim3(bs), 0, L.stream, L.k, t, s, xi, d,
                       total);
    return hipGetLastError();
}

}  // namespace hevmc
