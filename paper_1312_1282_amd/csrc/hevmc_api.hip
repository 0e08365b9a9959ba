// libhevmc C ABI: argument validation, launch planning, the ensemble layer and
// the host-buffer parity entry.  Declarations and contracts: include/hevmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hevmc.h"
#include "hevmc_internal.hpp"

using namespace hevmc;

namespace {

thread_local std::string g_err = "no error";

hevmc_status fail(hevmc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

hevmc_status hip_fail(hipError_t e, const char *what)
{
    return fail(HEVMC_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Static LDS of the kernels (partial sums: (2x2 + 4) doubles per wave plus two),
// with a margin.
size_t static_lds(int threads) { return (size_t)(threads / 64) * 8 * sizeof(double) + 64; }

struct DeviceLimits {
    int cus = 0;
    size_t lds_per_block = 0;
    size_t lds_per_cu = 0;
};

hevmc_status device_limits_query(int dev, DeviceLimits &d);

// Limits of the current device, queried once per device.
hevmc_status device_limits(DeviceLimits &d)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    static std::mutex mu;
    static std::map<int, DeviceLimits> known;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = known.find(dev);
        if (it != known.end()) {
            d = it->second;
            return HEVMC_OK;
        }
    }
    hevmc_status st = device_limits_query(dev, d);
    if (st == HEVMC_OK) {
        std::lock_guard<std::mutex> g(mu);
        known[dev] = d;
    }
    return st;
}

hevmc_status device_limits_query(int dev, DeviceLimits &d)
{
    hipError_t e;
    int v = 0;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute(MultiprocessorCount)");
    d.cus = v;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute(MaxSharedMemoryPerBlock)");
    d.lds_per_block = (size_t)v;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute(MaxSharedMemoryPerMultiprocessor)");
    d.lds_per_cu = (size_t)v;
    return HEVMC_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Box side as the kernels use it.  The FP32 form works in a box of the
// float-representable side so that wrap and minimum image agree.
double box_side(const hevmc_params *p)
{
    const double L = std::cbrt((double)p->n / p->density);
    return p->precision == HEVMC_FP32 ? (double)(float)L : L;
}

hevmc_status check_params(const hevmc_params *p)
{
    if (!p)
        return fail(HEVMC_EINVAL, "params is NULL");
    if (p->n < 2)
        return fail(HEVMC_EINVAL, "n = %d: need at least 2 atoms", p->n);
    if (p->n_walkers < 1)
        return fail(HEVMC_EINVAL, "n_walkers = %d: need at least 1", p->n_walkers);
    if (p->precision != HEVMC_FP64 && p->precision != HEVMC_FP32)
        return fail(HEVMC_EINVAL, "precision = %d is not HEVMC_FP64 or HEVMC_FP32", p->precision);
    if (p->order != HEVMC_SELECT_RANDOM && p->order != HEVMC_SELECT_SEQUENTIAL)
        return fail(HEVMC_EINVAL, "order = %d is not a hevmc_order", p->order);
    if (!finite_pos(p->density))
        return fail(HEVMC_EINVAL, "density = %g must be finite and > 0", p->density);
    if (!std::isfinite(p->b) || p->b < 0.0)
        return fail(HEVMC_EINVAL, "b = %g must be finite and >= 0", p->b);
    if (!finite_pos(p->hbar2_over_m))
        return fail(HEVMC_EINVAL, "hbar2_over_m = %g must be finite and > 0", p->hbar2_over_m);
    if (!finite_pos(p->step_sigma))
        return fail(HEVMC_EINVAL, "step_sigma = %g must be finite and > 0", p->step_sigma);
    if (p->threads != 0 && p->threads != 64 && p->threads != 128 && p->threads != 256 && p->threads != 512 &&
        p->threads != 1024)
        return fail(HEVMC_EINVAL, "threads = %d must be 0, 64, 128, 256, 512 or 1024", p->threads);
    if (p->variant < HEVMC_VARIANT_AUTO || p->variant > HEVMC_VARIANT_ROWS)
        return fail(HEVMC_EINVAL, "variant = %d is not a hevmc_variant", p->variant);
    return HEVMC_OK;
}

// Threads per walker when the caller leaves the choice to the library: one
// wave per walker (four walkers per workgroup) up to 8 atoms per lane, else
// about 8 atoms per lane, 2 to 8 waves.
int default_threads(int n)
{
    if (n <= 64 * kRowsPerLane)
        return 64;
    if (n <= 1024)
        return 128;
    if (n <= 3072)
        return 256;
    return 512;
}

// Waves one SIMD can hold for a kernel using vgprs registers per thread
// (512 registers per lane per SIMD, allocated in granules of 8; at most 8 waves).
int waves_per_simd(int vgprs)
{
    if (vgprs <= 0)
        return 8;
    const int alloc = (vgprs + 7) & ~7;
    const int w = 512 / alloc;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

size_t lds_needed(const hevmc_params *p)
{
    return (size_t)3 * (size_t)p->n * (p->precision == HEVMC_FP32 ? sizeof(float) : sizeof(double));
}

// LDS of one walker of the row-sum sweep.
size_t rows_lds_bytes(const hevmc_params *p)
{
    const size_t tsz = p->precision == HEVMC_FP32 ? sizeof(float) : sizeof(double);
    return rows_lds_offset(p->n, tsz) + (size_t)p->n * sizeof(double);
}

void make_kparams(const hevmc_params *p, KParams &k);

// Launch plan: threads per walker, sweep variant and the dynamic LDS request.
// The request is padded so that each compute unit holds r walkers, r the
// largest divisor of ceil(W / CUs) whose walkers fit in its LDS: the walkers
// are then spread evenly over the chip, in equal rounds.
// A walker whose coordinates do not fit in one workgroup's LDS (spread
// walker, plain form): C slices of S atoms, one workgroup of 256 threads each,
// C the fewest slices whose coordinates fit.
hevmc_status plan_spread(const hevmc_params *p, void *stream, Launch &L, const DeviceLimits &d)
{
    const bool fp32 = p->precision == HEVMC_FP32;
    const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
    // 512 threads (two waves per SIMD) unless the caller asks for 256 or 1024
    const int threads = (p->threads == 256 || p->threads == 1024) ? p->threads : 512;
    const size_t stat = static_lds(threads);
    const size_t max_dyn = d.lds_per_block > stat ? d.lds_per_block - stat : 0;
    // at most 14 slices: one wave polls a move's 4C + 6 mailbox words, one per lane
    const int c_max = std::min(14, d.cus);
    int C = 2;
    int S = (p->n + C - 1) / C;
    while ((size_t)3 * (size_t)S * tsz > max_dyn && C < c_max) {
        ++C;
        S = (p->n + C - 1) / C;
    }
    if ((size_t)3 * (size_t)S * tsz > max_dyn)
        return fail(HEVMC_ENOFIT, "walker of %d atoms does not fit in %d workgroups' LDS", p->n, c_max);
    make_kparams(p, L.k);
    L.k.sorted = 0;
    L.p.n_walkers_grid = p->n_walkers;
    L.threads = threads;
    L.fp32 = fp32;
    L.rows = false;
    L.rreg = false;
    L.spread = true;
    L.slices = C;
    L.slice_atoms = S;
    L.lds_bytes = ((size_t)3 * (size_t)S * tsz + 15) & ~(size_t)15;
    L.walker_lds = L.lds_bytes * (size_t)C;
    L.stream = (hipStream_t)stream;
    return HEVMC_OK;
}

hevmc_status plan(const hevmc_params *p, void *stream, Launch &L, int32_t gr_bins = 0, bool allow_spread = false)
{
    hevmc_status st = check_params(p);
    if (st != HEVMC_OK)
        return st;
    DeviceLimits d;
    if ((st = device_limits(d)) != HEVMC_OK)
        return st;
    const int threads = p->threads ? p->threads : default_threads(p->n);
    const bool wave_mode = threads == 64;
    // walkers per workgroup: one, or kWalkersPerGroup single-wave walkers
    const int per_group = wave_mode ? kWalkersPerGroup : 1;
    // static LDS per workgroup: the reservation below, or what the sweep
    // kernels actually declare if that is more
    const bool fp32 = p->precision == HEVMC_FP32;
    const SweepAttrs attr_plain = sweep_attrs(fp32, threads, false), attr_rows = sweep_attrs(fp32, threads, true);
    const size_t stat = std::max<size_t>(wave_mode ? 64 : static_lds(threads),
                                         (size_t)std::max(attr_plain.static_lds, attr_rows.static_lds));
    const size_t max_dyn = d.lds_per_block > stat ? d.lds_per_block - stat : 0;
    const size_t need_plain = lds_needed(p);
    const size_t need_rows = rows_lds_bytes(p);
    const size_t align16 = 15;
    if (need_plain > max_dyn || (wave_mode && per_group * ((need_plain + align16) & ~align16) > max_dyn)) {
        if (allow_spread && !wave_mode) {
            // a spread walker's histogram is formed by its local-energy kernels
            st = plan_spread(p, stream, L, d);
            L.k.gr_bins = gr_bins;
            return st;
        }
        return fail(HEVMC_ENOFIT, "walker of %d atoms needs %zu B of LDS; a workgroup can have %zu B", p->n,
                    need_plain * per_group, max_dyn);
    }
    const bool rows_ok = p->n <= kRowsPerLane * threads &&
                         per_group * ((need_rows + align16) & ~align16) <= max_dyn;
    // rows that do not fit in LDS can live in registers (FP32, 512 threads,
    // up to kRegChunks atoms per lane); the walker then needs the plain LDS
    const bool rreg_ok = !rows_ok && rreg_form(fp32, threads) && p->n <= kRegChunks * threads;
    if (p->variant == HEVMC_VARIANT_ROWS && !rows_ok && !rreg_ok)
        return fail(HEVMC_ENOFIT, "row-sum sweep needs N <= %d x threads and %zu B of LDS per walker",
                    kRowsPerLane, need_rows);
    const bool use_rows = p->variant == HEVMC_VARIANT_ROWS ||
                          (p->variant == HEVMC_VARIANT_AUTO && (rows_ok || rreg_ok));
    const bool rreg = use_rows && !rows_ok;
    const SweepAttrs attr_use = rreg ? sweep_attrs(fp32, threads, true, true) : use_rows ? attr_rows : attr_plain;
    // workgroups a compute unit can hold: by LDS, and by waves (4 SIMDs, register
    // file shared by the waves of a SIMD)
    const int waves_per_group = threads / 64 * per_group;
    const int by_waves = 4 * waves_per_simd(attr_use.vgprs) / waves_per_group;
    const int groups = (p->n_walkers + per_group - 1) / per_group;
    const int per_cu = (groups + d.cus - 1) / d.cus;
    // spatial order of the atoms (a resort per sweep; it lets whole waves skip
    // the short-range exponentials): used when it costs no workgroups per
    // compute unit.  The choice depends on (N, precision, threads, variant)
    // only, never on the launch's size, so a walker's results do not either.
    const bool lds_rows = use_rows && !rreg;
    const size_t base_need = ((lds_rows ? need_rows : need_plain) + align16) & ~align16;
    bool sorted = false;
    if (!wave_mode && p->n <= kRowsPerLane * threads && p->n <= 65535) {
        const size_t tsz = fp32 ? sizeof(float) : sizeof(double);
        const size_t with_sort = (sorted_walker_lds(p->n, tsz, lds_rows) + align16) & ~align16;
        auto fit = [&](size_t bytes) {
            const int g = bytes > max_dyn ? 0 : (int)(d.lds_per_cu / (bytes * per_group + stat));
            return by_waves > 0 ? std::min(g, by_waves) : g;
        };
        sorted = fit(with_sort) > 0 && fit(with_sort) >= fit(base_need);
    }
    // the pair histogram (when the caller collects it) goes behind everything
    // else; it never changes the plan's other choices, so a chain has the same
    // bits with or without it
    const size_t tsz_w = fp32 ? sizeof(float) : sizeof(double);
    const size_t walker_need =
        gr_bins > 0
            ? (hist_lds_offset(p->n, tsz_w, lds_rows, sorted) + (size_t)gr_bins * sizeof(uint32_t) + align16) &
                  ~align16
        : sorted ? (sorted_walker_lds(p->n, tsz_w, lds_rows) + align16) & ~align16
                 : base_need;
    if (walker_need * per_group > max_dyn)
        return fail(HEVMC_ENOFIT, "walker of %d atoms with a %d-bin pair histogram needs %zu B of LDS; "
                    "a workgroup can have %zu B", p->n, gr_bins, walker_need * per_group, max_dyn);
    const size_t need = walker_need * per_group;
    size_t lds = need;
    for (int r = per_cu; r >= 1; --r) {
        if (per_cu % r != 0)
            continue;
        if ((size_t)r * (need + stat) > d.lds_per_cu || (r > by_waves && r > 1))
            continue;
        size_t even = d.lds_per_cu / (size_t)r;
        even = even > stat + 128 ? even - stat - 128 : 0;
        even &= ~(size_t)255;
        if (even > lds)
            lds = even < max_dyn ? even : max_dyn;
        break;
    }
    make_kparams(p, L.k);
    L.k.sorted = sorted ? 1 : 0;
    L.k.gr_bins = gr_bins;
    L.p.n_walkers_grid = p->n_walkers;
    L.threads = threads;
    L.fp32 = p->precision == HEVMC_FP32;
    L.rows = use_rows;
    L.rreg = rreg;
    L.lds_bytes = lds;
    L.walker_lds = walker_need;
    L.stream = (hipStream_t)stream;
    return HEVMC_OK;
}

// Kernel-side constants of a parameter set.
void make_kparams(const hevmc_params *p, KParams &k)
{
    const double Ld = box_side(p);
    const double h = 0.5 * Ld;
    const double b = p->b;
    const double q = b / h;
    k.n = p->n;
    k.order = p->order;
    k.wid_base = p->walker_id_base;
    k.key0 = (uint32_t)p->seed;
    k.key1 = (uint32_t)(p->seed >> 32);
    k.L = Ld;
    k.invL = 1.0 / Ld;
    k.h2 = h * h;
    k.step = p->step_sigma;
    k.c5 = -0.5 * (b * b * b * b * b);
    k.u0 = q * q * q * q * q;   // -2 f(L/2) = (b / (L/2))^5
    k.kappa = 0.5 * p->hbar2_over_m;
    k.Lf = (float)Ld;
    k.invLf = (float)(1.0 / Ld);
    k.h2f = (float)(h * h);
    k.c5f = (float)k.c5;
    k.u0f = (float)k.u0;
    // FP32 form of V, HFD-B(HE) with eps and r_m folded into the constants and
    // e^a written 2^(a log2 e): see KParams
    {
        const double l2e = 1.0 / std::log(2.0), s = std::sqrt(l2e);
        k.vb = (float)(az::beta * l2e / az::rm2);
        k.va = (float)(az::alpha * l2e / az::rm);
        k.vl = (float)std::log2(az::epsA);
        k.vd = (float)(az::Drm * s);
        k.vs = (float)s;
        k.vdr = (float)az::Drm;
        k.vc6 = (float)az::eC6;
        k.vc8 = (float)az::eC8;
        k.vc10 = (float)az::eC10;
    }
    k.sorted = 0;
    k.gr_bins = 0;
    k.gr = nullptr;
    k.trace = nullptr;
    k.trace_cap = 0;
    k.share_tag = 0;
    k.movelog = nullptr;
    k.log_cap = 0;
    k.log_walkers = 0;
}

// A fresh nonzero 24-bit tag per sweep launch: walkers compare progress only
// with a partner of the same launch (walkers of other launches running on the
// same compute units, or words left over from earlier launches, are ignored).
static uint32_t next_share_tag()
{
    static std::atomic<uint32_t> counter{0};
    uint32_t t;
    do {
        t = (counter.fetch_add(1, std::memory_order_relaxed) + 1u) & 0xFFFFFFu;
    } while (t == 0u);
    return t;
}

hevmc_status launched(hipError_t e, const char *what) { return e == hipSuccess ? HEVMC_OK : hip_fail(e, what); }

void fcc_cells(int n, int &nc)
{
    nc = 1;
    while (4LL * nc * nc * nc < (long long)n)
        ++nc;
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" const char *hevmc_last_error(void) { return g_err.c_str(); }

extern "C" hevmc_status hevmc_box(const hevmc_params *p, double *L_out)
{
    hevmc_status st = check_params(p);
    if (st != HEVMC_OK)
        return st;
    if (!L_out)
        return fail(HEVMC_EINVAL, "L_out is NULL");
    *L_out = box_side(p);
    return HEVMC_OK;
}

extern "C" hevmc_status hevmc_plan_launch(const hevmc_params *p, hevmc_plan *out)
{
    if (!out)
        return fail(HEVMC_EINVAL, "out must not be NULL");
    Launch L;
    hevmc_status st = plan(p, nullptr, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    DeviceLimits d;
    if ((st = device_limits(d)) != HEVMC_OK)
        return st;
    const int per_group = L.threads == 64 ? kWalkersPerGroup : 1;
    out->threads = L.threads;
    out->variant = L.rows ? HEVMC_VARIANT_ROWS : HEVMC_VARIANT_PLAIN;
    out->spatial_order = L.k.sorted;
    out->walkers_per_cu =
        L.spread ? 0 : (int32_t)(d.lds_per_cu / (L.lds_bytes + static_lds(L.threads))) * per_group;
    out->lds_per_walker = L.walker_lds;
    out->lds_per_group = L.lds_bytes;
    out->slices = L.slices;
    out->reserved = 0;
    return HEVMC_OK;
}

extern "C" hevmc_status hevmc_footprint(const hevmc_params *p, size_t *lds_bytes_per_walker, size_t *hbm_bytes)
{
    Launch L;
    hevmc_status st = plan(p, nullptr, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    if (lds_bytes_per_walker)
        *lds_bytes_per_walker = L.walker_lds;
    if (hbm_bytes)
        *hbm_bytes = (lds_needed(p) + sizeof(hevmc_walker_acc) + (size_t)p->n * sizeof(double)) *
                     (size_t)p->n_walkers;
    return HEVMC_OK;
}

static hevmc_status spread_energy(const Launch &L, const void *coords, hevmc_walker_acc *acc, double *out, int mode);

extern "C" hevmc_status hevmc_init_walkers(const hevmc_params *p, void *coords, hevmc_walker_acc *acc,
                                           double *rows, int32_t fcc_start, void *stream)
{
    Launch L;
    hevmc_status st = plan(p, stream, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    if (!coords || !acc)
        return fail(HEVMC_EINVAL, "coords and acc must be device pointers");
    int nc;
    fcc_cells(p->n, nc);
    if (L.spread) {
        // spread walkers keep no rows (plain form)
        if (fcc_start && (st = launched(launch_fcc_global(L, coords, nc, L.k.L / nc), "fcc kernel launch")) !=
                             HEVMC_OK)
            return st;
        return spread_energy(L, coords, acc, nullptr, 0);
    }
    return launched(launch_init(L, coords, acc, rows, fcc_start ? 1 : 0, nc, L.k.L / nc), "init kernel launch");
}

// Whether the plan puts two or more multi-wave walkers on one compute unit
// (the case the sweep kernels balance by issue priority).
static bool shares_cu(const Launch &L)
{
    DeviceLimits d;
    if (L.threads <= 64 || device_limits(d) != HEVMC_OK)
        return false;
    return d.lds_per_cu / (L.lds_bytes + static_lds(L.threads)) >= 2;
}

// Optional per-move records of a sweep (hevmc_sweep_log).
struct MoveLog {
    double *log = nullptr;
    int32_t walkers = 0;
    int64_t cap = 0;
};

// Device workspace of the cooperative sweeps (mailboxes, arrival counters,
// status word): one grow-only buffer per device, kept until the process ends.
// Calls that overlap on one device would share it: they race (as calls that
// share buffers do).
static hevmc_status spread_workspace(size_t bytes, void **out, int slot = 0)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::pair<void *, size_t>> bufs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(mu);
    auto &b = bufs[{dev, slot}];
    if (b.second < bytes) {
        if (b.first) {
            e = hipDeviceSynchronize();
            if (e != hipSuccess)
                return hip_fail(e, "workspace release");
            (void)hipFree(b.first);
            b.first = nullptr;
            b.second = 0;
        }
        e = hipMalloc(&b.first, bytes);
        if (e != hipSuccess)
            return fail(HEVMC_ENOMEM, "hipMalloc of %zu B for the cooperative sweep's workspace failed", bytes);
        b.second = bytes;
    }
    *out = b.first;
    return HEVMC_OK;
}

// The local energy of spread walkers: partial sums in a workspace of its own
// (slot 1), then the per-walker finish.
static hevmc_status spread_energy(const Launch &L, const void *coords, hevmc_walker_acc *acc, double *out, int mode)
{
    const size_t bytes = (size_t)energy_blocks(L.p.n_walkers_grid, L.k.n) * (size_t)L.p.n_walkers_grid * 5 *
                         sizeof(double);
    void *part = nullptr;
    hevmc_status st = spread_workspace(bytes, &part, 1);
    if (st != HEVMC_OK)
        return st;
    return launched(launch_energy_global(L, coords, acc, out, mode, static_cast<double *>(part)),
                    "local-energy kernel launch");
}

// Polls a cooperative sweep's wait makes before it gives up: HEVMC_SPREAD_SPIN_CAP
// from the environment if set (tests force timeouts with it), else 2^22.
static uint32_t spread_spin_cap()
{
    const char *v = getenv("HEVMC_SPREAD_SPIN_CAP");
    if (v && *v) {
        char *end = nullptr;
        const unsigned long x = strtoul(v, &end, 10);
        if (end && *end == 0)
            return (uint32_t)std::min<unsigned long>(x, 0xFFFFFFFFul);
    }
    return 1u << 22;
}

// hevmc_sweep of spread walkers: groups of walkers that the chip holds at
// once (every workgroup of a cooperative launch must be resident), each group
// in launches that end at the local-energy samples, which run between them.
// Waits for the stream and reports a wait that gave up as HEVMC_EDEVICE.
static hevmc_status sweep_spread(const Launch &L, const hevmc_params *p, void *coords, hevmc_walker_acc *acc,
                                 uint32_t sweep0, int32_t n_sweeps, uint32_t mstart, int32_t m, const MoveLog &mlog)
{
    DeviceLimits d;
    hevmc_status st = device_limits(d);
    if (st != HEVMC_OK)
        return st;
    int bpc = 0;
    if ((st = launched(coop_blocks_per_cu(L, &bpc), "cooperative occupancy query")) != HEVMC_OK)
        return st;
    const int C = L.slices;
    const int max_group = bpc * d.cus / C;
    if (max_group < 1)
        return fail(HEVMC_ENOFIT, "a walker of %d slices does not fit on the chip at once", C);
    const int W = p->n_walkers, G = std::min(W, max_group);
    const size_t mail_bytes = (size_t)G * 2 * (size_t)(4 * C + 8) * sizeof(uint64_t);
    const size_t bytes = mail_bytes + 64;
    void *ws = nullptr;
    if ((st = spread_workspace(bytes, &ws)) != HEVMC_OK)
        return st;
    CoopArgs c;
    c.mail = static_cast<uint64_t *>(ws);
    c.status = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + mail_bytes);
    c.spin_cap = spread_spin_cap();
    c.C = C;
    c.S = L.slice_atoms;
    hipError_t e = hipMemsetAsync(c.status, 0, sizeof(uint32_t), L.stream);
    if (e != hipSuccess)
        return hip_fail(e, "status reset");
    const size_t tsz = L.fp32 ? sizeof(float) : sizeof(double);
    const size_t per_walker = (size_t)3 * (size_t)p->n * tsz;
    const uint64_t end = (uint64_t)sweep0 + (uint64_t)n_sweeps;
    for (int w0 = 0; w0 < W; w0 += G) {
        const int g = std::min(G, W - w0);
        Launch Lg = L;
        Lg.p.n_walkers_grid = g;
        Lg.k.wid_base = L.k.wid_base + (uint32_t)w0;
        if (L.k.gr)
            Lg.k.gr = L.k.gr + (size_t)w0 * (size_t)L.k.gr_bins;
        if (L.k.trace)
            Lg.k.trace = L.k.trace + (size_t)w0 * (size_t)L.k.trace_cap * 6;
        if (mlog.log && w0 < mlog.walkers) {
            Lg.k.movelog = mlog.log + (size_t)w0 * (size_t)mlog.cap * 4;
            Lg.k.log_walkers = mlog.walkers - w0;
            Lg.k.log_cap = mlog.cap;
        } else {
            Lg.k.movelog = nullptr;
            Lg.k.log_walkers = 0;
        }
        void *cg = static_cast<char *>(coords) + (size_t)w0 * per_walker;
        hevmc_walker_acc *ag = acc + w0;
        uint64_t t = sweep0;
        while (t < end) {
            // the launch runs to the next sampled sweep (inclusive) or to the end
            uint64_t te = end - 1;
            bool sample = false;
            if (m > 0 && mstart != 0xFFFFFFFFu) {
                const uint64_t first = std::max<uint64_t>(t, mstart);
                const uint64_t k = (first - mstart + (uint64_t)m) / (uint64_t)m;   // ceil((first - mstart + 1) / m)
                const uint64_t ts = mstart + k * (uint64_t)m - 1;
                if (ts < end) {
                    te = ts;
                    sample = true;
                }
            }
            c.log_base = (int64_t)(t - sweep0) * p->n;
            // sequence numbers restart with each launch
            e = hipMemsetAsync(c.mail, 0, (size_t)g * 2 * (size_t)(4 * C + 8) * sizeof(uint64_t), L.stream);
            if (e != hipSuccess)
                return hip_fail(e, "mailbox reset");
            if ((st = launched(launch_sweep_coop(Lg, c, cg, ag, (uint32_t)t, (int32_t)(te - t + 1), mstart, g),
                               "cooperative sweep launch")) != HEVMC_OK)
                return st;
            if (sample && (st = spread_energy(Lg, cg, ag, nullptr, 1)) != HEVMC_OK)
                return st;
            t = te + 1;
        }
    }
    uint32_t status = 0;
    e = hipMemcpyAsync(&status, c.status, sizeof(uint32_t), hipMemcpyDeviceToHost, L.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(L.stream);
    if (e != hipSuccess)
        return hip_fail(e, "cooperative sweep");
    if (status)
        return fail(HEVMC_EDEVICE, "a cooperative sweep's wait gave up after %u polls (a workgroup of a walker "
                    "stopped arriving); the walkers' state is not valid", c.spin_cap);
    return HEVMC_OK;
}

// The sweep with its optional outputs: pair histogram, per-sample trace and
// per-move records.
static hevmc_status sweep_with(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                               uint64_t *gr, int32_t gr_bins, double *trace, int32_t trace_cap, uint32_t sweep0,
                               int32_t n_sweeps, uint32_t measure_start, int32_t energy_every, void *stream,
                               const MoveLog &mlog = MoveLog())
{
    if (gr && (gr_bins < 1 || gr_bins > HEVMC_MAX_GR_BINS))
        return fail(HEVMC_EINVAL, "gr_bins = %d must be in [1, %d]", gr_bins, HEVMC_MAX_GR_BINS);
    if (trace && trace_cap < 1)
        return fail(HEVMC_EINVAL, "trace_cap = %d must be >= 1", trace_cap);
    Launch L;
    hevmc_status st = plan(p, stream, L, gr ? gr_bins : 0, true);
    if (st != HEVMC_OK)
        return st;
    L.k.gr = gr;
    L.k.trace = trace;
    L.k.trace_cap = trace ? trace_cap : 0;
    if (mlog.log) {
        if (mlog.walkers < 1 || mlog.walkers > p->n_walkers)
            return fail(HEVMC_EINVAL, "log_walkers = %d must be in [1, n_walkers = %d]", mlog.walkers, p->n_walkers);
        if (mlog.cap < 1)
            return fail(HEVMC_EINVAL, "log_cap = %lld must be >= 1", (long long)mlog.cap);
        L.k.movelog = mlog.log;
        L.k.log_walkers = mlog.walkers;
        L.k.log_cap = mlog.cap;
    }
    if (!coords || !acc)
        return fail(HEVMC_EINVAL, "coords and acc must be device pointers");
    if (n_sweeps < 0)
        return fail(HEVMC_EINVAL, "n_sweeps = %d must be >= 0", n_sweeps);
    if (energy_every < 0)
        return fail(HEVMC_EINVAL, "energy_every = %d must be >= 0", energy_every);
    if ((uint64_t)sweep0 + (uint64_t)n_sweeps > 0xFFFFFFFFull)
        return fail(HEVMC_EINVAL, "sweep counter would pass 2^32 - 1");
    if (n_sweeps == 0)
        return HEVMC_OK;
    if (L.spread)
        return sweep_spread(L, p, coords, acc, sweep0, n_sweeps, measure_start, energy_every, mlog);
    L.k.share_tag = shares_cu(L) ? next_share_tag() : 0u;
    return launched(launch_sweep(L, coords, acc, rows, sweep0, n_sweeps, measure_start, energy_every),
                    "sweep kernel launch");
}

extern "C" hevmc_status hevmc_sweep(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                                    uint32_t sweep0, int32_t n_sweeps, uint32_t measure_start, int32_t energy_every,
                                    void *stream)
{
    return sweep_with(p, coords, acc, rows, nullptr, 0, nullptr, 0, sweep0, n_sweeps, measure_start, energy_every,
                      stream);
}

extern "C" hevmc_status hevmc_sweep_gr(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                                       uint64_t *gr, int32_t gr_bins, uint32_t sweep0, int32_t n_sweeps,
                                       uint32_t measure_start, int32_t energy_every, void *stream)
{
    return sweep_with(p, coords, acc, rows, gr, gr_bins, nullptr, 0, sweep0, n_sweeps, measure_start, energy_every,
                      stream);
}

extern "C" hevmc_status hevmc_sweep_trace(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                                          double *trace, int32_t trace_cap, uint32_t sweep0, int32_t n_sweeps,
                                          uint32_t measure_start, int32_t energy_every, void *stream)
{
    return sweep_with(p, coords, acc, rows, nullptr, 0, trace, trace_cap, sweep0, n_sweeps, measure_start,
                      energy_every, stream);
}

extern "C" hevmc_status hevmc_sweep_log(const hevmc_params *p, void *coords, hevmc_walker_acc *acc, double *rows,
                                        double *log, int32_t log_walkers, int64_t log_cap, uint32_t sweep0,
                                        int32_t n_sweeps, uint32_t measure_start, int32_t energy_every, void *stream)
{
    if (!log)
        return fail(HEVMC_EINVAL, "log must be a device pointer");
    MoveLog ml;
    ml.log = log;
    ml.walkers = log_walkers;
    ml.cap = log_cap;
    return sweep_with(p, coords, acc, rows, nullptr, 0, nullptr, 0, sweep0, n_sweeps, measure_start, energy_every,
                      stream, ml);
}

extern "C" hevmc_status hevmc_sweep_batch(int32_t n_requests, const hevmc_request *requests, const int32_t *map,
                                          int32_t n_slots, void *coords, hevmc_walker_acc *acc, double *rows,
                                          int32_t n_sweeps, void *stream)
{
    if (n_requests < 1 || n_requests > HEVMC_MAX_BATCH)
        return fail(HEVMC_EINVAL, "n_requests = %d must be in [1, %d]", n_requests, HEVMC_MAX_BATCH);
    if (!requests || !map || !coords || !acc)
        return fail(HEVMC_EINVAL, "requests, map, coords and acc must not be NULL");
    if (n_slots < 1)
        return fail(HEVMC_EINVAL, "n_slots = %d must be >= 1", n_slots);
    if (n_sweeps < 0)
        return fail(HEVMC_EINVAL, "n_sweeps = %d must be >= 0", n_sweeps);
    const hevmc_params &p0 = requests[0].params;
    BatchArgs b = {};
    b.count = n_requests;
    for (int r = 0; r < n_requests; ++r) {
        const hevmc_request &q = requests[r];
        hevmc_status st = check_params(&q.params);
        if (st != HEVMC_OK)
            return fail(st, "request %d: %s", r, g_err.c_str());
        if (q.params.n != p0.n || q.params.precision != p0.precision || q.params.threads != p0.threads ||
            q.params.variant != p0.variant)
            return fail(HEVMC_EINVAL, "request %d differs from request 0 in n, precision, threads or variant", r);
        if (q.energy_every < 0)
            return fail(HEVMC_EINVAL, "request %d: energy_every = %d must be >= 0", r, q.energy_every);
        if ((uint64_t)q.sweep0 + (uint64_t)n_sweeps > 0xFFFFFFFFull)
            return fail(HEVMC_EINVAL, "request %d: sweep counter would pass 2^32 - 1", r);
        make_kparams(&q.params, b.k[r]);
        b.sweep0[r] = q.sweep0;
        b.mstart[r] = q.measure_start;
        b.m[r] = q.energy_every;
    }
    hevmc_params shape = p0;
    shape.n_walkers = n_slots;
    Launch L;
    hevmc_status st = plan(&shape, stream, L);
    if (st != HEVMC_OK)
        return st;
    // the batched kernels keep rows in LDS or not at all: a walker whose rows
    // would need registers runs the plain sweep here (same LDS layout)
    if (L.rreg) {
        L.rows = false;
        L.rreg = false;
    }
    if (n_sweeps == 0)
        return HEVMC_OK;
    // every slot of the launch runs n_sweeps sweeps of the same N, so their
    // progress is comparable: one tag for all requests
    const uint32_t tag = shares_cu(L) ? next_share_tag() : 0u;
    for (int r = 0; r < n_requests; ++r) {
        b.k[r].sorted = L.k.sorted;
        b.k[r].share_tag = tag;
    }
    return launched(launch_sweep_batch(L, b, map, n_slots, coords, acc, rows, n_sweeps), "batched sweep launch");
}

extern "C" hevmc_status hevmc_local_energy(const hevmc_params *p, const void *coords, double *out, void *stream)
{
    Launch L;
    hevmc_status st = plan(p, stream, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    if (!coords || !out)
        return fail(HEVMC_EINVAL, "coords and out must be device pointers");
    if (L.spread)
        return spread_energy(L, coords, nullptr, out, 2);
    return launched(launch_local_energy(L, coords, out), "local-energy kernel launch");
}

extern "C" hevmc_status hevmc_pair_histogram(const hevmc_params *p, const void *coords, int32_t n_bins,
                                            uint64_t *counts, void *stream)
{
    if (n_bins < 1 || n_bins > HEVMC_MAX_GR_BINS)
        return fail(HEVMC_EINVAL, "n_bins = %d must be in [1, %d]", n_bins, HEVMC_MAX_GR_BINS);
    Launch L;
    hevmc_status st = plan(p, stream, L);
    if (st != HEVMC_OK)
        return st;
    if (!coords || !counts)
        return fail(HEVMC_EINVAL, "coords and counts must be device pointers");
    const size_t tsz = p->precision == HEVMC_FP32 ? sizeof(float) : sizeof(double);
    DeviceLimits d;
    if ((st = device_limits(d)) != HEVMC_OK)
        return st;
    if (hist_lds_offset(p->n, tsz, false, false) + (size_t)n_bins * sizeof(uint32_t) + 1024 > d.lds_per_block)
        return fail(HEVMC_ENOFIT, "a %d-atom configuration and %d bins do not fit in one workgroup's LDS", p->n,
                    n_bins);
    L.k.gr_bins = n_bins;
    return launched(launch_pair_hist(L, coords, counts), "pair-histogram kernel launch");
}

extern "C" hevmc_status hevmc_move_delta(const hevmc_params *p, const void *coords, const int32_t *s,
                                         const double *delta, double *out, void *stream)
{
    Launch L;
    hevmc_status st = plan(p, stream, L);
    if (st != HEVMC_OK)
        return st;
    if (!coords || !s || !delta || !out)
        return fail(HEVMC_EINVAL, "coords, s, delta and out must be device pointers");
    return launched(launch_move_delta(L, coords, s, delta, out), "move-delta kernel launch");
}

extern "C" hevmc_status hevmc_draw_moves(const hevmc_params *p, uint32_t sweep, int32_t *s_out, double *xi_out,
                                         double *delta_out, void *stream)
{
    Launch L;
    hevmc_status st = plan(p, stream, L);
    if (st != HEVMC_OK)
        return st;
    if (!s_out || !xi_out || !delta_out)
        return fail(HEVMC_EINVAL, "s_out, xi_out and delta_out must be device pointers");
    if ((long long)p->n * (long long)p->n_walkers > 0x7FFFFFFFLL)
        return fail(HEVMC_EINVAL, "n * n_walkers too large for one call");
    return launched(launch_draw_moves(L, sweep, s_out, xi_out, delta_out), "draw kernel launch");
}

// ---------------------------------------------------------------------------
// Ensemble layer.

struct hevmc_ensemble {
    hevmc_params p;
    hipStream_t stream;
    void *coords;
    hevmc_walker_acc *acc;
    double *rows;       // row sums kept between launches (always owned), or null
    bool owns;          // coords and acc allocated by the library
    uint32_t sweep;
    uint32_t mstart;
    std::atomic<bool> busy{false};   // a call on the ensemble is running
};

namespace {

// Holds an ensemble for the duration of one call; a second call on another
// thread meanwhile gets HEVMC_EBUSY instead of racing on its state.
struct EnsembleHold {
    hevmc_ensemble *e;
    bool held;
    explicit EnsembleHold(hevmc_ensemble *e_) : e(e_), held(e_ && !e_->busy.exchange(true)) {}
    ~EnsembleHold()
    {
        if (held)
            e->busy.store(false);
    }
    hevmc_status refused() const
    {
        return fail(HEVMC_EBUSY, "the ensemble is in use by a call on another thread");
    }
};

}  // namespace

namespace {

hevmc_status check_host_coords(const hevmc_params *p, const double *xyz, size_t count)
{
    const double L = box_side(p);
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(xyz[i]) || xyz[i] < 0.0 || xyz[i] >= L)
            return fail(HEVMC_EINVAL, "coordinate %zu = %g is not in [0, L = %.17g)", i, xyz[i], L);
    return HEVMC_OK;
}

hevmc_status upload_coords(const hevmc_params *p, const double *xyz, size_t count, void *dev, hipStream_t st)
{
    hipError_t e;
    if (p->precision == HEVMC_FP32) {
        std::vector<float> tmp(count);
        const float Lf = (float)box_side(p);
        for (size_t i = 0; i < count; ++i) {
            float v = (float)xyz[i];
            tmp[i] = v < Lf ? v : 0.0f;   // a value just below L may round up to L
        }
        e = hipMemcpyAsync(dev, tmp.data(), count * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
    } else {
        e = hipMemcpyAsync(dev, xyz, count * sizeof(double), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
    }
    return e == hipSuccess ? HEVMC_OK : hip_fail(e, "coordinate upload");
}

}  // namespace

extern "C" hevmc_status hevmc_create(const hevmc_params *p, const double *init_xyz, void *stream,
                                     hevmc_ensemble **out)
{
    Launch L;
    hevmc_status st = plan(p, stream, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    if (!out)
        return fail(HEVMC_EINVAL, "out is NULL");
    const size_t count = (size_t)p->n_walkers * 3 * (size_t)p->n;
    if (init_xyz && (st = check_host_coords(p, init_xyz, count)) != HEVMC_OK)
        return st;
    auto *e = new (std::nothrow) hevmc_ensemble();
    if (!e)
        return fail(HEVMC_ENOMEM, "host allocation failed");
    e->p = *p;
    e->stream = (hipStream_t)stream;
    e->owns = true;
    e->sweep = 0;
    e->mstart = 0xFFFFFFFFu;
    const size_t cbytes = count * (p->precision == HEVMC_FP32 ? sizeof(float) : sizeof(double));
    hipError_t he = hipMalloc(&e->coords, cbytes);
    if (he != hipSuccess) {
        delete e;
        return fail(HEVMC_ENOMEM, "hipMalloc of %zu B for coordinates failed", cbytes);
    }
    he = hipMalloc((void **)&e->acc, sizeof(hevmc_walker_acc) * (size_t)p->n_walkers);
    if (he == hipSuccess)
        he = hipMalloc((void **)&e->rows, sizeof(double) * (size_t)p->n * (size_t)p->n_walkers);
    if (he != hipSuccess) {
        (void)hipFree(e->coords);
        (void)hipFree(e->acc);
        delete e;
        return fail(HEVMC_ENOMEM, "hipMalloc of walker state failed");
    }
    if (init_xyz)
        st = upload_coords(p, init_xyz, count, e->coords, e->stream);
    if (st == HEVMC_OK)
        st = hevmc_init_walkers(p, e->coords, e->acc, e->rows, init_xyz ? 0 : 1, stream);
    if (st == HEVMC_OK) {
        he = hipStreamSynchronize(e->stream);
        if (he != hipSuccess)
            st = hip_fail(he, "initialisation");
    }
    if (st != HEVMC_OK) {
        std::string msg = g_err;
        hevmc_destroy(e);
        g_err = msg;
        return st;
    }
    *out = e;
    return HEVMC_OK;
}

extern "C" hevmc_status hevmc_create_on(const hevmc_params *p, void *dev_coords, hevmc_walker_acc *dev_acc,
                                        void *stream, hevmc_ensemble **out)
{
    Launch L;
    hevmc_status st = plan(p, stream, L, 0, true);
    if (st != HEVMC_OK)
        return st;
    if (!out || !dev_coords || !dev_acc)
        return fail(HEVMC_EINVAL, "out, dev_coords and dev_acc must not be NULL");
    auto *e = new (std::nothrow) hevmc_ensemble();
    if (!e)
        return fail(HEVMC_ENOMEM, "host allocation failed");
    e->p = *p;
    e->stream = (hipStream_t)stream;
    e->coords = dev_coords;
    e->acc = dev_acc;
    e->rows = nullptr;
    e->owns = false;
    e->sweep = 0;
    e->mstart = 0xFFFFFFFFu;
    // the row sums of the row-sum sweep persist between runs in a buffer of
    // the ensemble's own (8 N W bytes), as for hevmc_create
    if (L.rows || L.rreg) {
        const size_t rbytes = sizeof(double) * (size_t)p->n * (size_t)p->n_walkers;
        if (hipMalloc((void **)&e->rows, rbytes) != hipSuccess) {
            delete e;
            return fail(HEVMC_ENOMEM, "hipMalloc of %zu B for row sums failed", rbytes);
        }
    }
    st = hevmc_init_walkers(p, dev_coords, dev_acc, e->rows, 0, stream);
    if (st != HEVMC_OK) {
        std::string msg = g_err;
        hevmc_destroy(e);
        g_err = msg;
        return st;
    }
    *out = e;
    return HEVMC_OK;
}

extern "C" hevmc_status hevmc_run(hevmc_ensemble *e, int32_t n_sweeps, int32_t energy_every, int32_t measure)
{
    if (!e)
        return fail(HEVMC_EINVAL, "ensemble is NULL");
    EnsembleHold hold(e);
    if (!hold.held)
        return hold.refused();
    if (n_sweeps < 0)
        return fail(HEVMC_EINVAL, "n_sweeps = %d must be >= 0", n_sweeps);
    if (measure && e->mstart == 0xFFFFFFFFu)
        e->mstart = e->sweep;
    const uint32_t mstart = measure ? e->mstart : 0xFFFFFFFFu;
    hevmc_status st =
        hevmc_sweep(&e->p, e->coords, e->acc, e->rows, e->sweep, n_sweeps, mstart, energy_every, e->stream);
    if (st == HEVMC_OK)
        e->sweep += (uint32_t)n_sweeps;
    return st;
}

namespace {

hevmc_status get_acc(hevmc_ensemble *e, hevmc_walker_acc *host_out)
{
    hipError_t he = hipMemcpyAsync(host_out, e->acc, sizeof(hevmc_walker_acc) * (size_t)e->p.n_walkers,
                                   hipMemcpyDeviceToHost, e->stream);
    if (he == hipSuccess)
        he = hipStreamSynchronize(e->stream);
    if (he != hipSuccess)
        return hip_fail(he, "accumulator download");
    for (int w = 0; w < e->p.n_walkers; ++w) {
        const hevmc_walker_acc &a = host_out[w];
        const double vals[] = {a.u_run, a.v_run, a.sum_e, a.sum_e2, a.sum_v, a.sum_tpb, a.sum_tjf, a.sum_tf, a.sum_vs};
        for (double v : vals)
            if (!std::isfinite(v))
                return fail(HEVMC_ESTATE, "walker %d has a non-finite running state or accumulator", w);
    }
    return HEVMC_OK;
}

}  // namespace

extern "C" hevmc_status hevmc_get_acc(hevmc_ensemble *e, hevmc_walker_acc *host_out)
{
    if (!e || !host_out)
        return fail(HEVMC_EINVAL, "ensemble and host_out must not be NULL");
    EnsembleHold hold(e);
    if (!hold.held)
        return hold.refused();
    return get_acc(e, host_out);
}

extern "C" hevmc_status hevmc_sync(hevmc_ensemble *e)
{
    if (!e)
        return fail(HEVMC_EINVAL, "ensemble is NULL");
    EnsembleHold hold(e);
    if (!hold.held)
        return hold.refused();
    std::vector<hevmc_walker_acc> tmp((size_t)e->p.n_walkers);
    return get_acc(e, tmp.data());
}

extern "C" hevmc_status hevmc_get_coords(hevmc_ensemble *e, double *host_out)
{
    if (!e || !host_out)
        return fail(HEVMC_EINVAL, "ensemble and host_out must not be NULL");
    EnsembleHold hold(e);
    if (!hold.held)
        return hold.refused();
    const size_t count = (size_t)e->p.n_walkers * 3 * (size_t)e->p.n;
    hipError_t he;
    if (e->p.precision == HEVMC_FP32) {
        std::vector<float> tmp(count);
        he = hipMemcpyAsync(tmp.data(), e->coords, count * sizeof(float), hipMemcpyDeviceToHost, e->stream);
        if (he == hipSuccess)
            he = hipStreamSynchronize(e->stream);
        for (size_t i = 0; i < count; ++i)
            host_out[i] = tmp[i];
    } else {
        he = hipMemcpyAsync(host_out, e->coords, count * sizeof(double), hipMemcpyDeviceToHost, e->stream);
        if (he == hipSuccess)
            he = hipStreamSynchronize(e->stream);
    }
    return he == hipSuccess ? HEVMC_OK : hip_fail(he, "coordinate download");
}

extern "C" hevmc_status hevmc_get_sweep(hevmc_ensemble *e, uint32_t *sweep_out)
{
    if (!e || !sweep_out)
        return fail(HEVMC_EINVAL, "ensemble and sweep_out must not be NULL");
    EnsembleHold hold(e);
    if (!hold.held)
        return hold.refused();
    *sweep_out = e->sweep;
    return HEVMC_OK;
}

extern "C" hevmc_status hevmc_destroy(hevmc_ensemble *e)
{
    if (!e)
        return HEVMC_OK;
    if (e->busy.exchange(true))
        return fail(HEVMC_EBUSY, "the ensemble is in use by a call on another thread; not destroyed");
    hevmc_status st = HEVMC_OK;
    if (e->owns || e->rows) {
        hipError_t he = hipStreamSynchronize(e->stream);
        if (he != hipSuccess)
            st = hip_fail(he, "synchronise before free");
    }
    if (e->owns) {
        (void)hipFree(e->coords);
        (void)hipFree(e->acc);
    }
    (void)hipFree(e->rows);
    delete e;
    return st;
}

extern "C" hevmc_status hevmc_eval_config(const hevmc_params *p, const double *xyz, int32_t s,
                                          const double delta[3], double *d_u, double *d_v, double out_el[6])
{
    if (!p)
        return fail(HEVMC_EINVAL, "params is NULL");
    hevmc_params q = *p;
    q.n_walkers = 1;
    Launch L;
    hevmc_status st = plan(&q, nullptr, L);
    if (st != HEVMC_OK)
        return st;
    if (!xyz || !delta || !d_u || !d_v || !out_el)
        return fail(HEVMC_EINVAL, "xyz, delta, d_u, d_v and out_el must not be NULL");
    if (s < 0 || s >= q.n)
        return fail(HEVMC_EINVAL, "s = %d is not in [0, %d)", s, q.n);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(delta[a]))
            return fail(HEVMC_EINVAL, "delta[%d] is not finite", a);
    const size_t count = 3 * (size_t)q.n;
    if ((st = check_host_coords(&q, xyz, count)) != HEVMC_OK)
        return st;
    const size_t cbytes = count * (q.precision == HEVMC_FP32 ? sizeof(float) : sizeof(double));
    void *dc = nullptr;
    int32_t *ds = nullptr;
    double *dd = nullptr, *dout = nullptr;
    hipError_t he = hipMalloc(&dc, cbytes);
    if (he == hipSuccess)
        he = hipMalloc((void **)&ds, sizeof(int32_t));
    if (he == hipSuccess)
        he = hipMalloc((void **)&dd, 3 * sizeof(double));
    if (he == hipSuccess)
        he = hipMalloc((void **)&dout, 8 * sizeof(double));
    if (he != hipSuccess) {
        st = fail(HEVMC_ENOMEM, "hipMalloc failed in hevmc_eval_config");
    } else {
        st = upload_coords(&q, xyz, count, dc, nullptr);
        if (st == HEVMC_OK) {
            he = hipMemcpy(ds, &s, sizeof(int32_t), hipMemcpyHostToDevice);
            if (he == hipSuccess)
                he = hipMemcpy(dd, delta, 3 * sizeof(double), hipMemcpyHostToDevice);
            if (he != hipSuccess)
                st = hip_fail(he, "argument upload");
        }
        if (st == HEVMC_OK)
            st = launched(launch_move_delta(L, dc, ds, dd, dout), "move-delta kernel launch");
        if (st == HEVMC_OK)
            st = launched(launch_local_energy(L, dc, dout + 2), "local-energy kernel launch");
        if (st == HEVMC_OK) {
            double host[8];
            he = hipMemcpy(host, dout, 8 * sizeof(double), hipMemcpyDeviceToHost);
            if (he != hipSuccess) {
                st = hip_fail(he, "result download");
            } else {
                *d_u = host[0];
                *d_v = host[1];
                for (int i = 0; i < 6; ++i)
                    out_el[i] = host[2 + i];
            }
        }
    }
    (void)hipFree(dc);
    (void)hipFree(ds);
    (void)hipFree(dd);
    (void)hipFree(dout);
    return st;
}

// ---------------------------------------------------------------------------
// hevmc_eval_config_noalloc: hevmc_eval_config with its staging buffers in a
// fixed device array instead of hipMalloc'ed memory.
//
// Layout of the array (doubles): [0, 3 NMAX) the configuration (doubles for
// FP64, floats for FP32 from the same base), then one slot for s (int32), three
// for delta and eight for the results (dU, dV, then the six local-energy
// quantities).  Every call overwrites everything it reads back, so nothing has
// to start at zero.  One copy per device, shared by all calls on that device:
// calls that overlap on one device race.
namespace {

constexpr int kNoallocSlotS = 3 * HEVMC_NOALLOC_MAX_N;
constexpr int kNoallocSlotDelta = kNoallocSlotS + 1;
constexpr int kNoallocSlotOut = kNoallocSlotDelta + 3;
constexpr int kNoallocDoubles = kNoallocSlotOut + 8;

}  // namespace

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of scratch (hipGetSymbolAddress,
// once per device, with that device current).  Host code uses only this
// address: the array's own name is a host-side stand-in.
hevmc_status scratch_on_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HEVMC_EDEVICE, "device %d is beyond the %d devices the no-alloc scratch serves", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return HEVMC_OK;
}

}  // namespace

extern "C" hevmc_status hevmc_eval_config_noalloc(const hevmc_params *p, const double *xyz, int32_t s,
                                                  const double delta[3], double *d_u, double *d_v,
                                                  double out_el[6])
{
    if (!p)
        return fail(HEVMC_EINVAL, "params is NULL");
    if (p->n > HEVMC_NOALLOC_MAX_N)
        return fail(HEVMC_EINVAL, "n = %d exceeds the %d atoms the no-alloc scratch holds", p->n,
                    HEVMC_NOALLOC_MAX_N);
    hevmc_params q = *p;
    q.n_walkers = 1;
    Launch L;
    hevmc_status st = plan(&q, nullptr, L);
    if (st != HEVMC_OK)
        return st;
    if (!xyz || !delta || !d_u || !d_v || !out_el)
        return fail(HEVMC_EINVAL, "xyz, delta, d_u, d_v and out_el must not be NULL");
    if (s < 0 || s >= q.n)
        return fail(HEVMC_EINVAL, "s = %d is not in [0, %d)", s, q.n);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(delta[a]))
            return fail(HEVMC_EINVAL, "delta[%d] is not finite", a);
    const size_t count = 3 * (size_t)q.n;
    if ((st = check_host_coords(&q, xyz, count)) != HEVMC_OK)
        return st;
    double *sc = nullptr;
    if ((st = scratch_on_current_device(&sc)) != HEVMC_OK)
        return st;
    void *dc = sc;
    int32_t *ds = reinterpret_cast<int32_t *>(sc + kNoallocSlotS);
    double *dd = sc + kNoallocSlotDelta, *dout = sc + kNoallocSlotOut;
    hipError_t he = hipSuccess;
    if (q.precision == HEVMC_FP32) {
        // rounded to float on the host through a fixed stack buffer, chunk by chunk
        float tmp[1024];
        const float Lf = (float)box_side(&q);
        float *dst = static_cast<float *>(dc);
        for (size_t i0 = 0; i0 < count && he == hipSuccess; i0 += 1024) {
            const size_t m = std::min<size_t>(1024, count - i0);
            for (size_t i = 0; i < m; ++i) {
                const float v = (float)xyz[i0 + i];
                tmp[i] = v < Lf ? v : 0.0f;   // a value just below L may round up to L
            }
            he = hipMemcpy(dst + i0, tmp, m * sizeof(float), hipMemcpyHostToDevice);
        }
    } else {
        he = hipMemcpy(dc, xyz, count * sizeof(double), hipMemcpyHostToDevice);
    }
    if (he == hipSuccess)
        he = hipMemcpy(ds, &s, sizeof(int32_t), hipMemcpyHostToDevice);
    if (he == hipSuccess)
        he = hipMemcpy(dd, delta, 3 * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess)
        return hip_fail(he, "argument upload");
    if ((st = launched(launch_move_delta(L, dc, ds, dd, dout), "move-delta kernel launch")) != HEVMC_OK)
        return st;
    if ((st = launched(launch_local_energy(L, dc, dout + 2), "local-energy kernel launch")) != HEVMC_OK)
        return st;
    double host[8];
    he = hipMemcpy(host, dout, 8 * sizeof(double), hipMemcpyDeviceToHost);
    if (he != hipSuccess)
        return hip_fail(he, "result download");
    *d_u = host[0];
    *d_v = host[1];
    for (int i = 0; i < 6; ++i)
        out_el[i] = host[2 + i];
    return HEVMC_OK;
}
