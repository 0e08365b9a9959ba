// Host/device shared declarations internal to libhevmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hevmc.h"
#include "hevmc_device.hpp"

namespace hevmc {

// Atoms per lane the row-sum variant of the sweep supports (its forward terms
// are kept in registers): N <= kRowsPerLane * threads.
constexpr int kRowsPerLane = 8;
// Atoms per lane whose rows the rows-in-registers sweep can hold.
constexpr int kRegChunks = 22;

// Walkers per workgroup of the one-wave-per-walker sweep (threads = 64).
constexpr int kWalkersPerGroup = 4;

// Byte offset of the row sums behind the coordinates in a walker's LDS.
__host__ __device__ constexpr size_t rows_lds_offset(int n, size_t tsize)
{
    return ((size_t)3 * (size_t)n * tsize + 15) & ~(size_t)15;
}

// Spatial order of a walker's atoms in LDS (sweeps with KParams::sorted):
// sort keys (Morton code of the atom's cell << 16 | atom label), padded to a
// power of two, then slot_of[label] (uint16).  They follow the coordinates, or
// the row sums of the row-sum variant.
constexpr int kSortCells = 16;   // cells per box side for the Morton code
__host__ __device__ constexpr int sort_keys(int n)
{
    int k = 1;
    while (k < n)
        k <<= 1;
    return k;
}
__host__ __device__ constexpr size_t sort_lds_offset(int n, size_t tsize, bool rows)
{
    return rows ? (rows_lds_offset(n, tsize) + (size_t)n * sizeof(double) + 15) & ~(size_t)15
                : ((size_t)3 * (size_t)n * tsize + 15) & ~(size_t)15;
}
__host__ __device__ constexpr size_t slot_of_lds_offset(int n, size_t tsize, bool rows)
{
    return sort_lds_offset(n, tsize, rows) + (size_t)sort_keys(n) * sizeof(uint32_t);
}
__host__ __device__ constexpr size_t sorted_walker_lds(int n, size_t tsize, bool rows)
{
    return slot_of_lds_offset(n, tsize, rows) + (size_t)n * sizeof(uint16_t);
}

// Byte offset of the pair histogram (uint32 [gr_bins]) in a walker's LDS,
// behind everything else the sweep keeps there.
__host__ __device__ constexpr size_t hist_lds_offset(int n, size_t tsize, bool rows, bool sorted)
{
    return ((sorted ? sorted_walker_lds(n, tsize, rows)
                    : rows ? rows_lds_offset(n, tsize) + (size_t)n * sizeof(double) : (size_t)3 * n * tsize) +
            15) &
           ~(size_t)15;
}

// Per-request constants of a batched sweep, passed by value in the kernel
// arguments (at most HEVMC_MAX_BATCH requests per launch).
struct BatchArgs {
    KParams k[HEVMC_MAX_BATCH];
    uint32_t sweep0[HEVMC_MAX_BATCH];
    uint32_t mstart[HEVMC_MAX_BATCH];
    int32_t m[HEVMC_MAX_BATCH];
    int32_t count;
};

// The mailbox of a cooperative sweep of spread walkers (walkers whose
// coordinates do not fit in one workgroup's LDS): per walker, the partial
// Eq. (7) sums of its C slices for the two parities of the micro-update
// counter ([W][2][C][2] doubles) and an arrival counter ([W], zero at launch);
// status becomes nonzero if a wait gave up after spin_cap polls.
// The cooperative sweep's exchange: per walker two rows of 4C + 8 mailbox
// words (zeroed before each launch), and a status word set by a workgroup
// whose wait gave up.
struct CoopArgs {
    uint64_t *mail;
    uint32_t *status;
    uint32_t spin_cap;
    int32_t C;          // workgroups (slices) per walker
    int32_t S;          // atoms per slice (the last may hold fewer)
    int64_t log_base;   // per-move records: micro-updates of the call before this launch
};

struct LaunchShape {
    int n_walkers_grid;  // workgroups (walkers) in the grid
};

// Everything a launcher needs: validated kernel constants and launch shape.
struct Launch {
    KParams k;
    LaunchShape p;
    int threads;        // threads per walker workgroup
    bool fp32;
    bool rows;          // row-sum variant of the sweep
    bool rreg;          // its rows in registers (walkers whose rows do not fit in LDS)
    size_t lds_bytes;   // dynamic LDS per workgroup of the sweep kernel
    size_t walker_lds;  // dynamic LDS of one walker (the per-walker kernels)
    hipStream_t stream;
    bool spread = false;  // the walker does not fit in one workgroup's LDS: C slices
    int slices = 1;       // C
    int slice_atoms = 0;  // S
};

hipError_t launch_sweep(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, uint32_t sweep0,
                        int32_t nsw, uint32_t mstart, int32_t m);
hipError_t launch_sweep_batch(const Launch &L, const BatchArgs &b, const int32_t *map, int32_t n_slots,
                              void *coords, hevmc_walker_acc *acc, double *rows, int32_t nsw);
hipError_t launch_local_energy(const Launch &L, const void *coords, double *out);
hipError_t launch_pair_hist(const Launch &L, const void *coords, uint64_t *counts);
hipError_t launch_init(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, int fcc, int nc,
                       double a_lat);
hipError_t launch_move_delta(const Launch &L, const void *coords, const int32_t *s, const double *d,
                             double *out);
hipError_t launch_draw_moves(const Launch &L, uint32_t t, int32_t *s, double *xi, double *d);
// Spread walkers: the cooperative sweep of `walkers` walkers from coords and
// acc (already offset), the one-workgroup-per-walker local energy in device
// memory (mode 0 start, 1 sample, 2 values to out), the fcc start, and the
// cooperative kernel's workgroups per compute unit.
hipError_t launch_sweep_coop(const Launch &L, const CoopArgs &c, void *coords, hevmc_walker_acc *acc,
                             uint32_t sweep0, int32_t nsw, uint32_t mstart, int32_t walkers);
// Local energy of spread walkers (mode 0 start, 1 sample, 2 values to out),
// with part a device buffer of energy_blocks(W, N) x W x 5 doubles.
int energy_blocks(int n_walkers, int n);
hipError_t launch_energy_global(const Launch &L, const void *coords, hevmc_walker_acc *acc, double *out, int mode,
                                double *part);
hipError_t launch_fcc_global(const Launch &L, void *coords, int nc, double a_lat);
hipError_t coop_blocks_per_cu(const Launch &L, int *blocks_per_cu);

// Registers per thread and static LDS bytes of the sweep kernel for
// (precision, threads, variant); zeros if unknown.
struct SweepAttrs {
    int vgprs;
    int static_lds;
};
SweepAttrs sweep_attrs(bool fp32, int threads, bool rows, bool rreg = false);
// Whether (precision, threads) has the rows-in-registers sweep.
bool rreg_form(bool fp32, int threads);

}  // namespace hevmc
