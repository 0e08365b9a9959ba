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

// Byte offset of the row sums behind the coordinates in a walker's LDS.
__host__ __device__ constexpr size_t rows_lds_offset(int n, size_t tsize)
{
    return ((size_t)3 * (size_t)n * tsize + 15) & ~(size_t)15;
}

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
    size_t lds_bytes;   // dynamic LDS per workgroup
    hipStream_t stream;
};

hipError_t launch_sweep(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, uint32_t sweep0,
                        int32_t nsw, uint32_t mstart, int32_t m);
hipError_t launch_local_energy(const Launch &L, const void *coords, double *out);
hipError_t launch_init(const Launch &L, void *coords, hevmc_walker_acc *acc, double *rows, int fcc, int nc,
                       double a_lat);
hipError_t launch_move_delta(const Launch &L, const void *coords, const int32_t *s, const double *d,
                             double *out);
hipError_t launch_draw_moves(const Launch &L, uint32_t t, int32_t *s, double *xi, double *d);

// Registers per thread of the sweep kernel for (precision, threads, variant);
// 0 if unknown.
int sweep_vgprs(bool fp32, int threads, bool rows);

}  // namespace hevmc
