// Host/device shared declarations internal to libhevmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hevmc.h"
#include "hevmc_device.hpp"

namespace hevmc {

struct LaunchShape {
    int n_walkers_grid;  // workgroups (walkers) in the grid
};

// Everything a launcher needs: validated kernel constants and launch shape.
struct Launch {
    KParams k;
    LaunchShape p;
    int threads;        // threads per walker workgroup
    bool fp32;
    size_t lds_bytes;   // dynamic LDS per workgroup
    hipStream_t stream;
};

hipError_t launch_sweep(const Launch &L, void *coords, hevmc_walker_acc *acc, uint32_t sweep0, int32_t nsw,
                        uint32_t mstart, int32_t m);
hipError_t launch_local_energy(const Launch &L, const void *coords, double *out);
hipError_t launch_init(const Launch &L, void *coords, hevmc_walker_acc *acc, int fcc, int nc, double a_lat);
hipError_t launch_move_delta(const Launch &L, const void *coords, const int32_t *s, const double *d,
                             double *out);
hipError_t launch_draw_moves(const Launch &L, uint32_t t, int32_t *s, double *xi, double *d);

}  // namespace hevmc
