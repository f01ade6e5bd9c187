// Kernel arguments and launch helpers of the binned map-maker (map_kernel.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pisco {

struct MapAccumArgs {
    int64_t nside, npix, n;
    const double *theta, *phi, *psi, *hwp;   // hwp may be null
    double zeta;
    double c_int, c_pol;                     // s (1 + eps) / 2, s (1 - eps) / 2
    double *accum;                           // [npix][10]
};

struct MapSolveArgs {
    int64_t npix;
    const double *accum;                     // [npix][10]
    double rcond_min;
    double *maps;                            // [3][npix]
    double *rcond;                           // [npix] or null
};

hipError_t launch_map_accumulate(const MapAccumArgs &a, const void *tod, bool f64, int num_cu, hipStream_t s);
hipError_t launch_map_solve(const MapSolveArgs &a, int num_cu, hipStream_t s);

}  // namespace pisco
