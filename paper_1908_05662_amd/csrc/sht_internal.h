// Kernel arguments and launch helpers of the harmonic analysis (sht_kernel.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pisco {

constexpr int SHT_MAX_NSIDE = 1024;        // ring FFT buffers (2 x 4N complex) fit one CU's LDS
constexpr int SHT_PAIRS_PER_LANE = 4;      // 512 lanes x 4 ring pairs = 2N pairs at the largest nside

struct ShtArgs {
    int nside, lmax, mmax, nfields;        // nfields: 1 (T) or 3 (T, Q, U)
    int nrings;                            // 4 nside - 1
    const double *map[3];                  // RING order, 12 nside^2 each
    double2 *F;                            // [nfields][mmax + 1][nrings]: weighted ring Fourier sums
    double *alm[3];                        // complex interleaved, m-major: T, E, B
    double *partial;                       // [SHT_WAVES][alm size][6]: per-wave partial sums
    const double *alm_in[3];               // synthesis input (complex interleaved)
    double *map_out[3];                    // synthesis output (RING order)
};

constexpr int SHT_WAVES = 8;               // waves per a_lm workgroup (one workgroup per m)

struct ClArgs {
    int lmax, nspec;                       // up to 6 spectra
    const double *x[6], *y[6];             // complex interleaved a_lm of each pair
    double *cl;                            // [nspec][lmax + 1]
};

hipError_t launch_ring_fourier(const ShtArgs &a, hipStream_t s);
hipError_t launch_alm(const ShtArgs &a, hipStream_t s);
hipError_t launch_alm2map(const ShtArgs &a, hipStream_t s);          // alm_in -> F (as G) -> map_out
hipError_t launch_axpy(double *y, const double *x, double alpha, int64_t n, bool reverse, hipStream_t s);
hipError_t launch_alm2cl(const ClArgs &a, hipStream_t s);

}  // namespace pisco
