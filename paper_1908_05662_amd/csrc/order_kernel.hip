// Spatial processing order of a pointing stream: samples sorted by the index
// of their (phi, z) cell along a Hilbert curve over a 2^16 x 2^16 grid
// (cylindrical equal-area coordinates), so that consecutive samples are close
// on the sky and 64-sample tiles are compact.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdint>

#include "pisco_internal.h"

namespace pisco {
namespace {

constexpr uint32_t GRID = 1u << 16;

// Distance along the Hilbert curve of cell (x, y) of a GRID x GRID square:
// at each scale s the quadrant adds s^2 times its rank along the curve, and
// the coordinates are turned into the quadrant's own frame.
__device__ inline uint32_t hilbert_rank(uint32_t x, uint32_t y) {
    uint32_t d = 0;
    for (uint32_t s = GRID >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = GRID - 1 - x;
                y = GRID - 1 - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

// Hilbert rank of the (phi, z) cell of one direction.
__device__ inline uint32_t cell_key(double th, double ph) {
    const double two_pi = 6.283185307179586477;
    double u = fmod(ph, two_pi) / two_pi;
    if (u < 0.0) u += 1.0;
    const double v = 0.5 * (cos(th) + 1.0);
    const double fx = floor(u * GRID), fy = floor(v * GRID);
    // non-finite pointing sorts anywhere (the convolution reports it)
    const uint32_t x = (fx >= 0.0 && fx < GRID) ? (uint32_t)fx : (fx >= GRID ? GRID - 1 : 0);
    const uint32_t y = (fy >= 0.0 && fy < GRID) ? (uint32_t)fy : (fy >= GRID ? GRID - 1 : 0);
    return hilbert_rank(x, y);
}

__global__ void order_keys_kernel(const double *__restrict__ th, const double *__restrict__ ph, int64_t n,
                                  uint32_t *__restrict__ keys, int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = cell_key(th[i], ph[i]);
    idx[i] = (int32_t)i;
}

// Key of each tile: the cell of its first sample (in processing order).
__global__ void tile_keys_kernel(const DetDesc *__restrict__ dets, const Tile *__restrict__ tiles, int32_t n,
                                 uint32_t *__restrict__ keys) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const Tile t = tiles[i];
    const DetDesc &D = dets[t.det];
    const int64_t s = D.order ? (int64_t)D.order[t.begin] : t.begin;
    keys[i] = cell_key(D.theta[s], D.phi[s]);
}

}  // namespace

hipError_t launch_tile_keys(const DetDesc *dets, const Tile *tiles, int32_t n, uint32_t *keys, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dets, tiles, n, keys);
    return hipGetLastError();
}

hipError_t spatial_order(const double *theta, const double *phi, int64_t n, int32_t *order, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > INT32_MAX) return hipErrorInvalidValue;
    uint32_t *keys = nullptr, *keys_sorted = nullptr;
    int32_t *idx = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
    hipError_t e = hipMalloc(&keys, sizeof(uint32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&keys_sorted, sizeof(uint32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&idx, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(order_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, phi, n, keys,
                           idx);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys, keys_sorted, idx, order, (int)n, 0, 32, s);
    if (e == hipSuccess) e = hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 1);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, idx, order, (int)n, 0, 32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(temp);
    (void)hipFree(idx);
    (void)hipFree(keys_sorted);
    (void)hipFree(keys);
    return e;
}

}  // namespace pisco
