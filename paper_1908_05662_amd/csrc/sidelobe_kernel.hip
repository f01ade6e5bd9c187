// Device steps of training the far-sidelobe network behind the C ABI
// (pisco_sidelobe_train): training pointings drawn by a counter-based
// generator, moments and standardisation of the exact targets, and the
// per-epoch shuffle of the training rows.
#include <hip/hip_runtime.h>

#include "mlp_internal.h"
#include "sidelobe_internal.h"

namespace pisco {
namespace {

constexpr double TWO_PI = 6.28318530717958647692;

// Output k of SplitMix64 (Steele, Lea & Flood 2014) from state `seed`: the
// generator's state after k + 1 steps of the Weyl sequence, finalised.  Each
// output depends only on (seed, k), so every sample draws its own numbers.
__device__ __host__ inline uint64_t splitmix_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ inline double unit53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// Pointing i: direction uniform on the sphere (cos theta uniform in [-1, 1],
// phi uniform in [0, 2 pi)), psi uniform in [0, 2 pi); draws 3i, 3i+1, 3i+2.
__global__ void draw_kernel(uint64_t seed, int64_t n, double *th, double *ph, double *ps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double z = 2.0 * unit53(splitmix_at(seed, 3 * (uint64_t)i)) - 1.0;
    th[i] = acos(fmin(1.0, fmax(-1.0, z)));
    ph[i] = TWO_PI * unit53(splitmix_at(seed, 3 * (uint64_t)i + 1));
    ps[i] = TWO_PI * unit53(splitmix_at(seed, 3 * (uint64_t)i + 2));
}

// Mean and standard deviation of each of the three target channels over n
// rows, in FP64 with a fixed summation order (one workgroup: per-thread
// strided sums, then a tree in LDS): mean first, then the sum of squared
// deviations from it.  out = (mean[3], std[3]); std = sqrt(M2 / (n - 1)).
constexpr int MOM_THREADS = 1024;
__global__ void __launch_bounds__(MOM_THREADS) moments_kernel(const float *p, int64_t n, double *out) {
    __shared__ double red[3][MOM_THREADS];
    __shared__ double mean[3];
    const int tid = threadIdx.x;
    for (int pass = 0; pass < 2; ++pass) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int64_t i = tid; i < n; i += MOM_THREADS)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = (double)p[3 * i + c];
                if (pass == 0) {
                    s[c] += v;
                } else {
                    const double d = v - mean[c];
                    s[c] += d * d;
                }
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) red[c][tid] = s[c];
        __syncthreads();
        for (int w = MOM_THREADS / 2; w >= 1; w >>= 1) {
            if (tid < w)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + w];
            __syncthreads();
        }
        if (tid < 3) {
            if (pass == 0) {
                mean[tid] = red[tid][0] / (double)n;
                out[tid] = mean[tid];
            } else {
                out[3 + tid] = sqrt(red[tid][0] / (double)(n > 1 ? n - 1 : 1));
            }
        }
        __syncthreads();
    }
}

// t = (p - mean) / std per channel, std clamped away from zero.
__global__ void standardise_kernel(const float *p, int64_t n, const double *mom, float *t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    const int c = (int)(i % 3);
    const double sd = fmax(mom[3 + c], 1e-300);
    t[i] = (float)(((double)p[i] - mom[c]) / sd);
}

// A pseudo-random bijection of [0, n): a four-round balanced Feistel network
// on 2^(2h) >= n indices (round function: SplitMix64 output of the key and
// the half), applied again while the result is >= n (cycle walking; the
// cycle through an index below n returns below n).
__device__ inline uint64_t feistel(uint64_t v, int h, uint64_t key) {
    const uint64_t mask = (1ULL << h) - 1;
    uint64_t L = v >> h, R = v & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t F = splitmix_at(key ^ (0x632be59bd9b4e019ULL * (uint64_t)(r + 1)), R) & mask;
        const uint64_t nl = R;
        R = L ^ F;
        L = nl;
    }
    return (L << h) | R;
}

__global__ void gather_kernel(const float *x, const float *t, int64_t n, int64_t rows, int h, uint64_t key,
                              float *xs, float *ts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    uint64_t j = feistel((uint64_t)i, h, key);
    while (j >= (uint64_t)n) j = feistel(j, h, key);
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) xs[i * MLP_IN + k] = x[j * MLP_IN + k];
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) ts[i * MLP_OUT + k] = t[j * MLP_OUT + k];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

uint64_t sl_splitmix_at(uint64_t seed, uint64_t k) { return splitmix_at(seed, k); }

hipError_t sl_draw(uint64_t seed, int64_t n, double *th, double *ph, double *ps, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(draw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, seed, n, th, ph, ps);
    return hipGetLastError();
}

hipError_t sl_moments(const float *p, int64_t n, double *out6, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(MOM_THREADS), 0, s, p, n, out6);
    return hipGetLastError();
}

hipError_t sl_standardise(const float *p, int64_t n, const double *mom6, float *t, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(standardise_kernel, dim3(blocks_for(3 * n, 256)), dim3(256), 0, s, p, n, mom6, t);
    return hipGetLastError();
}

hipError_t sl_gather(const float *x, const float *t, int64_t n, int64_t rows, uint64_t key, float *xs, float *ts,
                     hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (rows > n) return hipErrorInvalidValue;
    int h = 1;
    while ((1ULL << (2 * h)) < (uint64_t)n) ++h;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, s, x, t, n, rows, h, key, xs, ts);
    return hipGetLastError();
}

}  // namespace pisco
