// Binned map-making on the GPU: per-sample accumulation of the per-pixel
// normal equations (FP64 atomics) and the per-pixel 3 x 3 solve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "map_internal.h"

namespace pisco {
namespace {

constexpr double TWO_OVER_PI = 0.63661977236758134308;

// RING pixel holding (theta, phi), from the HEALPix tiling (Gorski et al.
// 2005, Sec. 4): with t = 2 phi / pi in [0, 4), the equatorial belt is cut by
// the line families N (1/2 + t) -/+ (3/4) N z = integer (their indices give
// the ring from z = 2/3 and the place along it), the polar caps by
// tp w and (1 - tp) w = integer with w = N sqrt(3 (1 - |z|)) and tp the place
// in the quadrant (their sum gives the ring from the pole).
__device__ inline int64_t ring_pixel(int64_t N, double theta, double phi) {
    const double z = cos(theta), az = fabs(z);
    double t = fmod(phi * TWO_OVER_PI, 4.0);
    if (t < 0.0) t += 4.0;
    const double fN = (double)N;
    if (az <= 2.0 / 3.0) {
        const double u = fN * (0.5 + t), v = 0.75 * fN * z;
        const int64_t up = (int64_t)floor(u - v), dn = (int64_t)floor(u + v);
        const int64_t r = N + 1 + up - dn;   // 1 .. 2N + 1, counted from z = 2/3
        int64_t k = (up + dn - N + 1 + ((r & 1) ? 0 : 1)) >> 1;
        if (k >= 4 * N) k -= 4 * N;
        return 2 * N * (N - 1) + (r - 1) * 4 * N + k;
    }
    const double w = fN * sqrt(3.0 * (1.0 - az));
    const double tp = t - floor(t);
    int64_t r = (int64_t)floor(tp * w) + (int64_t)floor((1.0 - tp) * w) + 1;   // 1 .. N, from the pole
    if (r > N) r = N;
    int64_t k = (int64_t)floor(t * (double)r);
    if (k >= 4 * r) k -= 4 * r;
    return (z > 0.0) ? 2 * r * (r - 1) + k : 12 * N * N - 2 * r * (r + 1) + k;
}

// One wave takes 64 consecutive samples per step.  Samples of a scan fall into
// the same pixel several at a time, so the wave first sums each run of lanes
// with equal pixels (a segmented scan over the lanes) and only the last lane
// of a run adds its ten sums to the pixel: far fewer atomics on the same
// addresses.  Invalid lanes form runs of their own and add nothing.
template <typename T>
__global__ void __launch_bounds__(256) map_accum_kernel(MapAccumArgs a, const T *__restrict__ tod) {
    constexpr int WV = 64;
    const int lane = threadIdx.x & (WV - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(WV - 1)); t0 < a.n; t0 += stride) {
        const int64_t t = t0 + lane;
        int32_t p = -1 - lane;
        double v[10];
        for (int k = 0; k < 10; ++k) v[k] = 0.0;
        if (t < a.n) {
            const double th = a.theta[t], ph = a.phi[t], ps = a.psi[t];
            const double hw = a.hwp ? a.hwp[t] : 0.0;
            const double d = (double)tod[t];
            if (isfinite(th) && isfinite(ph) && isfinite(ps) && isfinite(hw) && isfinite(d)) {
                const int64_t q = ring_pixel(a.nside, th, ph);
                if (q >= 0 && q < a.npix) {   // only finite directions reach here: always true
                    p = (int32_t)q;
                    double sn, cs;
                    sincos(2.0 * (ps + a.zeta) + 4.0 * hw, &sn, &cs);
                    const double w0 = a.c_int, w1 = a.c_pol * cs, w2 = a.c_pol * sn;
                    v[0] = w0 * w0;
                    v[1] = w0 * w1;
                    v[2] = w0 * w2;
                    v[3] = w1 * w1;
                    v[4] = w1 * w2;
                    v[5] = w2 * w2;
                    v[6] = w0 * d;
                    v[7] = w1 * d;
                    v[8] = w2 * d;
                    v[9] = 1.0;
                }
            }
        }
        // first lane of this lane's run: prefix maximum of the run heads
        const int32_t pu = __shfl_up(p, 1, WV);
        int start = (lane == 0 || pu != p) ? lane : 0;
#pragma unroll
        for (int off = 1; off < WV; off <<= 1) {
            const int o = __shfl_up(start, off, WV);
            if (lane >= off) start = max(start, o);
        }
        // segmented inclusive sums over [start, lane]
#pragma unroll
        for (int off = 1; off < WV; off <<= 1) {
            const bool take = lane - off >= start;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const double x = __shfl_up(v[k], off, WV);
                if (take) v[k] += x;
            }
        }
        const int32_t pd = __shfl_down(p, 1, WV);
        const bool last = (lane == WV - 1) || (pd != p);
        if (last && p >= 0) {
            double *q = a.accum + 10 * (int64_t)p;
#pragma unroll
            for (int k = 0; k < 10; ++k) unsafeAtomicAdd(q + k, v[k]);
        }
    }
}

// Extreme eigenvalues of a symmetric 3 x 3 matrix by the trigonometric form
// of the characteristic cubic's roots (Smith 1961).
__device__ inline void eig_extremes(double a00, double a01, double a02, double a11, double a12, double a22,
                                    double &lmin, double &lmax) {
    const double off = a01 * a01 + a02 * a02 + a12 * a12;
    const double m = (a00 + a11 + a22) / 3.0;
    const double d0 = a00 - m, d1 = a11 - m, d2 = a22 - m;
    const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * off;
    if (!(p2 > 0.0)) {
        lmin = lmax = m;
        return;
    }
    const double p = sqrt(p2 / 6.0), ip = 1.0 / p;
    const double b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip, b01 = a01 * ip, b02 = a02 * ip, b12 = a12 * ip;
    const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    const double ang = acos(r) / 3.0;
    lmax = m + 2.0 * p * cos(ang);
    lmin = m + 2.0 * p * cos(ang + 2.0943951023931954923);
}

__global__ void __launch_bounds__(256) map_solve_kernel(MapSolveArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npix; p += stride) {
        const double *q = a.accum + 10 * p;
        const double a00 = q[0], a01 = q[1], a02 = q[2], a11 = q[3], a12 = q[4], a22 = q[5];
        const double b0 = q[6], b1 = q[7], b2 = q[8], hits = q[9];
        double I = 0.0, Q = 0.0, U = 0.0, rc = 0.0;
        if (hits > 0.0) {
            double lmin, lmax;
            eig_extremes(a00, a01, a02, a11, a12, a22, lmin, lmax);
            rc = (lmax > 0.0) ? lmin / lmax : 0.0;
            if (rc >= a.rcond_min) {
                // adjugate (cofactors) of the symmetric matrix
                const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
                const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
                const double id = 1.0 / (a00 * c00 + a01 * c01 + a02 * c02);
                I = (c00 * b0 + c01 * b1 + c02 * b2) * id;
                Q = (c01 * b0 + c11 * b1 + c12 * b2) * id;
                U = (c02 * b0 + c12 * b1 + c22 * b2) * id;
            } else if (a00 > 0.0) {
                I = b0 / a00;
            }
        }
        a.maps[p] = I;
        a.maps[a.npix + p] = Q;
        a.maps[2 * a.npix + p] = U;
        if (a.rcond) a.rcond[p] = rc;
    }
}

int blocks_for(int64_t n, int cap) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_map_accumulate(const MapAccumArgs &a, const void *tod, bool f64, int num_cu, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const int g = blocks_for(a.n, 16 * num_cu);
    if (f64)
        hipLaunchKernelGGL((map_accum_kernel<double>), dim3(g), dim3(256), 0, s, a, static_cast<const double *>(tod));
    else
        hipLaunchKernelGGL((map_accum_kernel<float>), dim3(g), dim3(256), 0, s, a, static_cast<const float *>(tod));
    return hipGetLastError();
}

hipError_t launch_map_solve(const MapSolveArgs &a, int num_cu, hipStream_t s) {
    hipLaunchKernelGGL(map_solve_kernel, dim3(blocks_for(a.npix, 16 * num_cu)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pisco
