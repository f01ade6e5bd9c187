// Pixel-space polarised beam convolution on gfx950 (CDNA4).
//
// Operation: the pixelated convolution of Sec. 4.2 with the detector row
// folded into the beam (D(chi) Lambda(chi) = D(0), Sec. 4.1):
//   d = N sum_k [ bI I_k + bQ (c2 Q_k + s2 U_k) + bU (-s2 Q_k + c2 U_k) ],
//   c2 = cos 2chi_k, s2 = sin 2chi_k,
// over the HEALPix pixels within the disc (or annulus) around the boresight.
//
// Mapping onto the hardware:
//   * One wavefront owns a tile of consecutive samples of one detector
//     (consecutive scan samples share ~99% of their discs, so the sky and beam
//     lines they touch stay in L1/L2).  Tiles come from per-die work queues.
//   * Per sample, the 64 lanes set up 64 HEALPix rings at a time in FP64:
//     the ring's pixel interval inside the disc (one arccos per ring, no
//     per-pixel membership test) and the ring's coefficients for the pair
//     geometry.  These records and the prefix sums of the ring pixel counts
//     are staged in the wavefront's slice of LDS.
//   * The lanes then stride the flattened (ring, pixel) pairs, so neighbouring
//     lanes read neighbouring pixels of a ring: sky gathers are coalesced.
//   * Per pair, geometry is written in differences from the boresight
//     (h = 1 - cos dphi, S = sin dphi, and sin/cos of the colatitude
//     difference) so FP32 keeps relative precision on small offsets; the
//     position angle uses the great-circle carried co-polar vector (equal to
//     Ludwig's third definition, Appendix A) projected on the pixel's own
//     theta/phi basis, with no trigonometric call and no pole singularity.
//   * Sums are per-lane compensated (TwoSum) in FP32 and reduced across the
//     wavefront with shuffles; the FP64 kernel accumulates in FP64.
#include "pisco_internal.h"

#include <math.h>

namespace pisco {
namespace {

constexpr int WAVE = 64;
constexpr double PI = 3.14159265358979323846;
constexpr double TWO_PI = 6.28318530717958647692;

// ----------------------------------------------------------------------
// HEALPix RING geometry, ring-wise (Gorski et al. 2005)
// ----------------------------------------------------------------------
struct RingGeom {
    double z, s, phi0, dphi;
    int32_t first, n;
};

__device__ inline RingGeom ring_geom(int32_t N, int32_t r) {
    RingGeom g;
    const double NN = (double)N;
    if (r < N) {
        g.n = 4 * r;
        g.first = 2 * r * (r - 1);
        const double omz = (double)r * (double)r / (3.0 * NN * NN);
        g.z = 1.0 - omz;
        g.s = sqrt(omz * (2.0 - omz));
        g.phi0 = PI / (4.0 * r);
    } else if (r <= 3 * N) {
        g.n = 4 * N;
        g.first = 2 * N * (N - 1) + (r - N) * 4 * N;
        g.z = (double)(4 * N - 2 * r) / (3.0 * NN);
        g.s = sqrt((1.0 - g.z) * (1.0 + g.z));
        g.phi0 = ((r - N) & 1) ? 0.0 : PI / (4.0 * NN);
    } else {
        const int32_t rs = 4 * N - r;
        g.n = 4 * rs;
        g.first = 12 * N * N - 2 * rs * (rs + 1);
        const double opz = (double)rs * (double)rs / (3.0 * NN * NN);
        g.z = opz - 1.0;
        g.s = sqrt(opz * (2.0 - opz));
        g.phi0 = PI / (4.0 * rs);
    }
    g.dphi = TWO_PI / (double)g.n;
    return g;
}

// Continuous ring coordinate of colatitude th (inverse of the ring z formulas).
__device__ inline double ring_of_theta(int32_t N, double th) {
    const double z = cos(th);
    if (z >= 2.0 / 3.0) return (double)N * 2.449489742783178 * sin(0.5 * th);
    if (z <= -2.0 / 3.0) return 4.0 * N - (double)N * 2.449489742783178 * cos(0.5 * th);
    return (double)N * (2.0 - 1.5 * z);
}

// Pixels of ring g with cos(angular distance) >= cosr, as k in [lo, lo + cnt)
// counted from the pixel nearest the boresight longitude (cnt = n: whole ring).
__device__ inline void ring_interval(double cosr, double z0, double s0, const RingGeom &g, double dphic,
                                     int32_t &lo, int32_t &cnt) {
    const double num = cosr - g.z * z0;
    const double den = g.s * s0;
    lo = 0;
    if (den <= 0.0) {  // boresight on a pole: a ring is all in or all out
        cnt = (num <= 0.0) ? g.n : 0;
        return;
    }
    const double cm = num / den;
    if (cm > 1.0) { cnt = 0; return; }
    if (cm <= -1.0) { cnt = g.n; return; }
    const double dm = acos(cm);
    const int32_t klo = (int32_t)ceil((-dm - dphic) / g.dphi);
    const int32_t khi = (int32_t)floor((dm - dphic) / g.dphi);
    const int32_t c = khi - klo + 1;
    if (c >= g.n) { cnt = g.n; return; }
    if (c <= 0) { cnt = 0; return; }
    lo = klo;
    cnt = c;
}

// ----------------------------------------------------------------------
// Precision-dependent pieces
// ----------------------------------------------------------------------
template <typename T> struct Rec4;
template <> struct Rec4<float> { using type = float4; };
template <> struct Rec4<double> { using type = double4; };

// sin and cos of x for |x| <= pi/2 + a little.  FP32: Taylor series to x^13
// (sin) and x^14 (cos), truncation below 1e-9 on that range, keeping relative
// precision of sin near 0.  FP64: the device math library.
__device__ inline void half_sincos(float x, float &s, float &c) {
    constexpr float S3 = -1.0f / 6.0f, S5 = 1.0f / 120.0f, S7 = -1.0f / 5040.0f, S9 = 1.0f / 362880.0f,
                    S11 = -1.0f / 39916800.0f, S13 = 1.0f / 6227020800.0f;
    constexpr float C2 = -0.5f, C4 = 1.0f / 24.0f, C6 = -1.0f / 720.0f, C8 = 1.0f / 40320.0f,
                    C10 = -1.0f / 3628800.0f, C12 = 1.0f / 479001600.0f, C14 = -1.0f / 87178291200.0f;
    const float x2 = x * x;
    float ps = fmaf(x2, S13, S11);
    ps = fmaf(x2, ps, S9);
    ps = fmaf(x2, ps, S7);
    ps = fmaf(x2, ps, S5);
    ps = fmaf(x2, ps, S3);
    s = fmaf(x * x2, ps, x);
    float pc = fmaf(x2, C14, C12);
    pc = fmaf(x2, pc, C10);
    pc = fmaf(x2, pc, C8);
    pc = fmaf(x2, pc, C6);
    pc = fmaf(x2, pc, C4);
    pc = fmaf(x2, pc, C2);
    c = fmaf(x2, pc, 1.0f);
}
__device__ inline void half_sincos(double x, double &s, double &c) { sincos(x, &s, &c); }

// Per-lane accumulator: compensated (TwoSum) in FP32, plain in FP64.
template <typename T> struct Acc;
template <> struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x) {
        const float t = s + x;
        const float bp = t - s;
        c += (s - (t - bp)) + (x - bp);
        s = t;
    }
    __device__ inline void wave_reduce() {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const float os = __shfl_xor(s, m, WAVE);
            const float oc = __shfl_xor(c, m, WAVE);
            add(os);
            c += oc;
        }
    }
    __device__ inline double value() const { return (double)s + (double)c; }
};
template <> struct Acc<double> {
    double s = 0.0;
    __device__ inline void add(double x) { s += x; }
    __device__ inline void wave_reduce() {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, WAVE);
    }
    __device__ inline double value() const { return s; }
};

// One ring's staged record (one per lane of the current 64-ring chunk).
template <typename T>
struct RingRec {
    T a;      // sin(theta_r - theta0)
    T b;      // sin(theta_r) cos(theta0)
    T c;      // sin(theta_r) sin(theta0)
    T e;      // 1 - cos(theta_r - theta0)
    T s;      // sin(theta_r)
    T z;      // cos(theta_r)
    T cdt;    // cos(theta_r - theta0)
    T f;      // cos(theta_r) cos(theta0)
    T g;      // cos(theta_r) sin(theta0)
    T dphic;  // longitude of the nearest pixel minus the boresight longitude
    T dphi;   // pixel spacing on the ring
    int32_t first, n, jc, k0, k1;
};

template <typename T>
struct WaveLds {
    RingRec<T> rec[WAVE];
    int32_t seg_end[2 * WAVE];
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wave_inclusive_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int o = __shfl_up(v, d, WAVE);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T> __device__ inline T lerp(T a, T b, T t) { return fma(t, b - a, a); }

// Reciprocal: the hardware approximation (1 ulp) in FP32, exact division in FP64.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }

// ----------------------------------------------------------------------
// The kernel
// ----------------------------------------------------------------------
template <typename T, int MODE>
__device__ void convolve_sample(const ConvArgs &A, const DetDesc &D, int64_t t, WaveLds<T> &L, int lane) {
    using R4 = typename Rec4<T>::type;
    const R4 *__restrict__ sky = reinterpret_cast<const R4 *>(A.sky);
    const R4 *__restrict__ beam = reinterpret_cast<const R4 *>(D.beam);
    const int32_t N = (int32_t)A.nside;

    // FP64 set-up of the sample's frame
    const double th0 = D.theta[t];
    double ph0 = D.phi[t];
    const double ps0 = D.psi[t];
    double s0, z0, sp, cp, sg, cg;
    sincos(th0, &s0, &z0);
    ph0 -= TWO_PI * floor(ph0 * (1.0 / TWO_PI));
    sincos(ps0, &sp, &cp);
    sincos(ps0 + D.zeta, &sg, &cg);
    const T cpsi = (T)cp, spsi = (T)sp, g1 = (T)cg, g2 = (T)sg, z0t = (T)z0, s0t = (T)s0;
    const int32_t n = D.n;
    const T inv_h = (T)D.inv_h;
    const T c0 = (T)(0.5 * (n - 1));
    const T tmax = (T)(n - 1);

    const int32_t nring = 4 * N - 1;
    const double rho = D.rho_max;
    const int32_t r_lo = (th0 - rho <= 0.0) ? 1 : max(1, (int32_t)floor(ring_of_theta(N, th0 - rho)) - 1);
    const int32_t r_hi = (th0 + rho >= PI) ? nring : min(nring, (int32_t)ceil(ring_of_theta(N, th0 + rho)) + 1);

    Acc<T> acc0, acc1, acc2, accn;
    int64_t npairs = 0;

    for (int32_t rb = r_lo; rb <= r_hi; rb += WAVE) {
        const int32_t r = rb + lane;
        int32_t n0 = 0, n1 = 0;
        if (r <= r_hi) {
            const RingGeom g = ring_geom(N, r);
            const double a = g.s * z0 - g.z * s0;
            const double cdt = g.z * z0 + g.s * s0;
            const double e = a * a / (1.0 + cdt);
            const double rel = ph0 - g.phi0;
            int32_t jc = (int32_t)rint(rel / g.dphi);
            jc %= g.n;
            if (jc < 0) jc += g.n;
            double dphic = g.phi0 + (double)jc * g.dphi - ph0;
            if (dphic > PI) dphic -= TWO_PI;
            else if (dphic < -PI) dphic += TWO_PI;
            int32_t olo, ocnt;
            ring_interval(D.cos_rho_max, z0, s0, g, dphic, olo, ocnt);
            int32_t k0 = olo, k1 = 0;
            n0 = ocnt;
            if (D.has_inner && ocnt > 0) {
                int32_t ilo, icnt;
                ring_interval(D.cos_rho_min, z0, s0, g, dphic, ilo, icnt);
                if (icnt >= g.n) {
                    n0 = 0;
                } else if (icnt > 0) {
                    if (ocnt >= g.n) {
                        k0 = ilo + icnt;
                        n0 = g.n - icnt;
                    } else {
                        n0 = max(0, ilo - olo);
                        k1 = ilo + icnt;
                        n1 = max(0, olo + ocnt - k1);
                    }
                }
            }
            RingRec<T> R;
            R.a = (T)a;
            R.b = (T)(g.s * z0);
            R.c = (T)(g.s * s0);
            R.e = (T)e;
            R.s = (T)g.s;
            R.z = (T)g.z;
            R.cdt = (T)cdt;
            R.f = (T)(g.z * z0);
            R.g = (T)(g.z * s0);
            R.dphic = (T)dphic;
            R.dphi = (T)g.dphi;
            R.first = g.first;
            R.n = g.n;
            R.jc = jc;
            R.k0 = k0;
            R.k1 = k1;
            L.rec[lane] = R;
        }
        const int32_t tot = n0 + n1;
        const int32_t incl = wave_inclusive_scan(tot, lane);
        const int32_t excl = incl - tot;
        L.seg_end[2 * lane] = excl + n0;
        L.seg_end[2 * lane + 1] = incl;
        const int32_t total = __shfl(incl, WAVE - 1, WAVE);
        if (MODE == 2) {  // disc pixel count only
            npairs += total;
            continue;
        }
        wave_sync();

        int32_t seg = 0;
        for (int32_t f = lane; f < total; f += WAVE) {
            while (f >= L.seg_end[seg]) ++seg;
            const int32_t start = (seg == 0) ? 0 : L.seg_end[seg - 1];
            const RingRec<T> &R = L.rec[seg >> 1];
            const int32_t rn = R.n;
            const int32_t k = ((seg & 1) ? R.k1 : R.k0) + (f - start);
            const int32_t half = rn >> 1;
            int32_t kk = k;
            if (kk >= half) kk -= rn;
            if (kk >= half) kk -= rn;
            if (kk < -half) kk += rn;
            int32_t j = R.jc + kk;
            if (j < 0) j += rn;
            else if (j >= rn) j -= rn;

            // geometry in differences from the boresight
            const T dph = fma((T)kk, R.dphi, R.dphic);
            T sh, ch;
            half_sincos((T)0.5 * dph, sh, ch);
            const T h = (T)2 * sh * sh;            // 1 - cos dphi
            const T S = (T)2 * sh * ch;            // sin dphi
            const T nth = fma(-R.b, h, R.a);       // n . theta_hat0
            const T nph = R.s * S;                 // n . phi_hat0
            const T omz = fma(R.c, h, R.e);        // 1 - n . p0
            const T xp = fma(cpsi, nth, spsi * nph);
            const T yp = fma(-spsi, nth, cpsi * nph);
            const T rz = rcp((T)1 - omz);
            const T tu = fma(xp * rz, inv_h, c0);
            const T tv = fma(yp * rz, inv_h, c0);
            if (!(tu >= (T)0 && tu <= tmax && tv >= (T)0 && tv <= tmax)) continue;
            const int32_t iu = min((int32_t)tu, n - 2);
            const int32_t iv = min((int32_t)tv, n - 2);
            const T fu = tu - (T)iu, fv = tv - (T)iv;
            const int32_t b00 = iv * n + iu;
            const R4 q00 = beam[b00], q10 = beam[b00 + 1], q01 = beam[b00 + n], q11 = beam[b00 + n + 1];
            const R4 pix = sky[R.first + j];

            // co-polar direction carried along the great circle, projected on
            // the pixel's theta_hat / phi_hat (all in the boresight sky basis)
            const T w = fma(g1, nth, g2 * nph);
            const T q = w * rcp((T)2 - omz);
            const T eth = fma(-q, nth, g1);
            const T eph = fma(-q, nph, g2);
            const T cth = fma(-R.f, h, R.cdt);      // theta_hat_k . theta_hat0
            const T cpp = fma(-R.g, h, -R.a);       // theta_hat_k . p0
            const T cc = fma(eth, cth, fma(eph, R.z * S, -w * cpp));
            const T ss = fma(-eth, z0t * S, fma(eph, (T)1 - h, w * s0t * S));
            const T c2 = fma(cc, cc, -ss * ss);
            const T s2 = (T)2 * cc * ss;

            const T bT = lerp(lerp(q00.w, q10.w, fu), lerp(q01.w, q11.w, fu), fv);
            const T qr = fma(c2, pix.y, s2 * pix.z);    // Q rotated into the detector frame
            const T ur = fma(-s2, pix.y, c2 * pix.z);   // U rotated into the detector frame
            accn.add(bT);
            if (MODE == 0) {
                const T bI = lerp(lerp(q00.x, q10.x, fu), lerp(q01.x, q11.x, fu), fv);
                const T bQ = lerp(lerp(q00.y, q10.y, fu), lerp(q01.y, q11.y, fu), fv);
                const T bU = lerp(lerp(q00.z, q10.z, fu), lerp(q01.z, q11.z, fu), fv);
                acc0.add(fma(bI, pix.x, fma(bQ, qr, bU * ur)));
            } else {
                acc0.add(bT * pix.x);
                acc1.add(bT * qr);
                acc2.add(bT * ur);
            }
        }
        wave_sync();
    }

    if (MODE == 2) {
        if (lane == 0) reinterpret_cast<T *>(A.out)[D.out_offset + t] = (T)npairs;
        return;
    }
    accn.wave_reduce();
    acc0.wave_reduce();
    if (MODE == 1) {
        acc1.wave_reduce();
        acc2.wave_reduce();
    }
    if (lane == 0) {
        double Nrm = D.norm_scale;
        if (D.norm_mode == 1) {
            const double sn = accn.value();
            Nrm = (sn != 0.0) ? D.norm_scale / sn : 0.0;
        }
        T *out = reinterpret_cast<T *>(A.out);
        const int64_t o = D.out_offset + t;
        if (MODE == 0) {
            out[o] = (T)(acc0.value() * Nrm);
        } else {
            out[3 * o + 0] = (T)(acc0.value() * Nrm);
            out[3 * o + 1] = (T)(acc1.value() * Nrm);
            out[3 * o + 2] = (T)(acc2.value() * Nrm);
        }
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(512) conv_kernel(ConvArgs A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    WaveLds<T> &L = reinterpret_cast<WaveLds<T> *>(lds_raw)[wid];
    int32_t q = (A.n_queues > 1) ? (int32_t)(blockIdx.x % (uint32_t)A.n_queues) : 0;
    int32_t exhausted = 0;
    while (exhausted < A.n_queues) {
        int32_t ti = 0;
        if (lane == 0) ti = atomicAdd(&A.counters[q], 1);
        ti = __shfl(ti, 0, WAVE);
        if (ti >= A.queue_len[q]) {
            q = (q + 1 == A.n_queues) ? 0 : q + 1;
            ++exhausted;
            continue;
        }
        const Tile tl = A.tiles[(int64_t)q * A.tiles_per_queue + ti];
        const DetDesc &D = A.dets[tl.det];
        for (int64_t t = tl.begin; t < tl.begin + tl.count; ++t) convolve_sample<T, MODE>(A, D, t, L, lane);
    }
}

__global__ void zero_counters_kernel(int32_t *c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

template <typename T>
__global__ void repack4_kernel(const T *a, const T *b, const T *c, const T *d, typename Rec4<T>::type *out,
                               int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename Rec4<T>::type r;
    r.x = a[i];
    r.y = b[i];
    r.z = c[i];
    r.w = d ? d[i] : (T)0;
    out[i] = r;
}

__global__ void check_pointing_kernel(const double *th, const double *ph, const double *ps, int64_t n,
                                      int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = th[i];
    const bool ok = isfinite(t) && t >= 0.0 && t <= PI && isfinite(ph[i]) && isfinite(ps[i]);
    if (!ok) atomicOr(bad, 1);
}

}  // namespace

hipError_t launch_zero_counters(int32_t *counters, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_conv_t(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    const size_t lds = sizeof(WaveLds<T>) * (size_t)waves;
    if (a.out_mode == 0)
        hipLaunchKernelGGL((conv_kernel<T, 0>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    else if (a.out_mode == 1)
        hipLaunchKernelGGL((conv_kernel<T, 1>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    else
        hipLaunchKernelGGL((conv_kernel<T, 2>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_conv(const ConvArgs &a, bool f64, int waves_per_group, int groups, hipStream_t s) {
    return f64 ? launch_conv_t<double>(a, waves_per_group, groups, s)
               : launch_conv_t<float>(a, waves_per_group, groups, s);
}

hipError_t launch_repack4(const void *a, const void *b, const void *c, const void *d, void *out, int64_t n,
                          bool f64, hipStream_t s) {
    const int bs = 256;
    const int64_t g = (n + bs - 1) / bs;
    if (g == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(repack4_kernel<double>, dim3((unsigned)g), dim3(bs), 0, s, (const double *)a,
                           (const double *)b, (const double *)c, (const double *)d, (double4 *)out, n);
    else
        hipLaunchKernelGGL(repack4_kernel<float>, dim3((unsigned)g), dim3(bs), 0, s, (const float *)a,
                           (const float *)b, (const float *)c, (const float *)d, (float4 *)out, n);
    return hipGetLastError();
}

hipError_t launch_check_pointing(const double *theta, const double *phi, const double *psi, int64_t n,
                                 int32_t *bad, hipStream_t s) {
    const int bs = 256;
    const int64_t g = (n + bs - 1) / bs;
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(check_pointing_kernel, dim3((unsigned)g), dim3(bs), 0, s, theta, phi, psi, n, bad);
    return hipGetLastError();
}

}  // namespace pisco
