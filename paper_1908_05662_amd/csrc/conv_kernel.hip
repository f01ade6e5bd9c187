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

#include <algorithm>
#include <mutex>

// The structured buffer load (index mode, stride from the descriptor) of the
// LLVM AMDGPU back end, declared by its intrinsic name.
typedef int32_t pisco_cell_v4i __attribute__((ext_vector_type(4)));
__device__ pisco_cell_v4i pisco_cell_struct_load(__amdgpu_buffer_rsrc_t r, int32_t vindex, int32_t voffset,
                                                 int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");

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

// The caller's index of the sample at position t of a detector's processing
// order (the library may process an incoherent stream in spatial order; the
// pointing is read and the output written at the caller's index).
__device__ inline int64_t sample_at(const DetDesc &D, int64_t t) { return D.order ? (int64_t)D.order[t] : t; }

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

// Per-lane accumulator: compensated (Kahan) in FP32, plain in FP64.  The
// compensated sum is s - c.
template <typename T> struct Acc;
template <> struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
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
    __device__ inline double value() const { return (double)s - (double)c; }
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

// Tile-path accumulator: FP32 pre-sums of eight terms added in FP64 (a
// conversion and an FP64 add, cheaper than a compensated FP32 add and more
// accurate).
struct AccWide {
    double s = 0.0;
    __device__ inline void add(float x) { s += (double)x; }
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

// Inclusive prefix sum over the 64 lanes by DPP moves (no lane-index
// arithmetic, so nothing lane-dependent stays live between calls): shifts by
// 1, 2, 4, 8 inside each row of 16 lanes (lanes shifted in from outside the row
// add 0), then the total of row 0 (lane 15) is added into row 1 and that of
// row 2 (lane 47) into row 3, and the total of rows 0-1 (lane 31) into rows 2
// and 3.
__device__ inline int wave_inclusive_scan(int v, int) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return v;
}

template <typename T> __device__ inline T lerp(T a, T b, T t) { return fma(t, b - a, a); }

// Reciprocal: the hardware approximation (1 ulp) in FP32, exact division in FP64.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }

// ----------------------------------------------------------------------
// Beam grids
//   FULL   : one record (bI, bQ, bU, bT) per node, n*n records
//   SCALAR : beam = b(u, v) * (wI, wQ, wU, wT); one record per cell holding
//            the cell's four corner values (b00, b10, b01, b11), (n-1)^2 records,
//            so a bilinear lookup is a single 16/32-byte load
// ----------------------------------------------------------------------
// One-grid cell records: the (n + 1)^2 padded array (n odd, so the side is
// even) stores its rows in interleaved pairs, record (U, V) at
// 2 ((V >> 1) side + U) + (V & 1), so a 128-byte line holds a 4 x 2 block of
// cells.  The 64 lanes of a tile gather cells along a short segment whose
// direction follows the scan and the position angle; row-major lines of 8
// cells meet one line per row the segment crosses.
__host__ __device__ inline int64_t cell_index(int64_t U, int64_t V, int64_t side) {
    return 2 * ((V >> 1) * side + U) + (V & 1);
}
template <typename T>
struct BeamVals {
    T bI, bQ, bU, bT;
};

template <typename T, int BEAM>
__device__ inline BeamVals<T> beam_lookup(const void *beam, int32_t n, int32_t iu, int32_t iv, T fu, T fv) {
    using R4 = typename Rec4<T>::type;
    const R4 *__restrict__ g = reinterpret_cast<const R4 *>(beam);
    BeamVals<T> o;
    if (BEAM == BEAM_FULL) {
        const int32_t b00 = iv * n + iu;
        const R4 q00 = g[b00], q10 = g[b00 + 1], q01 = g[b00 + n], q11 = g[b00 + n + 1];
        o.bI = lerp(lerp(q00.x, q10.x, fu), lerp(q01.x, q11.x, fu), fv);
        o.bQ = lerp(lerp(q00.y, q10.y, fu), lerp(q01.y, q11.y, fu), fv);
        o.bU = lerp(lerp(q00.z, q10.z, fu), lerp(q01.z, q11.z, fu), fv);
        o.bT = lerp(lerp(q00.w, q10.w, fu), lerp(q01.w, q11.w, fu), fv);
    } else {
        // cell record (b00, b10 - b00, b01 - b00, b11 - b10 - b01 + b00); the
        // records carry a ring of extrapolated cells, so cell (iu, iv) is padded
        // cell (iu + 1, iv + 1) of side n + 1 (rows stored in pairs)
        const R4 c = g[cell_index(iu + 1, iv + 1, n + 1)];
        o.bT = fma(fv, fma(fu, c.w, c.z), fma(fu, c.y, c.x));
        o.bI = o.bQ = o.bU = o.bT;
    }
    return o;
}

// ----------------------------------------------------------------------
// Pixel-parallel path: one sample at a time, lanes over its disc pixels
// ----------------------------------------------------------------------
template <typename T, int MODE, int BEAM>
__device__ void convolve_sample(const ConvArgs &A, const DetDesc &D, int64_t pos, WaveLds<T> &L, int lane) {
    const int64_t t = sample_at(D, pos);
    using R4 = typename Rec4<T>::type;
    const R4 *__restrict__ sky = reinterpret_cast<const R4 *>(A.sky);
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
    const T wI = (T)D.w[0], wQ = (T)D.w[1], wU = (T)D.w[2], wV = (T)D.wv;
    // half-wave plate: the Stokes angle 2 chi becomes 2 chi + 4 phi_t and the
    // U-row and V terms change sign (no plate: identity)
    T c4 = (T)1, s4 = (T)0, sg4 = (T)1;
    if (D.hwp) {
        double sh4, ch4;
        sincos(4.0 * D.hwp[t], &sh4, &ch4);
        c4 = (T)ch4;
        s4 = (T)sh4;
        sg4 = (T)-1;
    }
    using R4c = typename Rec4<T>::type;
    const R4c *__restrict__ vcells = reinterpret_cast<const R4c *>(D.beam_v);

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
        if (MODE == MODE_COUNT) {
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
            const T su = xp * rz, sv = yp * rz;  // gnomonic u, v
            const T tu = fma(su, inv_h, c0);
            const T tv = fma(sv, inv_h, c0);
            if (!(tu >= (T)0 && tu <= tmax && tv >= (T)0 && tv <= tmax)) continue;
            const int32_t iu = min((int32_t)tu, n - 2);
            const int32_t iv = min((int32_t)tv, n - 2);
            // fraction relative to the chosen node in one rounding (tu itself is
            // rounded at the scale of the grid offset c0)
            const T fu = fma(su, inv_h, c0 - (T)iu), fv = fma(sv, inv_h, c0 - (T)iv);
            const BeamVals<T> bv = beam_lookup<T, BEAM>(D.beam, n, iu, iv, fu, fv);
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
            const T c2p = fma(cc, cc, -ss * ss);
            const T s2p = (T)2 * cc * ss;
            const T c2 = fma(c4, c2p, -s4 * s2p);   // cos(2 chi + 4 phi)
            const T s2 = fma(s4, c2p, c4 * s2p);    // sin(2 chi + 4 phi)

            const T qr = fma(c2, pix.y, s2 * pix.z);          // Q rotated into the detector frame
            const T ur = sg4 * fma(-s2, pix.y, c2 * pix.z);   // U rotated into the detector frame
            const T vv = sg4 * pix.w;                         // V (not rotated)
            accn.add(bv.bT);
            if (MODE == MODE_TOD) {
                if (BEAM == BEAM_FULL) {
                    T term = fma(bv.bI, pix.x, fma(bv.bQ, qr, bv.bU * ur));
                    if (vcells) {
                        const R4c cv = vcells[iv * (n - 1) + iu];
                        term = fma(fma(fv, fma(fu, cv.w, cv.z), fma(fu, cv.y, cv.x)), vv, term);
                    }
                    acc0.add(term);
                } else {
                    acc0.add(bv.bT * fma(wI, pix.x, fma(wQ, qr, fma(wU, ur, wV * vv))));
                }
            } else {
                acc0.add(bv.bT * pix.x);
                acc1.add(bv.bT * qr);
                acc2.add(bv.bT * ur);
            }
        }
        wave_sync();
    }

    if (MODE == MODE_COUNT) {
        if (lane == 0) reinterpret_cast<T *>(A.out)[D.out_offset + t] = (T)npairs;
        return;
    }
    accn.wave_reduce();
    acc0.wave_reduce();
    if (MODE == MODE_STOKES) {
        acc1.wave_reduce();
        acc2.wave_reduce();
    }
    if (lane == 0) {
        double Nrm = D.norm_scale;
        if (D.norm_mode == 1) {
            const double sn = accn.value() * (BEAM == BEAM_SCALAR ? D.w[3] : 1.0);
            Nrm = (sn != 0.0) ? D.norm_scale / sn : 0.0;
        }
        T *out = reinterpret_cast<T *>(A.out);
        const int64_t o = D.out_offset + t;
        if (MODE == MODE_TOD) {
            out[o] = (T)(acc0.value() * Nrm);
        } else {
            if (BEAM == BEAM_SCALAR) Nrm *= D.w[3];  // the Stokes pickup uses the scalar beam wT b
            out[3 * o + 0] = (T)(acc0.value() * Nrm);
            out[3 * o + 1] = (T)(acc1.value() * Nrm);
            out[3 * o + 2] = (T)(acc2.value() * Nrm);
        }
    }
}

// ----------------------------------------------------------------------
// Sample-parallel path: lane l owns sample begin + l of a tile of consecutive
// samples.  The wave stages the pixels of the union of the tile's discs (a
// cap around the tile centre) in LDS, a chunk at a time, and every lane walks
// the same pixel records (LDS broadcasts), testing its own disc membership.
// FP64 is used for the tile and ring set-up; pixel records and pairs are FP32
// differences from the tile centre.  Beam lookups of neighbouring lanes fall
// on neighbouring beam cells.
// ----------------------------------------------------------------------
// Wave-uniform values kept in scalar registers.
__device__ inline double uniform(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Beam records through a buffer resource (word 3 = raw 32-bit data format on
// gfx9-family parts): the offset is a 32-bit VGPR, the base stays in SGPRs.
struct BeamRsrc {
    __amdgpu_buffer_rsrc_t r;
};
__device__ inline BeamRsrc make_beam_rsrc(const void *p, uint32_t nrec) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    void *u = (void *)(((unsigned long long)hi << 32) | lo);
    const int bytes = (int)__builtin_amdgcn_readfirstlane(nrec * 16u);   // uniform: the descriptor stays in SGPRs
    return BeamRsrc{__builtin_amdgcn_make_buffer_rsrc(u, (short)0, bytes, 0x00020000)};
}
__device__ inline float4 beam_ld(const BeamRsrc &b, uint32_t off, int32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)off, soff, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

// Structured access to the cell records (stride 16): the range test is on the
// record index, so an index at or past the count reads zero.
__device__ inline BeamRsrc make_cell_rsrc(const void *p, uint32_t nrec) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    void *u = (void *)(((unsigned long long)hi << 32) | lo);
    const int cnt = (int)__builtin_amdgcn_readfirstlane(nrec);
    return BeamRsrc{__builtin_amdgcn_make_buffer_rsrc(u, (short)16, cnt, 0x00020000)};
}
__device__ inline float4 cell_ld(const BeamRsrc &b, uint32_t idx) {
    const pisco_cell_v4i v = pisco_cell_struct_load(b.r, (int32_t)idx, 0, 0, 0);
    return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
}

struct PixRec {
    float X, Y, W;      // n = X e1 + Y e2 + (1 - W) c in the tile frame
    float t1, t2, t3;   // the pixel's theta_hat in the tile frame
    float f1, f2, f3;   // the pixel's phi_hat in the tile frame
    float a, b, c;      // scalar beam, TOD: wI I, wQ Q + wU U, wQ U - wU Q; otherwise I, Q, U
};

// Pixel record of the one-grid TOD loop without a plate (the quadratic-form
// path): n as above, and the pixel's angle terms as a quadratic form in the
// first two tile-frame components of the carried theta'_0 (see tile_pairs).
struct PixRecQ {
    float G1, G2;         // gnomonic coordinates about the tile centre: n_xy / n_z
    float W, Z;           // 1 - n_z and n_z
    float ZX, ZY;         // n_z n_xy
    float A;              // wI I + wV V - B, B the turned Q, U term
    float P11, P12, P22;  // e^T P e = 2 cos gamma (B cos gamma + C sin gamma) / h^2 ... x h^2
    float pad0, pad1;
};

template <bool B, class T, class F> struct Cond { using type = T; };
template <class T, class F> struct Cond<false, T, F> { using type = F; };

// One ring of the union cap, with the ring's coefficients relative to the
// tile centre (the same difference formulas as the pixel path, with the
// centre in place of the boresight).
struct UnionRing {
    float a, b, c, e, s, z, cdt, f, g, dphic, dphi, dth;   // dth: colatitude minus the centre's
    int32_t first, n, jc, lo;   // pixels k = lo .. lo + cnt - 1 counted from the pixel nearest the centre
};

// Per-lane sample frame in the tile frame (all FP32; the small quantities keep
// relative precision because they are formed in FP64 first).
struct LaneFrame {
    float om, p1, p2, p3;   // 1 - p.c and p
    float a1, a2, a3;       // theta'_0
    float b1, b2, b3;       // phi'_0
    float g1, g2, g3;       // co-polar direction at the boresight (matrix-core variant)
    float c2p, s2p;         // cos, sin of 2 phi_t (half-wave plate; 1, 0 without one)
};

// The set-up helpers below are not inlined (their FP64 constants must not be
// hoisted into the pixel loops); they write their per-lane results straight
// into this LDS slice instead of returning them through the stack.
// The lane frames are read into registers before the first record is staged,
// so they share storage with the records.
template <int CH>
struct TileLds {
    UnionRing ring[WAVE];
    int32_t seg_end[WAVE];
    union {
        LaneFrame lane[WAVE];
        PixRec rec[CH];
    };
};
static_assert(sizeof(UnionRing) == 64 && sizeof(LaneFrame) == 60 && sizeof(PixRec) == 48 && sizeof(PixRecQ) == 48 &&
                  sizeof(TileLds<64>) == 4352 + 3840 && sizeof(TileLds<128>) == 4352 + 128 * 48 &&
                  sizeof(TileLds<256>) == 4352 + 256 * 48,
              "the runtime's LDS budget assumes 4352 bytes + max(3840, 48 per staged record) per wave");
// Launches with a V-column beam append one float per staged record and wave
// after the TileLds array (V of the staged pixels); others do not allocate it,
// so it costs them no occupancy.

struct TileFrame {
    double thc, phc, zc, sc, Ru;
    double cosRu;           // cos of the union radius
    int32_t r_lo, r_hi;     // rings that can meet the union cap
};

// FP64 set-up of a tile: the centre c (normalised mean boresight), the union
// radius, and each lane's sample expressed in the frame (e1, e2, c) with
// e1 = theta_hat(c), e2 = phi_hat(c).  Not inlined: its transcendental
// constants stay out of the pixel loops.
__device__ __attribute__((noinline)) TileFrame tile_setup(const DetDesc &D, int32_t N, int64_t t, bool valid,
                                                          LaneFrame *out) {
    const double th0 = D.theta[t], ph0 = D.phi[t], ps0 = D.psi[t];
    double st, ct, sf, cf, sp, cp, sg, cg;
    sincos(th0, &st, &ct);
    sincos(ph0, &sf, &cf);
    sincos(ps0, &sp, &cp);
    sincos(ps0 + D.zeta, &sg, &cg);
    const double p[3] = {st * cf, st * sf, ct};
    const double th[3] = {ct * cf, ct * sf, -st};
    const double ph[3] = {-sf, cf, 0.0};
    double sx = valid ? p[0] : 0.0, sy = valid ? p[1] : 0.0, sz = valid ? p[2] : 0.0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        sx += __shfl_xor(sx, m, WAVE);
        sy += __shfl_xor(sy, m, WAVE);
        sz += __shfl_xor(sz, m, WAVE);
    }
    const double sn = sqrt(sx * sx + sy * sy + sz * sz);
    const double c[3] = {sx / sn, sy / sn, sz / sn};
    const double rxy = sqrt(c[0] * c[0] + c[1] * c[1]);
    TileFrame T;
    T.thc = atan2(rxy, c[2]);
    T.phc = atan2(c[1], c[0]);
    if (T.phc < 0.0) T.phc += TWO_PI;
    T.zc = c[2];
    T.sc = rxy;
    double sfc, cfc;
    sincos(T.phc, &sfc, &cfc);
    const double e1[3] = {c[2] * cfc, c[2] * sfc, -rxy};
    const double e2[3] = {-sfc, cfc, 0.0};
    const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
    const double om = 0.5 * (dx * dx + dy * dy + dz * dz);  // 1 - p.c
    double ta[3], tb[3], tg[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ta[i] = cp * th[i] + sp * ph[i];   // theta'_0
        tb[i] = -sp * th[i] + cp * ph[i];  // phi'_0
        tg[i] = cg * th[i] + sg * ph[i];   // co-polar direction at the boresight
    }
    LaneFrame F;
    F.om = (float)om;
    F.p1 = (float)(p[0] * e1[0] + p[1] * e1[1] + p[2] * e1[2]);
    F.p2 = (float)(p[0] * e2[0] + p[1] * e2[1]);
    F.p3 = (float)(1.0 - om);
    F.a1 = (float)(ta[0] * e1[0] + ta[1] * e1[1] + ta[2] * e1[2]);
    F.a2 = (float)(ta[0] * e2[0] + ta[1] * e2[1]);
    F.a3 = (float)(ta[0] * c[0] + ta[1] * c[1] + ta[2] * c[2]);
    F.b1 = (float)(tb[0] * e1[0] + tb[1] * e1[1] + tb[2] * e1[2]);
    F.b2 = (float)(tb[0] * e2[0] + tb[1] * e2[1]);
    F.b3 = (float)(tb[0] * c[0] + tb[1] * c[1] + tb[2] * c[2]);
    F.g1 = (float)(tg[0] * e1[0] + tg[1] * e1[1] + tg[2] * e1[2]);
    F.g2 = (float)(tg[0] * e2[0] + tg[1] * e2[1]);
    F.g3 = (float)(tg[0] * c[0] + tg[1] * c[1] + tg[2] * c[2]);
    F.c2p = 1.0f;
    F.s2p = 0.0f;
    if (D.hwp) {
        double sh2, ch2;
        sincos(2.0 * D.hwp[t], &sh2, &ch2);
        F.c2p = (float)ch2;
        F.s2p = (float)sh2;
    }
    *out = F;
    double dist = valid ? 2.0 * asin(fmin(1.0, 0.5 * sqrt(2.0 * om))) : 0.0;  // angle from the centre
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) dist = fmax(dist, __shfl_xor(dist, m, WAVE));
    T.Ru = D.rho_max + dist + 1e-9;
    // wave-uniform from here (the reductions above leave every lane equal)
    T.cosRu = cos(T.Ru);
    const int32_t nring = 4 * N - 1;
    T.r_lo = (T.thc - T.Ru <= 0.0) ? 1 : max(1, (int32_t)floor(ring_of_theta(N, T.thc - T.Ru)) - 1);
    T.r_hi = (T.thc + T.Ru >= PI) ? nring : min(nring, (int32_t)ceil(ring_of_theta(N, T.thc + T.Ru)) + 1);
    return T;
}

// FP64 set-up of one union ring: its pixel interval within the cap and its
// coefficients relative to the tile centre.  Returns the pixel count.
__device__ __attribute__((noinline)) int32_t union_ring_setup(int32_t N, int32_t r, double phc, double zc, double sc,
                                                             double cosRu, UnionRing *out) {
    const RingGeom g = ring_geom(N, r);
    const double a = g.s * zc - g.z * sc;
    const double cdt = g.z * zc + g.s * sc;
    int32_t jc = (int32_t)rint((phc - g.phi0) / g.dphi);
    jc %= g.n;
    if (jc < 0) jc += g.n;
    double dphic = g.phi0 + (double)jc * g.dphi - phc;
    if (dphic > PI) dphic -= TWO_PI;
    else if (dphic < -PI) dphic += TWO_PI;
    int32_t lo, k;
    ring_interval(cosRu, zc, sc, g, dphic, lo, k);
    UnionRing u;
    u.a = (float)a;
    u.b = (float)(g.s * zc);
    u.c = (float)(g.s * sc);
    u.e = (float)(a * a / (1.0 + cdt));
    u.s = (float)g.s;
    u.z = (float)g.z;
    u.cdt = (float)cdt;
    u.f = (float)(g.z * zc);
    u.g = (float)(g.z * sc);
    u.dphic = (float)dphic;
    u.dphi = (float)g.dphi;
    u.dth = (float)atan2(a, cdt);
    u.first = g.first;
    u.n = g.n;
    u.jc = jc;
    u.lo = lo;
    *out = u;
    return k;
}

// A lane's own disc, for narrowing the union cap ring by ring, in FP32:
// colatitude offset from the tile centre (FP64 difference, so small offsets
// keep their precision), 1 / sine of the colatitude, longitude offset from the
// centre (in (-pi, pi]) and rho_max.  `ok` (uniform) is false when some lane's
// boresight is within asin(1/4) of a pole or the disc is wider than 1.5 rad.
struct LaneHull {
    float dth, rsl, dphl, R;
    bool ok;
};

__device__ __attribute__((noinline)) LaneHull lane_hull(const DetDesc &D, int64_t t, bool valid, double phc,
                                                        double zc, double sc) {
    double st, ct;
    sincos(D.theta[t], &st, &ct);
    double d = D.phi[t] - phc;
    d -= TWO_PI * rint(d / TWO_PI);
    LaneHull h;
    h.dth = (float)atan2(st * zc - ct * sc, ct * zc + st * sc);
    h.rsl = (float)(1.0 / fmax(st, 0.25));
    h.dphl = (float)d;
    h.R = (float)D.rho_max;
    h.ok = (__ballot(valid && !(st >= 0.25)) == 0) && D.rho_max <= 1.5;
    return h;
}

// Narrow each ring of a batch (ring i's union-cap interval in L.ring[i].lo and
// lane i's `rc`) to the hull of the valid lanes' own disc intervals on it.  A
// lane's half-width dm on a ring at colatitude offset dtheta from it follows
// from hav(dm) = sin((rho_max - |dtheta|) / 2) sin((rho_max + |dtheta|) / 2) /
// (sin theta_ring sin theta_lane) (the law of cosines with the difference of
// cosines as a product), which keeps relative precision in FP32 down to the
// tangent ring.  Rounding (and the hardware square root, within 1 ulp) is
// covered by raising the first angle by 1.5e-7 rad, hav by a relative 1e-6 and
// each end by 0.02 pixel, so the hull holds every
// pixel of every lane's disc; pairs are still tested one by one.  Rings that
// the cap covers whole or that lie near a pole keep the cap interval.
__device__ void narrow_rings(UnionRing *ring, int32_t &rc, int32_t nb, const LaneHull &H, bool valid, int lane) {
    for (int32_t i = 0; i < nb; ++i) {
        const int32_t cnt = __builtin_amdgcn_readlane(rc, i);
        const int32_t rn = __builtin_amdgcn_readfirstlane(ring[i].n);
        const float sr = ring[i].s;
        if (cnt == 0 || cnt >= rn || !(sr >= 0.25f)) continue;
        const int32_t lo = __builtin_amdgcn_readfirstlane(ring[i].lo), hi = lo + cnt - 1;
        const float dth = fabsf(ring[i].dth - H.dth);
        const float ha = fmaf(0.5f, H.R - dth, 1.5e-7f);
        int32_t klo = 0x7fffffff, khi = -0x7fffffff;
        if (valid && ha > 0.0f) {
            float sa, ca, sb, cb;
            half_sincos(ha, sa, ca);
            half_sincos(ha + dth, sb, cb);
            const float hav = sa * sb * (H.rsl * __builtin_amdgcn_rcpf(sr)) * (1.0f + 1e-6f);
            if (hav >= 1.0f) {
                klo = lo;
                khi = hi;
            } else {
                // asin by its odd series to y^11 below 0.3 (truncation 1e-8 and
                // FP32 rounding 3e-7 relative: under 0.002 pixel), the library above
                const float y = __builtin_amdgcn_sqrtf(hav), y2 = y * y;
                float ps = fmaf(y2, 63.0f / 2816.0f, 35.0f / 1152.0f);
                ps = fmaf(y2, ps, 5.0f / 112.0f);
                ps = fmaf(y2, ps, 3.0f / 40.0f);
                ps = fmaf(y2, ps, 1.0f / 6.0f);
                const float as = (y < 0.3f) ? y * fmaf(y2, ps, 1.0f) : asinf(y);
                const float dm = 2.0f * as;
                const float inv = __builtin_amdgcn_rcpf(ring[i].dphi);
                const float base = H.dphl - ring[i].dphic;
                klo = max(lo, (int32_t)ceilf(fmaf(base - dm, inv, -0.02f)));
                khi = min(hi, (int32_t)floorf(fmaf(base + dm, inv, 0.02f)));
            }
        }
        klo = __ockl_wfred_min_i32(klo);
        khi = __ockl_wfred_max_i32(khi);
        // no lane meets the ring: empty (the sentinels must not enter the
        // arithmetic); otherwise lo <= nlo and nlo + ncnt - 1 <= hi
        int32_t nlo = lo, ncnt = 0;
        if (klo <= khi) {
            nlo = max(lo, klo);
            ncnt = max(0, min(hi, khi) - nlo + 1);
        }
        if (lane == i) {
            rc = ncnt;
            ring[i].lo = nlo;
        }
    }
}

// The same narrowing with the roles exchanged: lane i owns ring i of the batch
// and walks the tile's ns samples, whose (colatitude offset, 1 / sine of the
// colatitude, longitude offset) are staged in LDS (`hull`, broadcast reads; a
// sample outside the tile has an offset of 16 rad, so it meets no ring).  Each
// (ring, sample) interval is computed exactly as in narrow_rings (same
// expressions, so the narrowed intervals are the same) and the lane keeps
// their running minimum and maximum: no cross-lane reductions.
__device__ void narrow_rings_lanes(UnionRing *ring, int32_t &rc, int32_t nb, const float4 *hull, int32_t ns, float R,
                                   int lane) {
    const int32_t cnt = rc;
    const int32_t rn = ring[lane].n;
    const float sr = ring[lane].s;
    const bool act = lane < nb && cnt > 0 && cnt < rn && sr >= 0.25f;
    if (__ballot(act) == 0) return;
    const int32_t lo = ring[lane].lo, hi = lo + cnt - 1;
    const float rdth = ring[lane].dth, rsr = __builtin_amdgcn_rcpf(sr), inv = __builtin_amdgcn_rcpf(ring[lane].dphi);
    const float dphic = ring[lane].dphic;
    int32_t klo = 0x7fffffff, khi = -0x7fffffff;
    for (int32_t l = 0; l < ns; ++l) {
        const float4 h = hull[l];
        const float dth = fabsf(rdth - h.x);
        const float ha = fmaf(0.5f, R - dth, 1.5e-7f);
        const float hac = fmaxf(ha, 0.0f);   // a disc that misses the ring: hav = 0 (discarded below)
        float sa, ca, sb, cb;
        half_sincos(hac, sa, ca);
        half_sincos(hac + dth, sb, cb);
        const float hav = sa * sb * (h.y * rsr) * (1.0f + 1e-6f);
        const float y = __builtin_amdgcn_sqrtf(hav), y2 = y * y;
        float ps = fmaf(y2, 63.0f / 2816.0f, 35.0f / 1152.0f);
        ps = fmaf(y2, ps, 5.0f / 112.0f);
        ps = fmaf(y2, ps, 3.0f / 40.0f);
        ps = fmaf(y2, ps, 1.0f / 6.0f);
        const float as = (y < 0.3f) ? y * fmaf(y2, ps, 1.0f) : asinf(fminf(y, 1.0f));
        const float dm = 2.0f * as;
        const float base = h.z - dphic;
        int32_t a = max(lo, (int32_t)ceilf(fmaf(base - dm, inv, -0.02f)));
        int32_t b = min(hi, (int32_t)floorf(fmaf(base + dm, inv, 0.02f)));
        if (hav >= 1.0f) {
            a = lo;
            b = hi;
        }
        if (!(ha > 0.0f)) {
            a = 0x7fffffff;
            b = -0x7fffffff;
        }
        klo = min(klo, a);
        khi = max(khi, b);
    }
    if (act) {
        int32_t nlo = lo, ncnt = 0;
        if (klo <= khi) {
            nlo = max(lo, klo);
            ncnt = max(0, min(hi, khi) - nlo + 1);
        }
        rc = ncnt;
        ring[lane].lo = nlo;
    }
}

// Per-sample constants of the tile consume loop.
struct PairCtx {
    LaneFrame F;
    float omax, omin;
    bool clip;
    float inv_h, c0, tmax, cmax, row;
    int32_t row_bytes;
    float sg4;            // -1 with a half-wave plate: U-row and V terms change sign
    float rowc;           // cells per grid row (bV cell polynomials)
    float tmin;           // lower grid bound of t: 1 for one-grid beams (their t counts the extrapolated ring), else 0
    uint32_t irow;        // records per row, as an integer
};

// Masked contributions of NP consecutive (pixel record, sample) pairs,
// summed in FP32: v0 (TOD term or I pickup), v1, v2 (Q, U pickups), vn (beam
// value for the normaliser); a pixel outside the sample's disc adds zero.
// The NP pairs are interleaved phase by phase (geometry, beam loads, position
// angle, terms) so their beam loads are in flight together.
struct PairOut {
    float v0, v1, v2, vn;
};
// Records per consume step (their beam loads are in flight together), and the
// minimum waves per SIMD each tile kernel is compiled for: four (at most 128
// VGPRs) for one-grid TOD and pair counts, whose pair loop fits without spills
// and gains from the latency hiding; two (up to 256 VGPRs) for four-channel
// TOD and Stokes pickups, which would spill inside the loop at four.
constexpr int TILE_NP = 4;
template <int MODE, int BEAM>
constexpr int tile_min_waves() {
    return (MODE == MODE_STOKES || (MODE == MODE_TOD && BEAM == BEAM_FULL)) ? 2 : 4;
}

// A byte offset past every beam-record array (grids have at most 4096^2 cell
// records, 256 MiB), with room before 2^32 for a load at it plus a row
// (at most 16 x 4095 bytes) plus 16; as a record index, past every record count.
constexpr uint32_t OOB_OFFSET = 0x80000000u;

// SC (small cap): every pair inside the disc has omega = 1 - n.p <= SC_OMEGA, so
// 1 / z' = 1 / (1 - omega) and 1 / (1 + z') = (1/2) / (1 - omega / 2) are their
// geometric series instead of a quarter-rate reciprocal; pairs outside the disc
// are masked.  SC = 1: 1 / z' to the third power (truncation below
// omega^4 = 2.6e-10, inside FP32's rounding); SC = 2, for omega <= SC2_OMEGA: to
// the second power (truncation below omega^3 = 1e-9).  1 / (1 + z') only scales
// q = (a.n) / (1 + z') in e = a - q (p + n), with a.n at most sin(rho) ~
// sqrt(2 omega) and |p + n| <= 2, so one power fewer suffices there: the
// truncation moves e by less than sqrt(2 omega) omega^3 / 8 of |a| (SC = 1,
// 7e-10) and sqrt(2 omega) omega^2 / 4 (SC = 2, 1.1e-8), both under FP32's half
// ulp.
constexpr double SC_OMEGA = 4e-3;
constexpr double SC2_OMEGA = 1e-3;
// The quadratic-form records take the gnomonic scale 1 / (1 - t) instead of
// 1 / z' (see tile_pairs), with |t| <= max(omega_max, (1 - cos R_u) / cos R_u)
// for every pair inside the disc (R_u the tile's union radius); its series
// to the second power for |t| <= SCT2 (truncation below 8e-9) and the third
// for |t| <= SCT1 (below 4.1e-9), both an order under FP32's rounding.
constexpr double SCT2 = 2e-3;
constexpr double SCT1 = 8e-3;

template <int MODE, int BEAM, bool PS, int NP, bool HWP, bool CLIP, bool INNER, int SC = 0, bool QF = false>
__device__ __forceinline__ PairOut tile_pairs(const typename Cond<QF, PixRecQ, PixRec>::type *Rp, const float *Vp,
                                              const PairCtx &C, const BeamRsrc &beam, const BeamRsrc &vbeam) {
    static_assert(!QF || (MODE == MODE_TOD && BEAM == BEAM_SCALAR && !HWP), "quadratic form: one-grid TOD, no plate");
    constexpr bool ZMASK = BEAM == BEAM_SCALAR && SC != 0 && MODE == MODE_TOD;
    const LaneFrame &F = C.F;
    typename Cond<QF, PixRecQ, PixRec>::type R[NP];
    float omg[NP], xp[NP], yp[NP], rzh[NP], rq[NP], fu[NP], fv[NP];
    bool in[NP];
    uint32_t off[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        R[k] = Rp[k];
        if constexpr (QF) {
            // gnomonic form about the tile centre: with G = n_xy / n_z and
            // t = om - p1 G1 - p2 G2, n.p / n_z = p3 + p.G = 1 - t, so
            // 1 - n.p = W + n_z t, and n.theta'_0 / n_z = a3 + a1 G1 + a2 G2
            // (phi'_0 likewise): the grid coordinates are these over 1 - t,
            // two products each instead of three
            const float tt = fmaf(-R[k].G2, F.p2, fmaf(-R[k].G1, F.p1, F.om));
            omg[k] = fmaf(R[k].Z, tt, R[k].W);
            in[k] = omg[k] <= C.omax;
            xp[k] = fmaf(R[k].G2, F.a2, fmaf(R[k].G1, F.a1, F.a3));   // n.theta'_0 / n_z, grid units
            yp[k] = fmaf(R[k].G2, F.b2, fmaf(R[k].G1, F.b1, F.b3));
            const float w = omg[k];
            if (SC == 2) {
                rzh[k] = fmaf(tt, tt + 1.0f, 1.0f);                              // 1 / (1 - t)
                rq[k] = fmaf(w, 0.25f, 0.5f);                                    // 1 / (1 + z')
            } else if (SC == 1) {
                rzh[k] = fmaf(tt, fmaf(tt, tt + 1.0f, 1.0f), 1.0f);
                rq[k] = fmaf(w, fmaf(w, 0.125f, 0.25f), 0.5f);
            } else {
                const float dn = 1.0f - tt, zq = 2.0f - w;
                const float rr = rcp(dn * zq);
                rzh[k] = rr * zq;
                rq[k] = rr * dn;
            }
        } else {
        // n = X e1 + Y e2 + (1 - W) c in the tile frame
        omg[k] = fmaf(-R[k].Y, F.p2, fmaf(-R[k].X, F.p1, fmaf(R[k].W, F.p3, F.om)));  // 1 - n.p
        in[k] = INNER ? ((omg[k] <= C.omax) & (omg[k] > C.omin)) : (omg[k] <= C.omax);
        // n . theta'_0 and n . phi'_0 in grid units (the lane's rows carry 1 / h)
        xp[k] = fmaf(-R[k].W, F.a3, fmaf(R[k].Y, F.a2, fmaf(R[k].X, F.a1, F.a3)));
        yp[k] = fmaf(-R[k].W, F.b3, fmaf(R[k].Y, F.b2, fmaf(R[k].X, F.b1, F.b3)));
        if (SC == 2) {
            const float w = omg[k];
            rzh[k] = fmaf(w, w + 1.0f, 1.0f);                                  // 1 / z'
            rq[k] = fmaf(w, 0.25f, 0.5f);                                      // 1 / (1 + z')
        } else if (SC == 1) {
            const float w = omg[k];
            rzh[k] = fmaf(w, fmaf(w, w + 1.0f, 1.0f), 1.0f);                   // 1 / z'
            rq[k] = fmaf(w, fmaf(w, 0.125f, 0.25f), 0.5f);                      // 1 / (1 + z')
        } else {
            // one reciprocal for both divisions of the pair: 1 / (z' (1 + z')), z' = n.p
            const float zp = 1.0f - omg[k], zq = 2.0f - omg[k];
            const float rr = rcp(zp * zq);
            rzh[k] = rr * zq;            // gnomonic scale 1 / z'
            rq[k] = rr * zp;             // 1 / (1 + z')
        }
        }
        const float tu = fmaf(xp[k], rzh[k], C.c0);
        const float tv = fmaf(yp[k], rzh[k], C.c0);
        if (CLIP) in[k] = in[k] & (tu >= C.tmin) & (tu <= C.tmax) & (tv >= C.tmin) & (tv <= C.tmax);
        // cell indices.  One-grid beams: t counts from the extrapolated ring
        // (C.c0 is one larger), and there is no clamp -- a pair inside the disc
        // (and, with CLIP, inside the grid) has t in [1, n] up to rounding, so
        // floor(t) is a record of the grid's cells or of the ring around them,
        // whose polynomials continue the edge cells' (the value the clamped
        // lookup extrapolates to); other pairs are masked, and the buffer
        // resource turns any offset past the records into a zero read.
        // Four-channel beams: clamped node indices.
        if (BEAM == BEAM_SCALAR) {
            // truncation is the floor there (t >= 0 up to rounding; a masked pair's
            // index only picks some record or a zero read, and wide discs send it
            // to record 0 below), fract gives t - floor(t) exactly, and the record
            // index takes a shift and two 24-bit multiply-adds (row < 4097)
            const uint32_t iu = (uint32_t)(int32_t)tu, iv = (uint32_t)(int32_t)tv;
            fu[k] = __builtin_amdgcn_fractf(tu);
            fv[k] = __builtin_amdgcn_fractf(tv);
            // the record index in row pairs: 2 ((iv >> 1) (side - 1) + iu) + iv
            const uint32_t m = (uint32_t)__umul24(iv >> 1, C.irow - 1u) + iu;
            off[k] = (m << 1) + iv;
        } else {
            const float ku = floorf(__builtin_amdgcn_fmed3f(tu, 0.0f, C.cmax));
            const float kv = floorf(__builtin_amdgcn_fmed3f(tv, 0.0f, C.cmax));
            fu[k] = tu - ku;   // exact; carries the rounding of tu (half an ulp)
            fv[k] = tv - kv;
            off[k] = (uint32_t)fmaf(kv, C.row, ku) << 4;  // exact: row^2 < 2^24
        }
        // wide discs: a masked pair's unclamped cell can be anywhere in a large
        // record array, so its load is sent to record 0 (kept in cache)
        if (BEAM == BEAM_SCALAR && SC == 0) off[k] = in[k] ? off[k] : 0u;
        // series geometry (every factor of a pair finite): a masked pair's load is
        // sent past the records, so it reads zero without a cache access, and that
        // zero is its mask
        if (ZMASK) off[k] = in[k] ? off[k] : OOB_OFFSET;
        // four-channel beams: the four node loads of a masked pair likewise
        // (the term keeps its select: a V column is read from another array)
        if (BEAM == BEAM_FULL && MODE == MODE_TOD && SC != 0) off[k] = in[k] ? off[k] : OOB_OFFSET;
    }
    float4 cl[NP][BEAM == BEAM_SCALAR ? 1 : 4];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        cl[k][0] = BEAM == BEAM_SCALAR ? cell_ld(beam, off[k]) : beam_ld(beam, off[k], 0);
        if (BEAM != BEAM_SCALAR) {
            cl[k][1] = beam_ld(beam, off[k] + 16, 0);
            cl[k][2] = beam_ld(beam, off[k], C.row_bytes);
            cl[k][3] = beam_ld(beam, off[k] + 16, C.row_bytes);
        }
    }
    float vv[NP], vb[NP];
    if (BEAM == BEAM_FULL && MODE == MODE_TOD && Vp) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            vv[k] = Vp[k];
            const float ku = floorf(__builtin_amdgcn_fmed3f(fmaf(xp[k], rzh[k], C.c0), 0.0f, C.cmax));
            const float kv = floorf(__builtin_amdgcn_fmed3f(fmaf(yp[k], rzh[k], C.c0), 0.0f, C.cmax));
            const float4 c = beam_ld(vbeam, (uint32_t)fmaf(kv, C.rowc, ku) << 4, 0);
            vb[k] = fmaf(fv[k], fmaf(fu[k], c.w, c.z), fmaf(fu[k], c.y, c.x));
        }
    }
    PairOut o{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        // position angle.  The co-polar direction at the boresight is
        // cos(zeta) theta'_0 + sin(zeta) phi'_0, and carrying vectors along the
        // great circle is linear and keeps angles, so chi = gamma + zeta with
        // gamma the angle of theta'_0 carried to the pixel; the turn by 2 zeta
        // is in the staged Q, U coefficients.  theta'_0 carried from the
        // boresight to the pixel is e = a - q (p + n), q = a.n / (1 + n.p), and
        // the pixel's theta_hat and phi_hat are normal to n, so their
        // projections take a - q p.  a.n is xp, in grid units like the lane's
        // a rows, so e, its projections and the angle terms below carry the
        // grid scale (1/h, 1/h^2); the records carry h^2.
        const float q = xp[k] * rq[k];
        if constexpr (QF) {
            // e is normal to n, so its first two tile-frame components fix it:
            // for vectors v, w normal to n, v.w = v_xy . (w_xy - (w_z / n_z) n_xy),
            // and the records hold 2 cos gamma (B cos gamma + C sin gamma), the
            // product of the projections on theta_hat and on B theta_hat + C phi_hat,
            // as the quadratic form e_xy^T P e_xy (x h^2).  Here xp is
            // a.n / n_z, so q (p + n) = (xp rq) n_z (p + n).
            const float ex = fmaf(-q, fmaf(R[k].Z, F.p1, R[k].ZX), F.a1);
            const float ey = fmaf(-q, fmaf(R[k].Z, F.p2, R[k].ZY), F.a2);
            const float4 c = cl[k][0];
            const float bT = fmaf(fv[k], fmaf(fu[k], c.w, c.z), fmaf(fu[k], c.y, c.x));
            const float bTm = ZMASK ? bT : (in[k] ? bT : 0.0f);
            if (PS) o.vn += bTm;
            const float quad = fmaf(ex, fmaf(R[k].P11, ex, R[k].P12 * ey), fmaf(R[k].P22 * ey, ey, R[k].A));
            o.v0 += bTm * quad;
            continue;
        } else {
        const float ex = fmaf(-q, F.p1, F.a1);
        const float ey = fmaf(-q, F.p2, F.a2);
        const float ez = fmaf(-q, F.p3, F.a3);
        float cc = fmaf(ex, R[k].t1, fmaf(ey, R[k].t2, ez * R[k].t3));   // cos gamma / h
        float ss = fmaf(ex, R[k].f1, fmaf(ey, R[k].f2, ez * R[k].f3));   // sin gamma / h
        if (HWP) {
            // the plate advances 2 chi by 4 phi_t: gamma turned by 2 phi_t
            const float c0 = cc;
            cc = fmaf(F.c2p, c0, -F.s2p * ss);
            ss = fmaf(F.s2p, c0, F.c2p * ss);
        }
        const float sgn = HWP ? C.sg4 : 1.0f;
        float bT, bI = 0.0f, bQ = 0.0f, bU = 0.0f;
        if (BEAM == BEAM_SCALAR) {
            const float4 c = cl[k][0];
            bT = fmaf(fv[k], fmaf(fu[k], c.w, c.z), fmaf(fu[k], c.y, c.x));
        } else {
            const float4 q00 = cl[k][0], q10 = cl[k][1], q01 = cl[k][2], q11 = cl[k][3];
            bI = lerp(lerp(q00.x, q10.x, fu[k]), lerp(q01.x, q11.x, fu[k]), fv[k]);
            bQ = lerp(lerp(q00.y, q10.y, fu[k]), lerp(q01.y, q11.y, fu[k]), fv[k]);
            bU = lerp(lerp(q00.z, q10.z, fu[k]), lerp(q01.z, q11.z, fu[k]), fv[k]);
            bT = lerp(lerp(q00.w, q10.w, fu[k]), lerp(q01.w, q11.w, fu[k]), fv[k]);
        }
        if (PS) o.vn += (ZMASK || in[k]) ? bT : 0.0f;
        if (MODE == MODE_TOD && BEAM == BEAM_SCALAR) {
            // a + cos 2gamma B + sin 2gamma C = (a - B) + 2 cos gamma (cos gamma B
            // + sin gamma C), as cc^2 + ss^2 = 1/h^2: the records hold a - B,
            // 2 h^2 B and 2 h^2 C (the plate's signs included); the mask goes on
            // the beam value (every factor is finite)
            const float bTm = ZMASK ? bT : (in[k] ? bT : 0.0f);
            o.v0 += bTm * fmaf(cc, fmaf(R[k].b, cc, R[k].c * ss), R[k].a);
            continue;
        }
        const float c2 = fmaf(cc, cc, -ss * ss);   // cos(2gamma (+ 4phi)) / h^2
        const float sh = cc * ss;                  // sin(2gamma (+ 4phi)) / (2 h^2)
        if (MODE == MODE_TOD) {
            float term;
            {
                const float s2 = 2.0f * sh;
                const float sbU = sgn * bU;
                const float bq = fmaf(bQ, R[k].b, sbU * R[k].c);
                const float bu = fmaf(bQ, R[k].c, -sbU * R[k].b);
                term = fmaf(bI, R[k].a, fmaf(c2, bq, s2 * bu));
                if (Vp) term = fmaf(sgn * vb[k], vv[k], term);
            }
            o.v0 += in[k] ? term : 0.0f;
        } else {
            const float s2 = 2.0f * sh;
            o.v0 += in[k] ? bT * R[k].a : 0.0f;
            o.v1 += in[k] ? bT * fmaf(c2, R[k].b, s2 * R[k].c) : 0.0f;
            o.v2 += in[k] ? bT * (sgn * fmaf(-s2, R[k].b, c2 * R[k].c)) : 0.0f;
        }
        }
    }
    return o;
}

// Every lane (sample) against the staged records [0, m_end): TILE_NP records
// per step, then the remainder one by one.  CLIP (the disc-versus-grid test)
// and INNER (the inner-disc test of an annulus) are uniform per detector and
// template switches, so the common case runs a loop without either.
template <int MODE, int BEAM, bool PS, bool HWP, bool CLIP, bool INNER, int SC = 0, bool QF = false>
__device__ __forceinline__ void consume_records(const typename Cond<QF, PixRecQ, PixRec>::type *rec,
                                                const float *vrec, int32_t m_end, const PairCtx &C,
                                                const BeamRsrc &beam, const BeamRsrc &vbeam, AccWide &acc0,
                                                AccWide &acc1, AccWide &acc2, AccWide &accn) {
    // pairs whose beam loads are in flight together: four for one-grid beams (one
    // 16-byte cell record each), two for four-channel beams (four node records
    // each), so that a step's loaded records stay in registers
    constexpr int NP = BEAM == BEAM_SCALAR ? TILE_NP : 2;
    int32_t m = 0;
    // two groups per compensated add: 2 NP masked terms summed in FP32
    for (; m + 2 * NP - 1 < m_end; m += 2 * NP) {
        const PairOut a = tile_pairs<MODE, BEAM, PS, NP, HWP, CLIP, INNER, SC, QF>(
            &rec[m], vrec ? &vrec[m] : nullptr, C, beam, vbeam);
        const PairOut b = tile_pairs<MODE, BEAM, PS, NP, HWP, CLIP, INNER, SC, QF>(
            &rec[m + NP], vrec ? &vrec[m + NP] : nullptr, C, beam, vbeam);
        acc0.add(a.v0 + b.v0);
        if (MODE == MODE_STOKES) {
            acc1.add(a.v1 + b.v1);
            acc2.add(a.v2 + b.v2);
        }
        if (PS) accn.add(a.vn + b.vn);
    }
    for (; m + NP - 1 < m_end; m += NP) {
        const PairOut a = tile_pairs<MODE, BEAM, PS, NP, HWP, CLIP, INNER, SC, QF>(
            &rec[m], vrec ? &vrec[m] : nullptr, C, beam, vbeam);
        acc0.add(a.v0);
        if (MODE == MODE_STOKES) {
            acc1.add(a.v1);
            acc2.add(a.v2);
        }
        if (PS) accn.add(a.vn);
    }
    for (; m < m_end; ++m) {
        const PairOut a = tile_pairs<MODE, BEAM, PS, 1, HWP, CLIP, INNER, SC, QF>(&rec[m], vrec ? &vrec[m] : nullptr, C,
                                                                              beam, vbeam);
        acc0.add(a.v0);
        if (MODE == MODE_STOKES) {
            acc1.add(a.v1);
            acc2.add(a.v2);
        }
        if (PS) accn.add(a.vn);
    }
}

template <int MODE, int BEAM, int CH, bool PS, bool HWP>
__device__ void convolve_tile(const ConvArgs &A, const DetDesc &D, int64_t begin, int32_t cnt, TileLds<CH> &L,
                              float *vrec, int lane) {
    static_assert(CH % WAVE == 0, "chunks are whole waves of records");
    const float4 *__restrict__ sky = reinterpret_cast<const float4 *>(A.sky);
    const int32_t N = (int32_t)A.nside;
    const bool valid = lane < cnt;
    const int64_t t = sample_at(D, begin + (valid ? lane : 0));

    const TileFrame T = tile_setup(D, N, t, valid, &L.lane[lane]);
    const LaneFrame F = L.lane[lane];
    wave_sync();   // every lane holds its frame before records overwrite the slice
    const double phc = uniform(T.phc), zc = uniform(T.zc), sc = uniform(T.sc);
    const double cosRu = uniform(T.cosRu);
    const float zcf = (float)zc, scf = (float)sc;

    const int32_t n = D.n;
    const float inv_h = (float)D.inv_h;
    // one-grid TOD without a plate: the angle terms as a quadratic form in the
    // tangent-plane components of the carried theta'_0 (caps up to 60 deg, so
    // that the third component n_z >= 1/2 of every staged pixel stays large)
    const bool qf = MODE == MODE_TOD && BEAM == BEAM_SCALAR && !HWP && D.needs_clip == 0 && D.has_inner == 0 &&
                    cosRu >= 0.5;
    const float c0 = (float)(0.5 * (n - 1));
    const float tmax = (float)(n - 1);
    // the lane's theta'_0 and phi'_0 rows scaled to grid units for the pair loop
    LaneFrame Fg = F;
    Fg.a1 *= inv_h;
    Fg.a2 *= inv_h;
    Fg.a3 *= inv_h;
    Fg.b1 *= inv_h;
    Fg.b2 *= inv_h;
    Fg.b3 *= inv_h;
    // omin = -1 without an inner disc, so `omg > omin` holds for every pixel (omg >= 0)
    const float omax = (float)D.omega_max, omin = D.has_inner ? (float)D.omega_min : -1.0f;
    const bool inner = D.has_inner != 0;
    const bool clip = D.needs_clip != 0;
    const bool small_cap = D.omega_max <= SC_OMEGA;    // reciprocal-free pair geometry (see tile_pairs)
    const bool tiny_cap = D.omega_max <= SC2_OMEGA;
    // the quadratic-form records' series orders (the bound on |t| uses the union radius)
    const double tb = fmax(D.omega_max, (1.0 - cosRu) / cosRu);
    const bool tiny_q = tiny_cap && tb <= SCT2, small_q = small_cap && tb <= SCT1;
    const float wI = (float)D.w[0], wQ = (float)D.w[1], wU = (float)D.w[2];
    const float cmax = (float)(n - 2);          // largest cell index
    const float row = (float)(BEAM == BEAM_SCALAR ? n + 1 : n);
    const float ringoff = BEAM == BEAM_SCALAR ? 1.0f : 0.0f;   // one-grid t counts from the extrapolated ring
    // beam records through a buffer resource: 32-bit byte offsets, reads past
    // the end return zero
    const uint32_t nrec = (uint32_t)(BEAM == BEAM_SCALAR ? (n + 1) * (n + 1) : n * n);
    const BeamRsrc beam = BEAM == BEAM_SCALAR ? make_cell_rsrc(D.beam, nrec) : make_beam_rsrc(D.beam, nrec);
    const int32_t row_bytes = __builtin_amdgcn_readfirstlane(16 * n);   // buffer-load soffset: must stay in an SGPR
    // full beams with a V column: bV cell polynomials, and the V of each staged pixel
    const bool has_v = (BEAM == BEAM_FULL) && (MODE == MODE_TOD) && D.beam_v != nullptr && vrec != nullptr;
    const BeamRsrc vbeam = make_beam_rsrc(has_v ? D.beam_v : D.beam, (uint32_t)((n - 1) * (n - 1)));
    // half-wave plate: U-row and V terms change sign (records of one-grid beams carry it)
    const float sg4 = D.hwp ? -1.0f : 1.0f;
    const float wV = (float)D.wv;
    const float rz0 = (float)D.rot2z[0], rz1 = (float)D.rot2z[1];   // (cos 2 zeta, sin 2 zeta) h^2
    const float ih2 = (float)(D.inv_h * D.inv_h);

    AccWide acc0, acc1, acc2, accn;
    int32_t npairs = 0;

    const int32_t r_lo = __builtin_amdgcn_readfirstlane(T.r_lo), r_hi = __builtin_amdgcn_readfirstlane(T.r_hi);

    const LaneHull H = lane_hull(D, t, valid, phc, zc, sc);
    const float4 hull_mine = make_float4(valid ? H.dth : 16.0f, H.rsl, H.dphl, 0.0f);
    for (int32_t rb = r_lo; rb <= r_hi; rb += WAVE) {
        const int32_t r = rb + lane;
        int32_t rc = 0;
        if (r <= r_hi) rc = union_ring_setup(N, r, phc, zc, sc, cosRu, &L.ring[lane]);
        if (H.ok) {
            // the lanes' discs, staged where the records go (free between batches)
            float4 *hull = reinterpret_cast<float4 *>(L.rec);
            hull[lane] = hull_mine;
            wave_sync();
            narrow_rings_lanes(L.ring, rc, min(WAVE, r_hi - rb + 1), hull, cnt, H.R, lane);
            wave_sync();
        }
        const int32_t incl = wave_inclusive_scan(rc, lane);
        L.seg_end[lane] = incl;
        const int32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, WAVE - 1, WAVE));
        wave_sync();

        // ring of the chunk's first record, or an earlier one: each lane's search
        // starts there instead of at the batch's first ring
        int32_t seg0 = 0;
        for (int32_t pb = 0; pb < total; pb += CH) {
            const int32_t m_end = min(CH, total - pb);
            // fill: one pixel record per lane, FP32 differences from the centre
            int32_t seg = seg0;
            for (int32_t m = lane; m < m_end; m += WAVE) {
                const int32_t f = pb + m;
                while (f >= L.seg_end[seg]) ++seg;
                const int32_t start = (seg == 0) ? 0 : L.seg_end[seg - 1];
                const UnionRing &u = L.ring[seg];
                const int32_t rn = u.n, half = rn >> 1;
                int32_t kk = u.lo + (f - start);
                if (kk >= half) kk -= rn;
                if (kk >= half) kk -= rn;
                if (kk < -half) kk += rn;
                int32_t j = u.jc + kk;
                if (j < 0) j += rn;
                else if (j >= rn) j -= rn;
                const float dph = fmaf((float)kk, u.dphi, u.dphic);
                float sh, ch;
                half_sincos(0.5f * dph, sh, ch);
                const float h = 2.0f * sh * sh;  // 1 - cos(dphi)
                const float S = 2.0f * sh * ch;  // sin(dphi)
                PixRec R;
                R.X = fmaf(-u.b, h, u.a);
                R.Y = u.s * S;
                R.W = fmaf(u.c, h, u.e);
                R.t1 = fmaf(-u.f, h, u.cdt);
                R.t2 = u.z * S;
                R.t3 = fmaf(-u.g, h, -u.a);
                R.f1 = -zcf * S;
                R.f2 = 1.0f - h;
                R.f3 = -scf * S;
                const float4 sv = sky[u.first + j];
                // Q, U coefficients turned by 2 zeta and scaled by h^2 (the pair
                // loop's angle terms are those of 2 gamma = 2 chi - 2 zeta, x 1/h^2)
                if (MODE == MODE_TOD && BEAM == BEAM_SCALAR) {
                    // B = wQ Q + wU U, C = wQ U - wU Q turned by 2 zeta (x h^2); the
                    // pair loop takes a - B, 2 B and 2 C (its cos^2 gamma form)
                    const float swU = sg4 * wU;
                    const float cq = fmaf(wQ, sv.y, swU * sv.z), cu = fmaf(wQ, sv.z, -swU * sv.y);
                    const float bh = fmaf(rz1, cu, rz0 * cq);
                    R.a = fmaf(-bh, ih2, fmaf(sg4 * wV, sv.w, wI * sv.x));
                    R.b = 2.0f * bh;
                    R.c = 2.0f * fmaf(rz0, cu, -rz1 * cq);
                } else {
                    R.a = sv.x;
                    R.b = fmaf(rz1, sv.z, rz0 * sv.y);
                    R.c = fmaf(rz0, sv.z, -rz1 * sv.y);
                }
                if (qf) {
                    // theta_hat and phi_hat reduced to the first two components
                    // (w_xy - (w_z / n_z) n_xy, the pair loop's tangent-plane dot
                    // product), then P = sym(theta~ (b theta~ + c phi~)^T)
                    const float nz = 1.0f - R.W;                             // n_z >= 1/2
                    const float rnz = __builtin_amdgcn_rcpf(nz);
                    const float tz = R.t3 * rnz, fz = R.f3 * rnz;
                    const float t1 = fmaf(-tz, R.X, R.t1), t2 = fmaf(-tz, R.Y, R.t2);
                    const float f1 = fmaf(-fz, R.X, R.f1), f2 = fmaf(-fz, R.Y, R.f2);
                    const float w1 = fmaf(R.b, t1, R.c * f1), w2 = fmaf(R.b, t2, R.c * f2);
                    PixRecQ Q;
                    Q.G1 = R.X * rnz;
                    Q.G2 = R.Y * rnz;
                    Q.W = R.W;
                    Q.Z = nz;
                    Q.ZX = nz * R.X;
                    Q.ZY = nz * R.Y;
                    Q.A = R.a;
                    Q.P11 = t1 * w1;
                    Q.P12 = fmaf(t1, w2, t2 * w1);
                    Q.P22 = t2 * w2;
                    Q.pad0 = 0.0f;
                    Q.pad1 = 0.0f;
                    reinterpret_cast<PixRecQ *>(L.rec)[m] = Q;
                } else {
                    L.rec[m] = R;
                }
                if (has_v) vrec[m] = sv.w;
            }
            // the last lane filled the chunk's last record (CH is a multiple of
            // the wave; only the batch's last chunk is partial)
            seg0 = __builtin_amdgcn_readlane(seg, WAVE - 1);
            wave_sync();

            // consume: every lane (sample) against every staged pixel
            if (valid) {
                if (MODE == MODE_COUNT) {
                    for (int32_t m = 0; m < m_end; ++m) {
                        const PixRec R = L.rec[m];
                        const float omg = fmaf(-R.Y, F.p2, fmaf(-R.X, F.p1, fmaf(R.W, F.p3, F.om)));
                        npairs += ((omg <= omax) & (omg > omin)) ? 1 : 0;
                    }
                } else {
                    // two records per step: their masked terms are added in FP32
                    // and the pair enters the compensated sums (halves the
                    // compensation work; each pre-sum rounds once)
                    const PairCtx C{Fg, omax, omin, clip, inv_h, c0 + ringoff, tmax + ringoff, cmax, row, row_bytes,
                                    sg4, (float)(n - 1), ringoff, (uint32_t)row};
                    const float *vr = has_v ? vrec : nullptr;
                    if constexpr (MODE == MODE_TOD && BEAM == BEAM_SCALAR && !HWP) {
                        if (qf) {
                            const PixRecQ *rq = reinterpret_cast<const PixRecQ *>(L.rec);
                            if (tiny_q)
                                consume_records<MODE, BEAM, PS, HWP, false, false, 2, true>(rq, vr, m_end, C, beam, vbeam,
                                                                                            acc0, acc1, acc2, accn);
                            else if (small_q)
                                consume_records<MODE, BEAM, PS, HWP, false, false, 1, true>(rq, vr, m_end, C, beam, vbeam,
                                                                                            acc0, acc1, acc2, accn);
                            else
                                consume_records<MODE, BEAM, PS, HWP, false, false, 0, true>(rq, vr, m_end, C, beam, vbeam,
                                                                                            acc0, acc1, acc2, accn);
                            goto consumed;
                        }
                    }
                    if (clip) {
                        if (inner)
                            consume_records<MODE, BEAM, PS, HWP, true, true>(L.rec, vr, m_end, C, beam, vbeam, acc0,
                                                                             acc1, acc2, accn);
                        else
                            consume_records<MODE, BEAM, PS, HWP, true, false>(L.rec, vr, m_end, C, beam, vbeam, acc0,
                                                                              acc1, acc2, accn);
                    } else {
                        if (inner)
                            consume_records<MODE, BEAM, PS, HWP, false, true>(L.rec, vr, m_end, C, beam, vbeam, acc0,
                                                                              acc1, acc2, accn);
                        else if (tiny_cap)
                            consume_records<MODE, BEAM, PS, HWP, false, false, 2>(L.rec, vr, m_end, C, beam, vbeam,
                                                                                  acc0, acc1, acc2, accn);
                        else if (small_cap)
                            consume_records<MODE, BEAM, PS, HWP, false, false, 1>(L.rec, vr, m_end, C, beam, vbeam,
                                                                                  acc0, acc1, acc2, accn);
                        else
                            consume_records<MODE, BEAM, PS, HWP, false, false>(L.rec, vr, m_end, C, beam, vbeam, acc0,
                                                                               acc1, acc2, accn);
                    }
                }
            }
        consumed:
            wave_sync();
        }
    }

    if (!valid) return;
    float *out = reinterpret_cast<float *>(A.out);
    const int64_t o = D.out_offset + t;
    if (MODE == MODE_COUNT) {
        out[o] = (float)npairs;
        return;
    }
    double Nrm = D.norm_scale;
    if (PS && D.norm_mode == 1) {
        const double snm = accn.value() * (BEAM == BEAM_SCALAR ? D.w[3] : 1.0);
        Nrm = (snm != 0.0) ? D.norm_scale / snm : 0.0;
    }
    if (MODE == MODE_TOD) {
        out[o] = (float)(acc0.value() * Nrm);
    } else {
        if (BEAM == BEAM_SCALAR) Nrm *= D.w[3];
        out[3 * o + 0] = (float)(acc0.value() * Nrm);
        out[3 * o + 1] = (float)(acc1.value() * Nrm);
        out[3 * o + 2] = (float)(acc2.value() * Nrm);
    }
}

// ----------------------------------------------------------------------
// Sample-parallel path with the pixel-linear parts of every pair on the
// matrix cores.  For a tile of 64 samples and a group of 16 staged pixels,
// FP32 MFMAs (16 x 16 x 4) form, for every (pixel, sample) pair, the
// quantities that are linear in the pixel record:
//   1 - n.p, n.theta'_0, n.phi'_0, g.n   on the pixel basis (1, X, Y, W)
//   g.theta_hat_k, p.theta_hat_k         on the pixel basis (t1, t2, t3, 0)
//   g.phi_hat_k, p.phi_hat_k             on the pixel basis (f1, f2, f3, 0)
// with g the co-polar direction at the boresight.  The co-polar vector carried
// to the pixel, e = g - q (p + n) with q = g.n / (1 + n.p), projects on the
// pixel's basis as e.theta_hat_k = g.theta_hat_k - q p.theta_hat_k (theta_hat_k
// and phi_hat_k are normal to n), so only the nonlinear steps of a pair run on
// the vector ALU.  MFMA operands: A = pixel basis (lane l: pixel l % 16,
// component l / 16), B = per-sample coefficients (lane l: component l / 16,
// sample l % 16 of a 16-sample block); lane l receives pixels 4 (l / 16) + i
// for sample l % 16 and keeps that sample's sums, reduced over the four lane
// groups at the end of the tile.
// ----------------------------------------------------------------------
template <int CH, int NACC>
struct TileLdsMx {
    UnionRing ring[WAVE];
    LaneFrame lane[WAVE];
    int32_t seg_end[WAVE];
    float b1[4][CH];          // (1, X, Y, W)
    float bt[4][CH];          // the pixel's theta_hat (t1, t2, t3, 0)
    float bf[4][CH];          // the pixel's phi_hat (f1, f2, f3, 0)
    float4 sky[CH];           // (a, b, c, 0) as in PixRec
    float acc[4][NACC][WAVE]; // running sums of the four 16-sample blocks
};

template <int MODE>
constexpr int mx_nacc() { return MODE == MODE_STOKES ? 8 : 4; }

typedef float mx4 __attribute__((ext_vector_type(4)));

__device__ inline mx4 mx(float a, float b) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, mx4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
}

// Compensated sums over the four lane groups l / 16 (lanes l, l ^ 16, l ^ 32, l ^ 48).
__device__ inline void reduce_groups(Acc<float> &a) {
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) {
        const float os = __shfl_xor(a.s, m, WAVE);
        const float oc = __shfl_xor(a.c, m, WAVE);
        a.add(os);
        a.c += oc;
    }
}

template <int MODE, int BEAM, int CH, bool PS>
__device__ void convolve_tile_mx(const ConvArgs &A, const DetDesc &D, int64_t begin, int32_t cnt,
                                 TileLdsMx<CH, mx_nacc<MODE>()> &L, int lane) {
    constexpr int NACC = mx_nacc<MODE>();
    static_assert(CH % WAVE == 0, "chunks are whole waves of records");
    const float4 *__restrict__ sky = reinterpret_cast<const float4 *>(A.sky);
    const int32_t N = (int32_t)A.nside;
    const bool valid = lane < cnt;
    const int64_t t = sample_at(D, begin + (valid ? lane : 0));

    const TileFrame T = tile_setup(D, N, t, valid, &L.lane[lane]);
    const double phc = uniform(T.phc), zc = uniform(T.zc), sc = uniform(T.sc);
    const double cosRu = uniform(T.cosRu);
    const float zcf = (float)zc, scf = (float)sc;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int a = 0; a < NACC; ++a) L.acc[j][a][lane] = 0.0f;
    wave_sync();  // lanes read the frames of a 16-sample block below

    const int32_t n = D.n;
    const float inv_h = (float)D.inv_h;
    const float c0 = (float)(0.5 * (n - 1));
    const float tmax = (float)(n - 1);
    // omin = -1 without an inner disc, so `omg > omin` holds for every pixel (omg >= 0)
    const float omax = (float)D.omega_max, omin = D.has_inner ? (float)D.omega_min : -1.0f;
    const bool clip = D.needs_clip != 0;
    const float wI = (float)D.w[0], wQ = (float)D.w[1], wU = (float)D.w[2];
    const float cmax = (float)(n - 2);
    const float row = (float)(BEAM == BEAM_SCALAR ? n + 1 : n);
    const float kbase = BEAM == BEAM_SCALAR ? row + 1.0f : 0.0f;   // cell (0, 0) past the extrapolated ring
    const uint32_t nrec = (uint32_t)(BEAM == BEAM_SCALAR ? (n + 1) * (n + 1) : n * n);
    const BeamRsrc beam = make_beam_rsrc(D.beam, nrec);
    const int32_t row_bytes = __builtin_amdgcn_readfirstlane(16 * n);   // buffer-load soffset: must stay in an SGPR
    const int k4 = lane >> 4, c16 = lane & 15;

    const int32_t r_lo = __builtin_amdgcn_readfirstlane(T.r_lo), r_hi = __builtin_amdgcn_readfirstlane(T.r_hi);

    const LaneHull H = lane_hull(D, t, valid, phc, zc, sc);
    for (int32_t rb = r_lo; rb <= r_hi; rb += WAVE) {
        const int32_t r = rb + lane;
        int32_t rc = 0;
        if (r <= r_hi) rc = union_ring_setup(N, r, phc, zc, sc, cosRu, &L.ring[lane]);
        if (H.ok) {
            wave_sync();
            narrow_rings(L.ring, rc, min(WAVE, r_hi - rb + 1), H, valid, lane);
            wave_sync();
        }
        const int32_t incl = wave_inclusive_scan(rc, lane);
        L.seg_end[lane] = incl;
        const int32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, WAVE - 1, WAVE));
        wave_sync();

        int32_t seg0 = 0;   // as in the vector tile kernel
        for (int32_t pb = 0; pb < total; pb += CH) {
            const int32_t m_end = min(CH, total - pb);
            const int32_t m_pad = (m_end + 15) & ~15;
            // fill: one pixel record per lane; padding records lie outside every disc
            int32_t seg = seg0;
            for (int32_t m = lane; m < m_pad; m += WAVE) {
                if (m < m_end) {
                    const int32_t f = pb + m;
                    while (f >= L.seg_end[seg]) ++seg;
                    const int32_t start = (seg == 0) ? 0 : L.seg_end[seg - 1];
                    const UnionRing &u = L.ring[seg];
                    const int32_t rn = u.n, half = rn >> 1;
                    int32_t kk = u.lo + (f - start);
                    if (kk >= half) kk -= rn;
                    if (kk >= half) kk -= rn;
                    if (kk < -half) kk += rn;
                    int32_t j = u.jc + kk;
                    if (j < 0) j += rn;
                    else if (j >= rn) j -= rn;
                    const float dph = fmaf((float)kk, u.dphi, u.dphic);
                    float sh, ch;
                    half_sincos(0.5f * dph, sh, ch);
                    const float h = 2.0f * sh * sh;  // 1 - cos(dphi)
                    const float S = 2.0f * sh * ch;  // sin(dphi)
                    L.b1[0][m] = 1.0f;
                    L.b1[1][m] = fmaf(-u.b, h, u.a);
                    L.b1[2][m] = u.s * S;
                    L.b1[3][m] = fmaf(u.c, h, u.e);
                    L.bt[0][m] = fmaf(-u.f, h, u.cdt);
                    L.bt[1][m] = u.z * S;
                    L.bt[2][m] = fmaf(-u.g, h, -u.a);
                    L.bt[3][m] = 0.0f;
                    L.bf[0][m] = -zcf * S;
                    L.bf[1][m] = 1.0f - h;
                    L.bf[2][m] = -scf * S;
                    L.bf[3][m] = 0.0f;
                    const float4 sv = sky[u.first + j];
                    float4 rec;
                    if (MODE == MODE_TOD && BEAM == BEAM_SCALAR) {
                        rec.x = wI * sv.x;
                        rec.y = fmaf(wQ, sv.y, wU * sv.z);
                        rec.z = 2.0f * fmaf(wQ, sv.z, -wU * sv.y);
                    } else {
                        rec.x = sv.x;
                        rec.y = sv.y;
                        rec.z = sv.z;
                    }
                    rec.w = 0.0f;
                    L.sky[m] = rec;
                } else {
                    // 1 - n.p = om + 4 p3 > 1 for every sample: never inside a disc
                    L.b1[0][m] = 1.0f;
                    L.b1[1][m] = 0.0f;
                    L.b1[2][m] = 0.0f;
                    L.b1[3][m] = 4.0f;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        L.bt[c][m] = 0.0f;
                        L.bf[c][m] = 0.0f;
                    }
                    L.sky[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
            }
            seg0 = __builtin_amdgcn_readlane(seg, WAVE - 1);
            wave_sync();

            // one pass per 16-sample block: its coefficients and running sums
            // come from LDS, so little stays live across the pixel groups
#pragma unroll 1
            for (int jb = 0; jb < 4; ++jb) {
                const LaneFrame &G = L.lane[16 * jb + c16];
                const float Bo = k4 == 0 ? G.om : k4 == 1 ? -G.p1 : k4 == 2 ? -G.p2 : G.p3;
                if (MODE == MODE_COUNT) {
                    float cntf = L.acc[jb][0][lane];
                    for (int32_t g = 0; g < m_pad; g += 16) {
                        const mx4 vo = mx(L.b1[k4][g + c16], Bo);
#pragma unroll
                        for (int q = 0; q < 4; ++q) cntf += ((vo[q] <= omax) & (vo[q] > omin)) ? 1.0f : 0.0f;
                    }
                    L.acc[jb][0][lane] = cntf;
                    continue;
                }
                const float Bx = k4 == 0 ? G.a3 : k4 == 1 ? G.a1 : k4 == 2 ? G.a2 : -G.a3;
                const float By = k4 == 0 ? G.b3 : k4 == 1 ? G.b1 : k4 == 2 ? G.b2 : -G.b3;
                const float Bn = k4 == 0 ? G.g3 : k4 == 1 ? G.g1 : k4 == 2 ? G.g2 : -G.g3;
                const float Bg = k4 == 0 ? G.g1 : k4 == 1 ? G.g2 : k4 == 2 ? G.g3 : 0.0f;
                const float Bp = k4 == 0 ? G.p1 : k4 == 1 ? G.p2 : k4 == 2 ? G.p3 : 0.0f;
                Acc<float> a0, a1s, a2s, an;
                a0.s = L.acc[jb][0][lane];
                a0.c = L.acc[jb][1][lane];
                if (PS) {
                    an.s = L.acc[jb][2][lane];
                    an.c = L.acc[jb][3][lane];
                }
                if (MODE == MODE_STOKES) {
                    a1s.s = L.acc[jb][4][lane];
                    a1s.c = L.acc[jb][5][lane];
                    a2s.s = L.acc[jb][6][lane];
                    a2s.c = L.acc[jb][7][lane];
                }
                for (int32_t g = 0; g < m_pad; g += 16) {
                    const float p1v = L.b1[k4][g + c16], ptv = L.bt[k4][g + c16], pfv = L.bf[k4][g + c16];
                    const mx4 vo = mx(p1v, Bo), vx = mx(p1v, Bx), vy = mx(p1v, By), vn = mx(p1v, Bn);
                    const mx4 gt = mx(ptv, Bg), pt = mx(ptv, Bp), gf = mx(pfv, Bg), pf = mx(pfv, Bp);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float4 sk = L.sky[g + 4 * k4 + q];
                        const float omg = vo[q];  // 1 - n.p
                        bool in = (omg <= omax) & (omg > omin);
                        const float rz = rcp(1.0f - omg);
                        const float su = vx[q] * rz, sv = vy[q] * rz;  // gnomonic u, v
                        const float tu = fmaf(su, inv_h, c0);
                        const float tv = fmaf(sv, inv_h, c0);
                        if (clip) in = in & (tu >= 0.0f) & (tu <= tmax) & (tv >= 0.0f) & (tv <= tmax);
                        const float ku = floorf(__builtin_amdgcn_fmed3f(tu, 0.0f, cmax));
                        const float kv = floorf(__builtin_amdgcn_fmed3f(tv, 0.0f, cmax));
                        const float fu = fmaf(su, inv_h, c0 - ku), fv = fmaf(sv, inv_h, c0 - kv);
                        // one-grid records: padded cell (ku + 1, kv + 1) in row pairs
                        const uint32_t off =
                            BEAM == BEAM_SCALAR
                                ? (uint32_t)cell_index((int64_t)ku + 1, (int64_t)kv + 1, (int64_t)row) << 4
                                : (uint32_t)fmaf(kv, row, ku + kbase) << 4;
                        float bT, bI = 0.0f, bQ = 0.0f, bU = 0.0f;
                        if (BEAM == BEAM_SCALAR) {
                            const float4 cl = beam_ld(beam, off, 0);
                            bT = fmaf(fv, fmaf(fu, cl.w, cl.z), fmaf(fu, cl.y, cl.x));
                        } else {
                            const float4 q00 = beam_ld(beam, off, 0), q10 = beam_ld(beam, off + 16, 0),
                                         q01 = beam_ld(beam, off, row_bytes),
                                         q11 = beam_ld(beam, off + 16, row_bytes);
                            bI = lerp(lerp(q00.x, q10.x, fu), lerp(q01.x, q11.x, fu), fv);
                            bQ = lerp(lerp(q00.y, q10.y, fu), lerp(q01.y, q11.y, fu), fv);
                            bU = lerp(lerp(q00.z, q10.z, fu), lerp(q01.z, q11.z, fu), fv);
                            bT = lerp(lerp(q00.w, q10.w, fu), lerp(q01.w, q11.w, fu), fv);
                        }
                        const float qq = vn[q] * rcp(2.0f - omg);
                        const float cc = fmaf(-qq, pt[q], gt[q]);  // e . theta_hat_k
                        const float ss = fmaf(-qq, pf[q], gf[q]);  // e . phi_hat_k
                        const float c2 = fmaf(cc, cc, -ss * ss);
                        if (PS) an.add(in ? bT : 0.0f);
                        if (MODE == MODE_TOD) {
                            float term;
                            if (BEAM == BEAM_SCALAR) {
                                term = bT * fmaf(c2, sk.y, fmaf(cc * ss, sk.z, sk.x));
                            } else {
                                const float s2 = 2.0f * cc * ss;
                                const float bq = fmaf(bQ, sk.y, bU * sk.z);
                                const float bu = fmaf(bQ, sk.z, -bU * sk.y);
                                term = fmaf(bI, sk.x, fmaf(c2, bq, s2 * bu));
                            }
                            a0.add(in ? term : 0.0f);
                        } else {
                            const float s2 = 2.0f * cc * ss;
                            a0.add(in ? bT * sk.x : 0.0f);
                            a1s.add(in ? bT * fmaf(c2, sk.y, s2 * sk.z) : 0.0f);
                            a2s.add(in ? bT * fmaf(-s2, sk.y, c2 * sk.z) : 0.0f);
                        }
                    }
                }
                L.acc[jb][0][lane] = a0.s;
                L.acc[jb][1][lane] = a0.c;
                if (PS) {
                    L.acc[jb][2][lane] = an.s;
                    L.acc[jb][3][lane] = an.c;
                }
                if (MODE == MODE_STOKES) {
                    L.acc[jb][4][lane] = a1s.s;
                    L.acc[jb][5][lane] = a1s.c;
                    L.acc[jb][6][lane] = a2s.s;
                    L.acc[jb][7][lane] = a2s.c;
                }
            }
            wave_sync();
        }
    }

    float *out = reinterpret_cast<float *>(A.out);
#pragma unroll 1
    for (int jb = 0; jb < 4; ++jb) {
        const int smp = 16 * jb + c16;
        if (MODE == MODE_COUNT) {
            float v = L.acc[jb][0][lane];
            v += __shfl_xor(v, 16, WAVE);
            v += __shfl_xor(v, 32, WAVE);
            if (k4 == 0 && smp < cnt) out[D.out_offset + sample_at(D, begin + smp)] = v;
            continue;
        }
        Acc<float> a0, a1s, a2s, an;
        a0.s = L.acc[jb][0][lane];
        a0.c = L.acc[jb][1][lane];
        reduce_groups(a0);
        if (PS) {
            an.s = L.acc[jb][2][lane];
            an.c = L.acc[jb][3][lane];
            reduce_groups(an);
        }
        if (MODE == MODE_STOKES) {
            a1s.s = L.acc[jb][4][lane];
            a1s.c = L.acc[jb][5][lane];
            a2s.s = L.acc[jb][6][lane];
            a2s.c = L.acc[jb][7][lane];
            reduce_groups(a1s);
            reduce_groups(a2s);
        }
        if (k4 != 0 || smp >= cnt) continue;
        double Nrm = D.norm_scale;
        if (PS && D.norm_mode == 1) {
            const double snm = an.value() * (BEAM == BEAM_SCALAR ? D.w[3] : 1.0);
            Nrm = (snm != 0.0) ? D.norm_scale / snm : 0.0;
        }
        const int64_t o = D.out_offset + sample_at(D, begin + smp);
        if (MODE == MODE_TOD) {
            out[o] = (float)(a0.value() * Nrm);
        } else {
            if (BEAM == BEAM_SCALAR) Nrm *= D.w[3];
            out[3 * o + 0] = (float)(a0.value() * Nrm);
            out[3 * o + 1] = (float)(a1s.value() * Nrm);
            out[3 * o + 2] = (float)(a2s.value() * Nrm);
        }
    }
}

// Whether a group of consecutive samples overlaps enough for the tile path:
// its samples lie within `frac` disc radii of their mean direction.
__device__ inline bool tile_is_coherent(const DetDesc &D, int64_t begin, int32_t cnt, int lane, double frac) {
    const bool valid = lane < cnt;
    const int64_t t = sample_at(D, begin + (valid ? lane : 0));
    double st, ct, sf, cf;
    sincos(D.theta[t], &st, &ct);
    sincos(D.phi[t], &sf, &cf);
    const double p[3] = {st * cf, st * sf, ct};
    double sx = valid ? p[0] : 0.0, sy = valid ? p[1] : 0.0, sz = valid ? p[2] : 0.0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        sx += __shfl_xor(sx, m, WAVE);
        sy += __shfl_xor(sy, m, WAVE);
        sz += __shfl_xor(sz, m, WAVE);
    }
    const double sn = sqrt(sx * sx + sy * sy + sz * sz);
    if (!(sn > 0.5 * cnt)) return false;
    const double dx = p[0] - sx / sn, dy = p[1] - sy / sn, dz = p[2] - sz / sn;
    double d = valid ? sqrt(dx * dx + dy * dy + dz * dz) : 0.0;  // chord
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d = fmax(d, __shfl_xor(d, m, WAVE));
    const double lim = frac * D.rho_max;
    return (d <= lim) && (D.rho_max + lim < 0.45 * PI);
}

// ----------------------------------------------------------------------
// Kernels
// ----------------------------------------------------------------------
// Next tile of queue q for the calling wave (lane 0): a plain load first, so
// waves that find a queue drained add nothing to the atomics its counter
// serialises (thousands of waves checking every queue at the end of a launch).
// The counter only grows, so a stale load at worst leads to the atomic.
__device__ inline int32_t pop_tile(int32_t *counter, int32_t len) {
    if (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) return len;
    return atomicAdd(counter, 1);
}

template <typename T, int MODE, int BEAM>
__global__ void __launch_bounds__(512) conv_kernel(ConvArgs A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    WaveLds<T> &L = reinterpret_cast<WaveLds<T> *>(lds_raw)[wid];
    int32_t q = (A.n_queues > 1) ? (int32_t)(blockIdx.x % (uint32_t)A.n_queues) : 0;
    int32_t exhausted = 0;
    while (exhausted < A.n_queues) {
        int32_t ti = 0;
        if (lane == 0) ti = pop_tile(&A.counters[q], A.queue_len[q]);
        ti = __shfl(ti, 0, WAVE);
        if (ti >= A.queue_len[q]) {
            q = (q + 1 == A.n_queues) ? 0 : q + 1;
            ++exhausted;
            continue;
        }
        const Tile tl = A.tiles[(int64_t)q * A.tiles_per_queue + ti];
        const DetDesc &D = A.dets[tl.det];
        for (int64_t t = tl.begin; t < tl.begin + tl.count; ++t) convolve_sample<T, MODE, BEAM>(A, D, t, L, lane);
    }
}

template <int MODE, int BEAM, int CH, bool PS, bool HWP>
__global__ void __launch_bounds__(512, (tile_min_waves<MODE, BEAM>())) tile_kernel(ConvArgs A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    TileLds<CH> &L = reinterpret_cast<TileLds<CH> *>(lds_raw)[wid];
    float *vrec = (BEAM == BEAM_FULL && MODE == MODE_TOD && A.vbeam)
                      ? reinterpret_cast<float *>(lds_raw + sizeof(TileLds<CH>) * (blockDim.x / WAVE)) + wid * CH
                      : nullptr;
    int32_t q = (A.n_queues > 1) ? (int32_t)(blockIdx.x % (uint32_t)A.n_queues) : 0;
    int32_t exhausted = 0;
    while (exhausted < A.n_queues) {
        int32_t ti = 0;
        if (lane == 0) ti = pop_tile(&A.counters[q], A.queue_len[q]);
        ti = __builtin_amdgcn_readfirstlane(__shfl(ti, 0, WAVE));
        if (ti >= A.queue_len[q]) {
            q = (q + 1 == A.n_queues) ? 0 : q + 1;
            ++exhausted;
            continue;
        }
        const Tile tl = A.tiles[(int64_t)q * A.tiles_per_queue + ti];
        const DetDesc &D = A.dets[tl.det];
        convolve_tile<MODE, BEAM, CH, PS, HWP>(A, D, tl.begin, tl.count, L, vrec, lane);
    }
}

template <int MODE, int BEAM, int CH, bool PS>
__global__ void __launch_bounds__(512, 2) tile_mx_kernel(ConvArgs A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wid = threadIdx.x / WAVE;
    TileLdsMx<CH, mx_nacc<MODE>()> &L = reinterpret_cast<TileLdsMx<CH, mx_nacc<MODE>()> *>(lds_raw)[wid];
    int32_t q = (A.n_queues > 1) ? (int32_t)(blockIdx.x % (uint32_t)A.n_queues) : 0;
    int32_t exhausted = 0;
    while (exhausted < A.n_queues) {
        int32_t ti = 0;
        if (lane == 0) ti = pop_tile(&A.counters[q], A.queue_len[q]);
        ti = __builtin_amdgcn_readfirstlane(__shfl(ti, 0, WAVE));
        if (ti >= A.queue_len[q]) {
            q = (q + 1 == A.n_queues) ? 0 : q + 1;
            ++exhausted;
            continue;
        }
        const Tile tl = A.tiles[(int64_t)q * A.tiles_per_queue + ti];
        const DetDesc &D = A.dets[tl.det];
        convolve_tile_mx<MODE, BEAM, CH, PS>(A, D, tl.begin, tl.count, L, lane);
        wave_sync();  // the next tile's set-up overwrites the frames this one read
    }
}

// One wavefront per group of up to 64 consecutive samples: flag[g] = 1 when the
// group is coherent enough for the tile path.
__global__ void classify_kernel(const DetDesc *dets, const Tile *groups, int32_t n_groups, double frac,
                                int32_t *flag) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int32_t g = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    if (g >= n_groups) return;
    const Tile tl = groups[g];
    const bool ok = tile_is_coherent(dets[tl.det], tl.begin, tl.count, lane, frac);
    if (lane == 0) flag[g] = ok ? 1 : 0;
}

// Clear the work counters of both queue sets: ints [0, 8) and [16, 24) of the
// plan's control block ([8, 16) and [24, 32) hold the queue lengths).
__global__ void zero_counters_kernel(int32_t *c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (i & 8) == 0) c[i] = 0;
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

// Scalar beam: one record per cell holding the bilinear interpolant of its
// four corner nodes as a polynomial in the cell fractions (fu, fv):
// b = b00 + fu (b10 - b00) + fv (b01 - b00) + fu fv (b11 - b10 - b01 + b00).
// The differences are formed in FP64 and rounded once.
// HEALPix beam maps (beam at the map's north pole, theta = rho, phi = sigma)
// resampled onto the n x n gnomonic node grid ([v][u] over [-T, T]^2): per
// node, linear in phi between the two bracketing pixels of each of the two
// rings that bracket theta, then linear in theta between the rings; above the
// first ring (below the last) the pole, valued at the mean of that ring's four
// pixels, takes the place of the missing ring.  FP64 arithmetic.
__device__ inline double ring_theta(int32_t N, int32_t r) {
    const RingGeom g = ring_geom(N, r);
    return atan2(g.s, g.z);
}

template <typename T>
__device__ inline double ring_read(const T *__restrict__ map, const RingGeom &g, double phi) {
    const double x = (phi - g.phi0) / g.dphi;
    const double fl = floor(x);
    const double w = x - fl;
    int64_t j0 = (int64_t)fl % g.n;
    if (j0 < 0) j0 += g.n;
    const int64_t j1 = (j0 + 1 == g.n) ? 0 : j0 + 1;
    return (1.0 - w) * (double)map[g.first + j0] + w * (double)map[g.first + j1];
}

template <typename T>
__global__ void __launch_bounds__(256) healpix_grid_kernel(HpxGridArgs a) {
    const int64_t nodes = (int64_t)a.n * a.n;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nodes) return;
    const int32_t iu = (int32_t)(k % a.n), iv = (int32_t)(k / a.n);
    const double h = 2.0 * a.T / (double)(a.n - 1);
    const double u = -a.T + iu * h, v = -a.T + iv * h;
    const double th = atan(sqrt(u * u + v * v)), ph = atan2(v, u);
    const int32_t N = a.nside, nring = 4 * N - 1;
    const int64_t npix = 12 * (int64_t)N * N;
    const double th1 = ring_theta(N, 1), thl = ring_theta(N, nring);
    int mode = 0;            // 0: between rings ra and ra + 1; 1: north pole and ring 1; 2: ring nring and south pole
    int32_t ra = 1;
    double t;
    if (th < th1) {
        mode = 1;
        t = th / th1;
    } else if (th >= thl) {
        mode = 2;
        t = (PI - th) / (PI - thl);
        ra = nring;
    } else {
        ra = (int32_t)floor(ring_of_theta(N, th));
        ra = ra < 1 ? 1 : (ra > nring - 1 ? nring - 1 : ra);
        while (ra > 1 && ring_theta(N, ra) > th) --ra;
        while (ra + 1 < nring && ring_theta(N, ra + 1) <= th) ++ra;
        const double ta = ring_theta(N, ra), tb = ring_theta(N, ra + 1);
        t = (th - ta) / (tb - ta);
    }
    const RingGeom ga = ring_geom(N, mode == 1 ? 1 : ra);
    const RingGeom gb = ring_geom(N, mode == 0 ? ra + 1 : ra);
    for (int c = 0; c < a.nch; ++c) {
        const T *__restrict__ m = static_cast<const T *>(a.map[c]);
        double val;
        if (mode == 1) {
            const double pole = 0.25 * ((double)m[0] + (double)m[1] + (double)m[2] + (double)m[3]);
            val = (1.0 - t) * pole + t * ring_read(m, ga, ph);
        } else if (mode == 2) {
            const double pole =
                0.25 * ((double)m[npix - 4] + (double)m[npix - 3] + (double)m[npix - 2] + (double)m[npix - 1]);
            val = (1.0 - t) * pole + t * ring_read(m, ga, ph);
        } else {
            val = (1.0 - t) * ring_read(m, ga, ph) + t * ring_read(m, gb, ph);
        }
        static_cast<T *>(a.out[c])[k] = (T)val;
    }
}

// Cell polynomials (b00, b10 - b00, b01 - b00, b11 - b10 - b01 + b00) of the
// (n - 1)^2 grid cells, row-major; with `padded`, (n + 1)^2 records: a ring of
// cells one step outside the grid whose polynomials continue those of the
// nearest edge cell (P(x + du, y + dv) with du, dv in {-1, 0, 1}), the interior
// unchanged, stored in the row-pair order of cell_index.
template <typename T>
__global__ void repack_cells_kernel(const T *b, int32_t n, typename Rec4<T>::type *out, bool padded) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t side = padded ? n + 1 : n - 1;
    const int64_t m = (int64_t)side * side;
    if (i >= m) return;
    const int32_t iv = (int32_t)(i / side) - (padded ? 1 : 0), iu = (int32_t)(i % side) - (padded ? 1 : 0);
    const int32_t cv = min(max(iv, 0), n - 2), cu = min(max(iu, 0), n - 2);
    const int64_t k = (int64_t)cv * n + cu;
    const double b00 = b[k], b10 = b[k + 1], b01 = b[k + n], b11 = b[k + n + 1];
    const double c00 = b00, c10 = b10 - b00, c01 = b01 - b00, c11 = (b11 - b10) - (b01 - b00);
    typename Rec4<T>::type r;
    if (iu == cu && iv == cv) {
        r.x = (T)c00;
        r.y = (T)c10;
        r.z = (T)c01;
        r.w = (T)c11;
    } else {
        const double du = (double)(iu - cu), dv = (double)(iv - cv);
        r.x = (T)(c00 + c10 * du + c01 * dv + c11 * du * dv);
        r.y = (T)(c10 + c11 * dv);
        r.z = (T)(c01 + c11 * du);
        r.w = (T)c11;
    }
    if (padded)
        out[cell_index(iu + 1, iv + 1, side)] = r;   // rows in interleaved pairs (side = n + 1 is even)
    else
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

template <typename T, int MODE>
static hipError_t launch_pixel(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    const size_t lds = sizeof(WaveLds<T>) * (size_t)waves;
    if (a.beam_kind == BEAM_FULL)
        hipLaunchKernelGGL((conv_kernel<T, MODE, BEAM_FULL>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    else
        hipLaunchKernelGGL((conv_kernel<T, MODE, BEAM_SCALAR>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    return hipGetLastError();
}

template <int MODE, int BEAM, int CH, bool PS, bool HWP>
static hipError_t launch_tile_h(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    const bool v = BEAM == BEAM_FULL && MODE == MODE_TOD && a.vbeam;
    const size_t lds = (sizeof(TileLds<CH>) + (v ? sizeof(float) * CH : 0)) * (size_t)waves;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {  // allow the larger LDS allocations of gfx950 (160 KiB per CU)
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&tile_kernel<MODE, BEAM, CH, PS, HWP>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((tile_kernel<MODE, BEAM, CH, PS, HWP>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    return hipGetLastError();
}

template <int MODE, int BEAM, int CH, bool PS>
static hipError_t launch_tile_t(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    if (MODE != MODE_COUNT && a.hwp) return launch_tile_h<MODE, BEAM, CH, PS, true>(a, waves, groups, s);
    return launch_tile_h<MODE, BEAM, CH, PS, false>(a, waves, groups, s);
}

template <int MODE, int BEAM, int CH, bool PS>
static hipError_t launch_tile_mx_t(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    // the Stokes sums need more LDS per wave: keep a workgroup within one
    // compute unit's 160 KiB by splitting it (waves are independent)
    const size_t slice = sizeof(TileLdsMx<CH, mx_nacc<MODE>()>);
    const int wmax = (int)((160 * 1024) / slice);
    if (waves > wmax) {
        groups = (int)(((int64_t)groups * waves + wmax - 1) / wmax);
        waves = wmax;
    }
    const size_t lds = slice * (size_t)waves;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&tile_mx_kernel<MODE, BEAM, CH, PS>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((tile_mx_kernel<MODE, BEAM, CH, PS>), dim3(groups), dim3(WAVE * waves), lds, s, a);
    return hipGetLastError();
}

template <int MODE, int BEAM, bool PS>
static hipError_t launch_tile_c(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    if (a.algo == ALGO_TILE_MX) {
        switch (a.chunk) {
            case 64: return launch_tile_mx_t<MODE, BEAM, 64, PS>(a, waves, groups, s);
            case 256: return launch_tile_mx_t<MODE, BEAM, 256, PS>(a, waves, groups, s);
            default: return launch_tile_mx_t<MODE, BEAM, 128, PS>(a, waves, groups, s);
        }
    }
    switch (a.chunk) {
        case 64: return launch_tile_t<MODE, BEAM, 64, PS>(a, waves, groups, s);
        case 256: return launch_tile_t<MODE, BEAM, 256, PS>(a, waves, groups, s);
        default: return launch_tile_t<MODE, BEAM, 128, PS>(a, waves, groups, s);
    }
}

template <int MODE>
static hipError_t launch_tile(const ConvArgs &a, int waves, int groups, hipStream_t s) {
    const bool full = a.beam_kind == BEAM_FULL;
    if (MODE != MODE_COUNT && a.per_sample)
        return full ? launch_tile_c<MODE, BEAM_FULL, true>(a, waves, groups, s)
                    : launch_tile_c<MODE, BEAM_SCALAR, true>(a, waves, groups, s);
    return full ? launch_tile_c<MODE, BEAM_FULL, false>(a, waves, groups, s)
                : launch_tile_c<MODE, BEAM_SCALAR, false>(a, waves, groups, s);
}

hipError_t launch_conv(const ConvArgs &a, bool f64, int waves, int groups, hipStream_t s) {
    if (f64) {
        switch (a.out_mode) {
            case MODE_TOD: return launch_pixel<double, MODE_TOD>(a, waves, groups, s);
            case MODE_STOKES: return launch_pixel<double, MODE_STOKES>(a, waves, groups, s);
            default: return launch_pixel<double, MODE_COUNT>(a, waves, groups, s);
        }
    }
    if (a.algo == ALGO_TILE || a.algo == ALGO_TILE_MX) {
        switch (a.out_mode) {
            case MODE_TOD: return launch_tile<MODE_TOD>(a, waves, groups, s);
            case MODE_STOKES: return launch_tile<MODE_STOKES>(a, waves, groups, s);
            default: return launch_tile<MODE_COUNT>(a, waves, groups, s);
        }
    }
    switch (a.out_mode) {
        case MODE_TOD: return launch_pixel<float, MODE_TOD>(a, waves, groups, s);
        case MODE_STOKES: return launch_pixel<float, MODE_STOKES>(a, waves, groups, s);
        default: return launch_pixel<float, MODE_COUNT>(a, waves, groups, s);
    }
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

hipError_t launch_healpix_grid(const HpxGridArgs &a, bool f64, hipStream_t s) {
    const int64_t m = (int64_t)a.n * a.n;
    const int64_t g = (m + 255) / 256;
    if (g == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(healpix_grid_kernel<double>, dim3((unsigned)g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(healpix_grid_kernel<float>, dim3((unsigned)g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_repack_cells(const void *b, int32_t n, void *out, bool f64, bool padded, hipStream_t s) {
    const int bs = 256;
    const int64_t side = padded ? n + 1 : n - 1;
    const int64_t m = side * side;
    const int64_t g = (m + bs - 1) / bs;
    if (g == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(repack_cells_kernel<double>, dim3((unsigned)g), dim3(bs), 0, s, (const double *)b, n,
                           (double4 *)out, padded);
    else
        hipLaunchKernelGGL(repack_cells_kernel<float>, dim3((unsigned)g), dim3(bs), 0, s, (const float *)b, n,
                           (float4 *)out, padded);
    return hipGetLastError();
}

hipError_t launch_classify(const DetDesc *dets, const Tile *groups, int32_t n_groups, double frac, int32_t *flag,
                           hipStream_t s) {
    if (n_groups <= 0) return hipSuccess;
    const int per_block = 4;
    const unsigned blocks = (unsigned)((n_groups + per_block - 1) / per_block);
    hipLaunchKernelGGL(classify_kernel, dim3(blocks), dim3(WAVE * per_block), 0, s, dets, groups, n_groups, frac, flag);
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

// ----------------------------------------------------------------------
// Allocation-free single-detector launches: the plan of one call (control
// block, descriptor, both work queues) lives in the file-scope array below,
// built on the device so that no host round trip is needed.
// ----------------------------------------------------------------------
namespace {

// groups of 64 consecutive samples, classified as the plan builder does and
// appended to the tile-path or pixel-path queue
__global__ void static_plan_kernel(DetDesc D, int32_t n_groups, int32_t tile_path, double frac, unsigned char *base) {
    int32_t *ctrl = reinterpret_cast<int32_t *>(base);
    Tile *tq = reinterpret_cast<Tile *>(base + STATIC_TQ_OFF);
    Tile *pq = reinterpret_cast<Tile *>(base + STATIC_PQ_OFF);
    const int lane = threadIdx.x & (WAVE - 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<DetDesc *>(base + STATIC_DESC_OFF) = D;
    const int32_t g = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    if (g >= n_groups) return;   // uniform per wave
    Tile t;
    t.det = 0;
    t.begin = (int64_t)g * WAVE;
    t.count = (int32_t)min((int64_t)WAVE, D.n_samples - t.begin);
    const bool coherent = tile_path && tile_is_coherent(D, t.begin, t.count, lane, frac);
    if (lane == 0) {
        if (coherent) tq[atomicAdd(&ctrl[8], 1)] = t;
        else pq[atomicAdd(&ctrl[24], 1)] = t;
    }
}

__global__ void static_zero_kernel(int32_t *ctrl) {
    if (threadIdx.x < 32) ctrl[threadIdx.x] = 0;
}

}  // namespace

}  // namespace pisco

static_assert(sizeof(pisco::DetDesc) <= pisco::STATIC_TQ_OFF - pisco::STATIC_DESC_OFF,
              "the descriptor must fit between the control block and the queues");

// The plan of allocation-free launches: one copy per GPU for the life of the
// process.  Host code uses its address from hipGetSymbolAddress, never the name.
static __device__ __align__(256) unsigned char scratch[pisco::STATIC_SCRATCH_BYTES];

namespace pisco {

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
void *g_static_ptr[STATIC_MAX_DEVICES] = {};
std::mutex g_static_mu;
}  // namespace

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[device] = p;
    return hipSuccess;
}

void *static_scratch(int device) {
    if (device < 0 || device >= STATIC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_static_mu);
    return g_static_ptr[device];
}

hipError_t launch_static(ConvArgs tile, ConvArgs pix, const DetDesc &D, bool tile_path, bool f64, int waves,
                         int groups, void *base, hipStream_t s) {
    unsigned char *b = static_cast<unsigned char *>(base);
    int32_t *ctrl = reinterpret_cast<int32_t *>(b);
    const int64_t ng = (D.n_samples + WAVE - 1) / WAVE;
    if (ng > STATIC_MAX_GROUPS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(static_zero_kernel, dim3(1), dim3(64), 0, s, ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per_block = 4;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, (ng + per_block - 1) / per_block);
    hipLaunchKernelGGL(static_plan_kernel, dim3(blocks), dim3(WAVE * per_block), 0, s, D, (int32_t)ng,
                       (int32_t)tile_path, tile.coherence, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const DetDesc *dd = reinterpret_cast<const DetDesc *>(b + STATIC_DESC_OFF);
    for (ConvArgs *a : {&tile, &pix}) {
        a->dets = dd;
        a->n_queues = 1;
        a->tiles_per_queue = (int32_t)STATIC_MAX_GROUPS;
    }
    tile.tiles = reinterpret_cast<const Tile *>(b + STATIC_TQ_OFF);
    tile.counters = ctrl;
    tile.queue_len = ctrl + 8;
    pix.tiles = reinterpret_cast<const Tile *>(b + STATIC_PQ_OFF);
    pix.counters = ctrl + 16;
    pix.queue_len = ctrl + 24;
    if (tile_path) {
        e = launch_conv(tile, f64, waves, groups, s);
        if (e != hipSuccess) return e;
    }
    return launch_conv(pix, f64, waves, groups, s);
}

}  // namespace pisco
