// Spherical-harmonic analysis of HEALPix I, Q, U maps and their angular power
// spectra, in FP64: the spectrum estimator the paper applies to maps made from
// the TOD (Sec. 6.2).  Definitions (orthonormal Y_lm with the Condon-Shortley
// phase; spin-2 harmonics of Goldberg et al. 1967; E and B as in Zaldarriaga &
// Seljak 1997 with the HEALPix sign convention) are stated in include/pisco.h.
//
// Three kernels:
//   ring_fourier_kernel  one workgroup per ring: F_r(m) = w sum_j x_j e^{-i m phi_j}
//                        for every field, by an FFT in LDS (direct DFT over the
//                        odd factor of the ring length, then radix-2 Stockham
//                        passes over its power-of-two factor), read at m mod n;
//   alm_kernel           one workgroup per m: lanes own north/south ring pairs,
//                        run the recurrence for lambda_lm in l (mantissa plus a
//                        carried power-of-two exponent, so sin^m theta cannot
//                        underflow), form W_lm and X_lm from lambda_l and
//                        lambda_{l-1}, and accumulate the symmetric and
//                        antisymmetric ring-pair sums; every four l the
//                        workgroup sums its lanes through LDS;
//   alm2cl_kernel        one wave per l: C_l of up to six a_lm pairs;
//   alm2ring_kernel      the synthesis: one workgroup per m, lanes own ring pairs
//                        and sum over l in registers (no cross-lane sums);
//   ring_synth_kernel    one workgroup per ring: the m sums folded onto the ring
//                        length, then the same LDS FFT as the analysis.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sht_internal.h"

namespace pisco {
namespace {

constexpr int SCALE = 256;               // exponent step of the carried recurrence
constexpr int ALM_THREADS = 512;
constexpr int ALM_WAVES = ALM_THREADS / 64;
static_assert(ALM_WAVES == SHT_WAVES, "partial-sum layout");
constexpr int LBLOCK = 4;                // l values per LDS reduction
constexpr int NCOMP = 6;                 // a^T, a^E, a^B (re, im)
constexpr int LCHUNK = 64;               // l values per coefficient table

struct RingGeom {
    int64_t first;
    int n;
    double z, s, phi0_over_pi;
};

// Ring i = r + 1 of the RING scheme (Gorski et al. 2005, Sec. 4): colatitude
// from exact integer ratios, first pixel and its longitude / pi.
__device__ inline RingGeom sht_ring(int N, int r) {
    const int i = r + 1;
    RingGeom g;
    const double n3 = 3.0 * (double)N * (double)N;
    if (i < N || i > 3 * N) {
        const int k = i < N ? i : 4 * N - i;
        const double t = (double)k * (double)k / n3;      // 1 - |z|
        g.n = 4 * k;
        g.first = i < N ? 2LL * k * (k - 1) : 12LL * N * N - 2LL * k * (k + 1);
        g.z = i < N ? 1.0 - t : t - 1.0;
        g.s = sqrt(t * (2.0 - t));
        g.phi0_over_pi = 0.25 / (double)k;
    } else {
        g.n = 4 * N;
        g.first = 2LL * N * (N - 1) + (int64_t)(i - N) * 4 * N;
        g.z = (double)(4 * N - 2 * i) / (3.0 * N);
        g.s = sqrt((double)(2 * i - N) * (double)(7 * N - 2 * i)) / (3.0 * N);
        g.phi0_over_pi = ((i - N) & 1) == 0 ? 0.25 / (double)N : 0.0;
    }
    return g;
}

// Rings [r0, r1) and [r2, r3): one launch per ring-length class, so that the
// LDS each workgroup reserves matches the longest ring of its class.
struct RingRange {
    int r0, r1, r2, r3;
};

__global__ void __launch_bounds__(256) ring_fourier_kernel(ShtArgs a, RingRange rr) {
    extern __shared__ double2 sh_ring[];
    const int b = blockIdx.x;
    const int r = b < rr.r1 - rr.r0 ? rr.r0 + b : rr.r2 + (b - (rr.r1 - rr.r0));
    const RingGeom g = sht_ring(a.nside, r);
    const int n = g.n;
    const int P = n & -n;                // power-of-two factor
    const int q = n / P;                 // odd factor
    double2 *bufA = sh_ring;
    double2 *bufB = sh_ring + n;
    double2 *tab = sh_ring + 2 * n;          // e^{-2 pi i t / q}, t < q (q <= n / 4 when q > 1)
    double *xs = reinterpret_cast<double *>(bufB);
    const double w = 4.0 * M_PI / (12.0 * (double)a.nside * (double)a.nside);
    if (q > 1) {
        for (int t = threadIdx.x; t < q; t += blockDim.x) {
            double st, ct;
            sincospi(2.0 * (double)t / (double)q, &st, &ct);
            tab[t] = make_double2(ct, -st);
        }
    }
    for (int f = 0; f < a.nfields; ++f) {
        const double *x = a.map[f] + g.first;
        for (int j = threadIdx.x; j < n; j += blockDim.x) xs[j] = x[j];
        __syncthreads();
        // P DFTs of length q over the stride-P subsequences x[P j2 + j1]; the input is
        // real, so Y[q - k2] = conj Y[k2] and only k2 <= (q - 1) / 2 is summed
        const int h = (q + 1) / 2;
        for (int it = threadIdx.x; it < P * h; it += blockDim.x) {
            const int j1 = it / h, k2 = it - j1 * h;
            double re = 0.0, im = 0.0;
            if (q == 1) {
                re = xs[j1];
            } else {
                // twiddles e^{-2 pi i j2 k2 / q} from the ring's table (index j2 k2 mod q),
                // four interleaved accumulators (j2 = c mod 4)
                double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
                int idx = 0;
                int j2 = 0;
                for (; j2 + 3 < q; j2 += 4) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double2 tw = tab[idx];
                        const double xv = xs[P * (j2 + c) + j1];
                        ar[c] = fma(xv, tw.x, ar[c]);
                        ai[c] = fma(xv, tw.y, ai[c]);
                        idx += k2;
                        idx = idx >= q ? idx - q : idx;
                    }
                }
                for (; j2 < q; ++j2) {
                    const double2 tw = tab[idx];
                    const double xv = xs[P * j2 + j1];
                    ar[0] = fma(xv, tw.x, ar[0]);
                    ai[0] = fma(xv, tw.y, ai[0]);
                    idx += k2;
                    idx = idx >= q ? idx - q : idx;
                }
                re = (ar[0] + ar[1]) + (ar[2] + ar[3]);
                im = (ai[0] + ai[1]) + (ai[2] + ai[3]);
            }
            bufA[j1 * q + k2] = make_double2(re, im);
            if (k2 > 0) bufA[j1 * q + q - k2] = make_double2(re, -im);
        }
        __syncthreads();
        // radix-2 passes: sequences c and c + Ps/2 (offsets of stride Ps) merge into
        // sequence c of stride Ps/2 and twice the length
        double2 *src = bufA, *dst = bufB;
        int L = q;
        for (int Ps = P; Ps > 1; Ps >>= 1) {
            const int half = Ps >> 1;
            for (int it = threadIdx.x; it < half * L; it += blockDim.x) {
                const int c = it / L, k = it - c * L;
                const double2 E = src[c * L + k];
                const double2 O = src[(c + half) * L + k];
                double sn, cs;
                sincospi((double)k / (double)L, &sn, &cs);          // e^{-i pi k / L}
                const double tr = fma(O.x, cs, O.y * sn);
                const double ti = fma(O.y, cs, -O.x * sn);
                dst[c * 2 * L + k] = make_double2(E.x + tr, E.y + ti);
                dst[c * 2 * L + k + L] = make_double2(E.x - tr, E.y - ti);
            }
            __syncthreads();
            double2 *t = src;
            src = dst;
            dst = t;
            L <<= 1;
        }
        double2 *out = a.F + (size_t)f * (a.mmax + 1) * a.nrings + r;
        for (int m = threadIdx.x; m <= a.mmax; m += blockDim.x) {
            const double2 X = src[m % n];
            double sn, cs;
            sincospi((double)m * g.phi0_over_pi, &sn, &cs);        // e^{-i m phi0}
            out[(size_t)m * a.nrings] = make_double2(w * fma(X.x, cs, X.y * sn), w * fma(X.y, cs, -X.x * sn));
        }
        __syncthreads();
    }
}

struct Coef {
    double ra, rb;           // lambda_l = ra (z lambda_{l-1} - rb lambda_{l-2})
    double A, B, C, D;       // n_l (l - m^2), n_l l (l - 1) / 2, n_l (l + m) c_lm, n_l (l - 1)
};

__device__ inline Coef make_coef(int l, int m) {
    Coef c{};
    const double dl = l, dm = m;
    if (l == m + 1) c.ra = sqrt(2.0 * dm + 3.0);
    if (l >= m + 2) {
        c.ra = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
        c.rb = sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
    }
    if (l >= 2) {
        const double nl = 2.0 / sqrt((dl - 1.0) * dl * (dl + 1.0) * (dl + 2.0));
        const double clm = l > m ? sqrt((2.0 * dl + 1.0) * (dl - dm) / ((2.0 * dl - 1.0) * (dl + dm))) : 0.0;
        c.A = nl * (dl - dm * dm);
        c.B = nl * dl * (dl - 1.0) * 0.5;
        c.C = nl * (dl + dm) * clm;
        c.D = nl * (dl - 1.0);
    }
    return c;
}

struct PairState {
    double2 Tp, Tm, Qp, Qm, Up, Um;   // F_north +- F_south
    double z, inv_s2, z_s2, m_s2;
    double v, vp;                      // lambda_l, lambda_{l-1} in units of 2^(SCALE e)
    int e;
};

// lambda_mm = (-1)^m c_m s^m, split into a mantissa and a multiple of SCALE in the exponent
__device__ inline void start_value(double s, int m, double cm, double *v, int *e) {
    int es;
    const double fs = frexp(s, &es);
    double base = fs, res = 1.0;
    long long be = 0, re = 0;
    for (int k = m; k; k >>= 1) {
        int t;
        if (k & 1) {
            res = frexp(res * base, &t);
            re += be + t;
        }
        base = frexp(base * base, &t);
        be = 2 * be + t;
    }
    const long long E = re + (long long)es * m;
    long long q = E / SCALE;
    if (q * SCALE > E) --q;                       // floor
    *e = (int)q;
    *v = ((m & 1) ? -cm : cm) * ldexp(res, (int)(E - q * SCALE));
}

// Adds lambda_l F_T, W F_Q + i X F_U and W F_U - i X F_Q (the last two are
// -a^E and -a^B; the sign is applied when the sums are stored).  SCALED: the
// lane's values may still carry a power-of-two exponent (e < 0).
template <int P, bool POL, bool SCALED>
__device__ inline void pair_terms(const PairState &p, const Coef &c, double *acc) {
    double L = p.v, Lp = p.vp;
    if (SCALED) {
        const double f = p.e == 0 ? 1.0 : (p.e == -1 ? 0x1p-256 : 0.0);
        L *= f;
        Lp *= f;
    }
    const double2 FT = P ? p.Tm : p.Tp;
    acc[0] = fma(L, FT.x, acc[0]);
    acc[1] = fma(L, FT.y, acc[1]);
    if (POL) {
        // W = -(A / s^2 + B) lambda_l + C (z / s^2) lambda_{l-1};  X = (m / s^2)(C lambda_{l-1} - D z lambda_l)
        const double W = fma(-fma(c.A, p.inv_s2, c.B), L, c.C * p.z_s2 * Lp);
        const double X = p.m_s2 * fma(c.C, Lp, -c.D * p.z * L);
        const double2 Qa = P ? p.Qm : p.Qp, Ua = P ? p.Um : p.Up;    // parity of lambda and W
        const double2 Qb = P ? p.Qp : p.Qm, Ub = P ? p.Up : p.Um;    // parity of X
        acc[2] = fma(-X, Ub.y, fma(W, Qa.x, acc[2]));
        acc[3] = fma(X, Ub.x, fma(W, Qa.y, acc[3]));
        acc[4] = fma(X, Qb.y, fma(W, Ua.x, acc[4]));
        acc[5] = fma(-X, Qb.x, fma(W, Ua.y, acc[5]));
    }
}

template <bool SCALED>
__device__ inline void advance(PairState &p, const Coef &c) {
    const double vn = c.ra * fma(p.z, p.v, -c.rb * p.vp);
    p.vp = p.v;
    p.v = vn;
    if (SCALED && fabs(vn) > 0x1p256) {
        p.v *= 0x1p-256;
        p.vp *= 0x1p-256;
        p.e += 1;
    }
}

// Orders this wave's LDS writes before its later LDS reads (lanes exchange
// values inside one wave; no other wave touches the region).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int RED_STRIDE = LBLOCK * NCOMP + 1;   // padded row of one lane's sums (doubles)

template <bool POL>
__global__ void __launch_bounds__(ALM_THREADS) alm_kernel(ShtArgs a) {
    extern __shared__ double sh_alm[];
    const int m = blockIdx.x;
    const int N = a.nside, lmax = a.lmax;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // per-wave regions: [64][RED_STRIDE] lane sums, then LCHUNK coefficient records
    double *red = sh_alm + wave * (64 * RED_STRIDE + LCHUNK * (int)(sizeof(Coef) / sizeof(double)));
    Coef *coef = reinterpret_cast<Coef *>(red + 64 * RED_STRIDE);
    const int npairs = 2 * N;
    const int kcount = (npairs + ALM_THREADS - 1) / ALM_THREADS;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 2) / 2;

    // c_m = sqrt((4 pi)^-1 prod_{k=1..m} (2k + 1) / (2k)): partial products per lane, then across the wave
    double pr = 1.0;
    for (int k = lane + 1; k <= m; k += 64) pr *= (2.0 * k + 1.0) / (2.0 * k);
    for (int o = 32; o; o >>= 1) pr *= __shfl_xor(pr, o, 64);
    const double cm = sqrt(pr / (4.0 * M_PI));

    PairState ps[SHT_PAIRS_PER_LANE];
#pragma unroll
    for (int k = 0; k < SHT_PAIRS_PER_LANE; ++k) {
        PairState &p = ps[k];
        const int pi = tid + k * ALM_THREADS;
        const bool ok = k < kcount && pi < npairs;
        const int rn = ok ? pi : 0;
        const int rs = a.nrings - 1 - rn;                            // mirror ring; rs == rn on the equator
        const RingGeom g = sht_ring(N, rn);
        double2 fn[3] = {}, fs[3] = {};
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (ok && f < a.nfields) {
                const double2 *F = a.F + ((size_t)f * (a.mmax + 1) + m) * a.nrings;
                fn[f] = F[rn];
                if (rs != rn) fs[f] = F[rs];
            }
        }
        p.Tp = make_double2(fn[0].x + fs[0].x, fn[0].y + fs[0].y);
        p.Tm = make_double2(fn[0].x - fs[0].x, fn[0].y - fs[0].y);
        p.Qp = make_double2(fn[1].x + fs[1].x, fn[1].y + fs[1].y);
        p.Qm = make_double2(fn[1].x - fs[1].x, fn[1].y - fs[1].y);
        p.Up = make_double2(fn[2].x + fs[2].x, fn[2].y + fs[2].y);
        p.Um = make_double2(fn[2].x - fs[2].x, fn[2].y - fs[2].y);
        p.z = g.z;
        p.inv_s2 = 1.0 / (g.s * g.s);
        p.z_s2 = g.z * p.inv_s2;
        p.m_s2 = (double)m * p.inv_s2;
        start_value(g.s, m, cm, &p.v, &p.e);
        p.vp = 0.0;
        if (!ok) p.e = -1000000;                                     // never contributes
    }

    const int nl = lmax - m + 1;
    for (int c0 = 0; c0 < nl; c0 += LCHUNK) {
        if (c0 + lane < nl) coef[lane] = make_coef(m + c0 + lane, m);
        wave_sync();
        const int cend = min(nl, c0 + LCHUNK);
        for (int b0 = c0; b0 < cend; b0 += LBLOCK) {
            double acc[LBLOCK][NCOMP];
#pragma unroll
            for (int j = 0; j < LBLOCK; ++j) {
#pragma unroll
                for (int t = 0; t < NCOMP; ++t) acc[j][t] = 0.0;
                const int li = b0 + j;                               // l - m; even = same parity as m
                if (li < cend) {
                    const Coef c = coef[li - c0];
#pragma unroll
                    for (int k = 0; k < SHT_PAIRS_PER_LANE; ++k) {
                        if (k >= kcount) continue;
                        // once no lane of this band carries an exponent, its values stay
                        // O(1) and the checks and scale factors drop out (wave-uniform)
                        if (__ballot(ps[k].e != 0) == 0) {
                            if (li > 0) advance<false>(ps[k], c);
                            if (j & 1)
                                pair_terms<1, POL, false>(ps[k], c, acc[j]);
                            else
                                pair_terms<0, POL, false>(ps[k], c, acc[j]);
                        } else {
                            if (li > 0) advance<true>(ps[k], c);
                            if (__ballot(ps[k].e >= -1) == 0) continue;   // whole band below 2^-256
                            if (j & 1)
                                pair_terms<1, POL, true>(ps[k], c, acc[j]);
                            else
                                pair_terms<0, POL, true>(ps[k], c, acc[j]);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < LBLOCK; ++j)
#pragma unroll
                for (int t = 0; t < NCOMP; ++t) red[lane * RED_STRIDE + j * NCOMP + t] = acc[j][t];
            wave_sync();
            // lanes 0..47: sum o = lane / 2 over the half of the wave's lanes given by lane & 1
            double sum = 0.0;
            const int o = lane >> 1, half = lane & 1;
            if (lane < 2 * LBLOCK * NCOMP) {
                // four partial sums: short dependency chains (fixed order)
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 32; u += 4)
#pragma unroll
                    for (int c = 0; c < 4; ++c) s4[c] += red[(half * 32 + u + c) * RED_STRIDE + o];
                sum = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            }
            sum += __shfl_xor(sum, 1, 64);
            const int j = o / NCOMP, t = o - j * NCOMP;
            if (lane < 2 * LBLOCK * NCOMP && half == 0 && b0 + j < cend) {
                const int64_t idx = (int64_t)m * (2 * lmax + 1 - m) / 2 + m + b0 + j;
                a.partial[((int64_t)wave * nalm + idx) * NCOMP + t] = sum;
            }
            wave_sync();
        }
    }
}

// a_lm = sum of the waves' partial sums; E and B take the sign of their definitions.
__global__ void __launch_bounds__(256) alm_reduce_kernel(ShtArgs a) {
    const int64_t nalm = (int64_t)(a.lmax + 1) * (a.lmax + 2) / 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nalm * NCOMP) return;
    const int t = (int)(i % NCOMP);
    double *dst = a.alm[t >> 1];
    if (!dst) return;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < ALM_WAVES; ++w) s += a.partial[(int64_t)w * nalm * NCOMP + i];
    dst[2 * (i / NCOMP) + (t & 1)] = t < 2 ? s : -s;
}

struct SynPair {
    double z, inv_s2, z_s2, m_s2;
    double v, vp;
    int e;
    double2 acc[3][2];                 // [field][class]: north-ring sums split by their south sign
};

// Adds one l to the pair's sums: lambda and W terms go to class P = (l + m) & 1
// (south value (-1)^(l+m) times the north one), X terms to class 1 - P.
template <int P, bool POL, bool SCALED>
__device__ inline void syn_terms(SynPair &p, const Coef &c, const double *al) {
    double L = p.v, Lp = p.vp;
    if (SCALED) {
        const double f = p.e == 0 ? 1.0 : (p.e == -1 ? 0x1p-256 : 0.0);
        L *= f;
        Lp *= f;
    }
    const double2 aT = make_double2(al[0], al[1]);
    p.acc[0][P].x = fma(L, aT.x, p.acc[0][P].x);
    p.acc[0][P].y = fma(L, aT.y, p.acc[0][P].y);
    if (POL) {
        const double2 aE = make_double2(al[2], al[3]), aB = make_double2(al[4], al[5]);
        const double W = fma(-fma(c.A, p.inv_s2, c.B), L, c.C * p.z_s2 * Lp);
        const double X = p.m_s2 * fma(c.C, Lp, -c.D * p.z * L);
        // Q: -(aE W + i aB X);  U: -(aB W - i aE X)
        p.acc[1][P].x = fma(-W, aE.x, p.acc[1][P].x);
        p.acc[1][P].y = fma(-W, aE.y, p.acc[1][P].y);
        p.acc[1][1 - P].x = fma(X, aB.y, p.acc[1][1 - P].x);
        p.acc[1][1 - P].y = fma(-X, aB.x, p.acc[1][1 - P].y);
        p.acc[2][P].x = fma(-W, aB.x, p.acc[2][P].x);
        p.acc[2][P].y = fma(-W, aB.y, p.acc[2][P].y);
        p.acc[2][1 - P].x = fma(-X, aE.y, p.acc[2][1 - P].x);
        p.acc[2][1 - P].y = fma(X, aE.x, p.acc[2][1 - P].y);
    }
}

template <bool SCALED>
__device__ inline void syn_advance(SynPair &p, const Coef &c) {
    const double vn = c.ra * fma(p.z, p.v, -c.rb * p.vp);
    p.vp = p.v;
    p.v = vn;
    if (SCALED && fabs(vn) > 0x1p256) {
        p.v *= 0x1p-256;
        p.vp *= 0x1p-256;
        p.e += 1;
    }
}

// Synthesis workgroups: 12 waves of up to three ring pairs per lane (2304 >= 2N
// at the largest nside), three waves per SIMD.
constexpr int SYN_THREADS = 768;
constexpr int SYN_PAIRS = 3;
static_assert(SYN_THREADS * SYN_PAIRS >= 2 * SHT_MAX_NSIDE, "ring pairs per workgroup");

template <bool POL>
__global__ void __launch_bounds__(SYN_THREADS) alm2ring_kernel(ShtArgs a) {
    extern __shared__ double sh_syn[];
    const int m = blockIdx.x;
    const int N = a.nside, lmax = a.lmax;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int CW = (int)(sizeof(Coef) / sizeof(double));
    double *al = sh_syn + wave * LCHUNK * (CW + NCOMP);             // per wave: [LCHUNK][6] a_lm values
    Coef *coef = reinterpret_cast<Coef *>(al + LCHUNK * NCOMP);     // then [LCHUNK] coefficient records
    const int npairs = 2 * N;
    const int kcount = (npairs + SYN_THREADS - 1) / SYN_THREADS;

    double pr = 1.0;
    for (int k = lane + 1; k <= m; k += 64) pr *= (2.0 * k + 1.0) / (2.0 * k);
    for (int o = 32; o; o >>= 1) pr *= __shfl_xor(pr, o, 64);
    const double cm = sqrt(pr / (4.0 * M_PI));

    SynPair ps[SYN_PAIRS];
#pragma unroll
    for (int k = 0; k < SYN_PAIRS; ++k) {
        SynPair &p = ps[k];
        const int pi = tid + k * SYN_THREADS;
        const bool ok = k < kcount && pi < npairs;
        const RingGeom g = sht_ring(N, ok ? pi : 0);
        p.z = g.z;
        p.inv_s2 = 1.0 / (g.s * g.s);
        p.z_s2 = g.z * p.inv_s2;
        p.m_s2 = (double)m * p.inv_s2;
        start_value(g.s, m, cm, &p.v, &p.e);
        p.vp = 0.0;
        if (!ok) p.e = -1000000;
#pragma unroll
        for (int f = 0; f < 3; ++f) p.acc[f][0] = p.acc[f][1] = make_double2(0.0, 0.0);
    }

    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;        // index of (l = 0, m) minus 0: + l
    const int nl = lmax - m + 1;
    for (int c0 = 0; c0 < nl; c0 += LCHUNK) {
        if (c0 + lane < nl) {
            const int l = m + c0 + lane;
            coef[lane] = make_coef(l, m);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double *src = a.alm_in[f];
                const bool use = src && (f == 0 || POL);
                al[lane * NCOMP + 2 * f] = use ? src[2 * (base + l)] : 0.0;
                al[lane * NCOMP + 2 * f + 1] = use ? src[2 * (base + l) + 1] : 0.0;
            }
        }
        wave_sync();
        const int cend = min(nl, c0 + LCHUNK);
        for (int b0 = c0; b0 < cend; b0 += 2) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int li = b0 + j;                                // l - m; even = class 0
                if (li >= cend) break;
                const Coef c = coef[li - c0];
                const double *A = al + (li - c0) * NCOMP;
#pragma unroll
                for (int k = 0; k < SYN_PAIRS; ++k) {
                    if (k >= kcount) continue;
                    if (__ballot(ps[k].e != 0) == 0) {
                        if (li > 0) syn_advance<false>(ps[k], c);
                        if (j)
                            syn_terms<1, POL, false>(ps[k], c, A);
                        else
                            syn_terms<0, POL, false>(ps[k], c, A);
                    } else {
                        if (li > 0) syn_advance<true>(ps[k], c);
                        if (__ballot(ps[k].e >= -1) == 0) continue;
                        if (j)
                            syn_terms<1, POL, true>(ps[k], c, A);
                        else
                            syn_terms<0, POL, true>(ps[k], c, A);
                    }
                }
            }
        }
        wave_sync();
    }
#pragma unroll
    for (int k = 0; k < SYN_PAIRS; ++k) {
        const int pi = tid + k * SYN_THREADS;
        if (k >= kcount || pi >= npairs) continue;
        const int rn = pi, rs = a.nrings - 1 - pi;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (f >= a.nfields) break;
            const double2 s0 = ps[k].acc[f][0], s1 = ps[k].acc[f][1];
            double2 *G = a.F + ((size_t)f * (a.mmax + 1) + m) * a.nrings;
            G[rn] = make_double2(s0.x + s1.x, s0.y + s1.y);
            if (rs != rn) G[rs] = make_double2(s0.x - s1.x, s0.y - s1.y);
        }
    }
}

// x_j = Re sum_{m=0..mmax} c_m G_m e^{i m (phi0 + 2 pi j / n)}, c_0 = 1, c_m = 2:
// the m sums folded onto k = m mod n give H, and x = Re DFT(conj H) = DFT(conj Hs)
// with Hs[k] = (H[k] + conj H[n - k]) / 2 Hermitian.  Then the stride-P
// subsequences of conj Hs pair up: their q-point DFTs obey
// Y_{P-j1}[k] = e^{2 pi i k / q} conj Y_{j1}[k] (1 <= j1 < P), so only
// j1 = 0..P/2 are summed.
__global__ void __launch_bounds__(256) ring_synth_kernel(ShtArgs a, RingRange rr) {
    extern __shared__ double2 sh_ring[];
    const int b = blockIdx.x;
    const int r = b < rr.r1 - rr.r0 ? rr.r0 + b : rr.r2 + (b - (rr.r1 - rr.r0));
    const RingGeom g = sht_ring(a.nside, r);
    const int n = g.n;
    const int P = n & -n;
    const int q = n / P;
    double2 *bufA = sh_ring;
    double2 *bufB = sh_ring + n;
    double2 *tab = sh_ring + 2 * n;
    if (q > 1) {
        for (int t = threadIdx.x; t < q; t += blockDim.x) {
            double st, ct;
            sincospi(2.0 * (double)t / (double)q, &st, &ct);
            tab[t] = make_double2(ct, -st);
        }
    }
    for (int f = 0; f < a.nfields; ++f) {
        const double2 *G = a.F + (size_t)f * (a.mmax + 1) * a.nrings + r;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            double hr = 0.0, hi = 0.0;
            for (int m = k; m <= a.mmax; m += n) {
                const double2 v = G[(size_t)m * a.nrings];
                double sn, cs;
                sincospi((double)m * g.phi0_over_pi, &sn, &cs);       // e^{+i m phi0}
                const double c = m == 0 ? 1.0 : 2.0;
                hr = fma(c, fma(v.x, cs, -v.y * sn), hr);
                hi = fma(c, fma(v.x, sn, v.y * cs), hi);
            }
            bufA[k] = make_double2(hr, hi);
        }
        __syncthreads();
        // bufA <- conj Hs
        for (int k = threadIdx.x; 2 * k <= n; k += blockDim.x) {
            const int k2 = k == 0 ? 0 : n - k;
            const double2 u = bufA[k], v = bufA[k2];
            const double2 hs = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));   // (H[k] + conj H[n-k]) / 2
            bufA[k] = make_double2(hs.x, -hs.y);
            bufA[k2] = hs;                                                        // conj of Hs[n-k] = conj conj Hs[k]
        }
        __syncthreads();
        double2 *src = bufA, *dst = bufB;
        if (q > 1) {
            // complex input: all k2 < q for j1 = 0..P/2 (P >= 4 on every ring with q > 1);
            // four interleaved accumulators (j2 = c mod 4)
            const int jhalf = P >= 4 ? P / 2 : P - 1;
            for (int it = threadIdx.x; it < (jhalf + 1) * q; it += blockDim.x) {
                const int j1 = it / q, k2 = it - j1 * q;
                double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
                int idx = 0;
                int j2 = 0;
                for (; j2 + 3 < q; j2 += 4) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const double2 tw = tab[idx];
                        const double2 xv = bufA[P * (j2 + c) + j1];
                        ar[c] = fma(xv.x, tw.x, fma(-xv.y, tw.y, ar[c]));
                        ai[c] = fma(xv.x, tw.y, fma(xv.y, tw.x, ai[c]));
                        idx += k2;
                        idx = idx >= q ? idx - q : idx;
                    }
                }
                for (; j2 < q; ++j2) {
                    const double2 tw = tab[idx];
                    const double2 xv = bufA[P * j2 + j1];
                    ar[0] = fma(xv.x, tw.x, fma(-xv.y, tw.y, ar[0]));
                    ai[0] = fma(xv.x, tw.y, fma(xv.y, tw.x, ai[0]));
                    idx += k2;
                    idx = idx >= q ? idx - q : idx;
                }
                bufB[j1 * q + k2] = make_double2((ar[0] + ar[1]) + (ar[2] + ar[3]), (ai[0] + ai[1]) + (ai[2] + ai[3]));
            }
            __syncthreads();
            // the rest by the pairing: Y_{j1}[k] = e^{2 pi i k / q} conj Y_{P - j1}[k]
            for (int it = threadIdx.x; it < (P - 1 - jhalf) * q; it += blockDim.x) {
                const int j1 = jhalf + 1 + it / q, k2 = it % q;
                const double2 y = bufB[(P - j1) * q + k2];
                const double2 t = tab[k2];                                          // e^{-2 pi i k / q}
                // conj(t) * conj(y) = conj(t * y)
                bufB[j1 * q + k2] = make_double2(t.x * y.x - t.y * y.y, -(t.x * y.y + t.y * y.x));
            }
            __syncthreads();
            src = bufB;
            dst = bufA;
        }
        int L = q;
        for (int Ps = P; Ps > 1; Ps >>= 1) {
            const int half = Ps >> 1;
            for (int it = threadIdx.x; it < half * L; it += blockDim.x) {
                const int c = it / L, k = it - c * L;
                const double2 E = src[c * L + k];
                const double2 O = src[(c + half) * L + k];
                double sn, cs;
                sincospi((double)k / (double)L, &sn, &cs);
                const double tr = fma(O.x, cs, O.y * sn);
                const double ti = fma(O.y, cs, -O.x * sn);
                dst[c * 2 * L + k] = make_double2(E.x + tr, E.y + ti);
                dst[c * 2 * L + k + L] = make_double2(E.x - tr, E.y - ti);
            }
            __syncthreads();
            double2 *t = src;
            src = dst;
            dst = t;
            L <<= 1;
        }
        double *out = a.map_out[f] + g.first;
        for (int j = threadIdx.x; j < n; j += blockDim.x) out[j] = src[j].x;
        __syncthreads();
    }
}

// y <- x + alpha y (reverse) or y <- y + alpha x
__global__ void __launch_bounds__(256) axpy_kernel(double *y, const double *x, double alpha, int64_t n, bool reverse) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = reverse ? fma(alpha, y[i], x[i]) : fma(alpha, x[i], y[i]);
}

// One wave per l: lanes take m = lane, lane + 64, ...; then a shuffle tree.
__global__ void __launch_bounds__(64) alm2cl_kernel(ClArgs a) {
    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    for (int sp = 0; sp < a.nspec; ++sp) {
        double acc = 0.0;
        for (int m = lane; m <= l; m += 64) {
            const int64_t idx = (int64_t)m * (2 * a.lmax + 1 - m) / 2 + l;
            const double2 x = reinterpret_cast<const double2 *>(a.x[sp])[idx];
            const double2 y = reinterpret_cast<const double2 *>(a.y[sp])[idx];
            const double p = fma(x.x, y.x, x.y * y.y);
            acc += m == 0 ? p : 2.0 * p;
        }
        for (int o = 32; o; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) a.cl[(size_t)sp * (a.lmax + 1) + l] = acc / (2.0 * l + 1.0);
    }
}

}  // namespace

template <bool SYN>
hipError_t launch_rings(const ShtArgs &a, hipStream_t s) {
    const int N = a.nside;
    const void *kern = SYN ? (const void *)ring_synth_kernel : (const void *)ring_fourier_kernel;
    // LDS: two ring buffers and the odd-factor twiddle table (q <= length / 4)
    auto lds_for = [](int nmax) { return (2 * (size_t)nmax + (size_t)nmax / 4 + 1) * sizeof(double2); };
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_for(4 * N));
    if (e != hipSuccess) return e;
    // classes by cap ring index k (ring length 4k): k <= N/4, N/4 < k <= N/2, the rest
    // (longer polar rings and the equatorial belt, length 4N)
    const int c1 = N / 4, c2 = N / 2;
    const int bounds[3] = {c1, c2, N};
    int lo = 0;
    for (int c = 0; c < 3; ++c) {
        const int hi = bounds[c];
        RingRange rr{};
        if (c < 2) {       // north rings k = lo+1..hi and their southern mirrors
            rr = RingRange{lo, hi, a.nrings - hi, a.nrings - lo};
        } else {           // everything between
            rr = RingRange{lo, a.nrings - lo, 0, 0};
        }
        const int nblocks = (rr.r1 - rr.r0) + (rr.r3 - rr.r2);
        const int nmax = c < 2 ? 4 * hi : 4 * N;
        if (nblocks > 0) {
            if (SYN)
                hipLaunchKernelGGL(ring_synth_kernel, dim3(nblocks), dim3(256), lds_for(nmax), s, a, rr);
            else
                hipLaunchKernelGGL(ring_fourier_kernel, dim3(nblocks), dim3(256), lds_for(nmax), s, a, rr);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        lo = hi;
    }
    return hipSuccess;
}

hipError_t launch_ring_fourier(const ShtArgs &a, hipStream_t s) { return launch_rings<false>(a, s); }

hipError_t launch_alm2map(const ShtArgs &a, hipStream_t s) {
    const size_t lds = (size_t)(SYN_THREADS / 64) * LCHUNK * (sizeof(Coef) + NCOMP * sizeof(double));
    const void *k = a.nfields == 3 ? (const void *)alm2ring_kernel<true> : (const void *)alm2ring_kernel<false>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.nfields == 3)
        hipLaunchKernelGGL(alm2ring_kernel<true>, dim3(a.mmax + 1), dim3(SYN_THREADS), lds, s, a);
    else
        hipLaunchKernelGGL(alm2ring_kernel<false>, dim3(a.mmax + 1), dim3(SYN_THREADS), lds, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_rings<true>(a, s);
}

hipError_t launch_axpy(double *y, const double *x, double alpha, int64_t n, bool reverse, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, alpha, n, reverse);
    return hipGetLastError();
}

hipError_t launch_alm(const ShtArgs &a, hipStream_t s) {
    const size_t lds = (size_t)ALM_WAVES * (64 * RED_STRIDE * sizeof(double) + LCHUNK * sizeof(Coef));
    const void *k = a.nfields == 3 ? (const void *)alm_kernel<true> : (const void *)alm_kernel<false>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.nfields == 3)
        hipLaunchKernelGGL(alm_kernel<true>, dim3(a.mmax + 1), dim3(ALM_THREADS), lds, s, a);
    else
        hipLaunchKernelGGL(alm_kernel<false>, dim3(a.mmax + 1), dim3(ALM_THREADS), lds, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)(a.lmax + 1) * (a.lmax + 2) / 2 * NCOMP;
    hipLaunchKernelGGL(alm_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_alm2cl(const ClArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(alm2cl_kernel, dim3(a.lmax + 1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace pisco
