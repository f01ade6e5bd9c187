/*
 * Plain FP64 CPU oracle for pixel-space polarised beam convolution.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library and must never be used to produce
 * a product result.
 *
 * What it computes (Fluxa, Brewer & Dunner, "Pixel space convolution for
 * CMB experiments", Sec. 4.2 "Pixelated case", the discrete sum equation):
 *
 *   d(q0) = N * sum_k  D(chi_k) . Lambda(chi_k) . B_k . Lambda(-chi_k) . S_k
 *
 * over the sky pixels k whose centres lie within rho_max of the boresight
 * (and beyond rho_min when an annulus is asked for), with
 *   - D(chi, eps, s) the detector row vector of Sec. 4.1 (equation M_pol),
 *     evaluated at the pixel's polarisation angle chi,
 *   - Lambda the Stokes rotation matrix of Sec. 4.1 (equation lambda_operator),
 *   - B_k the 4x4 beamsor re-pixelated at the pixel's antenna coordinates by
 *     bilinear interpolation of a tangent-plane grid (u, v) = tan(rho) (cos sigma, sin sigma),
 *   - (rho, sigma, chi) from the spherical trigonometry of Appendix A,
 *   - N = norm_scale (FIXED) or norm_scale / sum_k B_TT(k) (PER_SAMPLE): the
 *     beamsor's 1/Omega~ normalisation (Sec. 3, equation beamsor), taken either
 *     as a given constant or as the discrete sum over the same pixels,
 *   - S_k = (I, Q, U, V) of pixel k (V = 0 when no V map is given).
 * Modulation (Sec. 7 notes that a modulated beamsor model is all PISCO needs
 * for a half-wave plate): with a per-sample plate angle phi_t the beamsor of
 * sample t is B_k . H(phi_t), H(phi) = Lambda(phi) . diag(1, 1, -1, -1) .
 * Lambda(-phi) the Mueller matrix of an ideal half-wave plate whose axis lies
 * at phi from the antenna frame's reference direction, sky side of the beam.
 * Every quantity is double precision; sums use long double accumulators in
 * ascending pixel order.  HEALPix pixel centres follow the closed forms of
 * Gorski et al. 2005 (the paper stores maps in HEALPix, Sec. 5.1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* HEALPix RING scheme, Gorski et al. 2005, pixel-index closed forms   */
/* ------------------------------------------------------------------ */

/* Centre of RING pixel `pix`: cos(theta), sin(theta), phi. */
void orc_pix2zphi(int64_t N, int64_t pix, double *z, double *sth, double *phi) {
    const int64_t npix = 12 * N * N;
    const int64_t ncap = 2 * N * (N - 1);
    const double NN = (double)N;
    if (pix < ncap) {
        /* northern cap: ring i holds 4i pixels starting at 2i(i-1) */
        int64_t i = (int64_t)floor((1.0 + sqrt(1.0 + 2.0 * (double)pix)) / 2.0);
        while (2 * i * (i - 1) > pix) --i;
        while (2 * (i + 1) * i <= pix) ++i;
        const int64_t j = pix - 2 * i * (i - 1) + 1; /* 1..4i */
        const double omz = (double)(i * i) / (3.0 * NN * NN);
        *z = 1.0 - omz;
        *sth = sqrt(omz * (2.0 - omz));
        *phi = M_PI / (2.0 * i) * ((double)j - 0.5);
    } else if (pix < npix - ncap) {
        /* equatorial belt: rings N..3N of 4N pixels */
        const int64_t p = pix - ncap;
        const int64_t i = p / (4 * N) + N;
        const int64_t j = p % (4 * N) + 1;
        /* first pixel at phi = 0 when (i - N) is odd, at pi/(4N) when even */
        const double shift = ((i - N) % 2 == 0) ? 0.5 : 1.0;
        *z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * NN);
        *sth = sqrt((1.0 - *z) * (1.0 + *z));
        *phi = M_PI / (2.0 * NN) * ((double)j - shift);
    } else {
        /* southern cap mirrors the northern one; pixels still run in increasing phi */
        const int64_t ps = npix - pix; /* 1 .. ncap */
        int64_t i = (int64_t)floor((1.0 + sqrt(2.0 * (double)ps - 1.0)) / 2.0);
        while (2 * i * (i - 1) >= ps) --i;
        while (2 * i * (i + 1) < ps) ++i;
        const int64_t j = 4 * i + 1 - (ps - 2 * i * (i - 1)); /* 1..4i */
        const double opz = (double)(i * i) / (3.0 * NN * NN);
        *z = opz - 1.0;
        *sth = sqrt(opz * (2.0 - opz));
        *phi = M_PI / (2.0 * i) * ((double)j - 0.5);
    }
}

void orc_pix2ang(int64_t N, int64_t pix, double *theta, double *phi) {
    double z, s;
    orc_pix2zphi(N, pix, &z, &s, phi);
    *theta = atan2(s, z);
}

/*
 * RING pixel containing the direction (theta, phi), Gorski et al. 2005, Sec. 4:
 * with t = 2 phi / pi in [0, 4), the equatorial belt (|z| <= 2/3) is tiled by
 * the two families of lines N (1/2 + t) -/+ (3/4) N z = integer, whose indices
 * give the ring (counted from z = 2/3) and the position along it; in the polar
 * caps the lines are tp sqrt(3 (1 - |z|)) N and (1 - tp) sqrt(3 (1 - |z|)) N =
 * integer, tp being the position within the quadrant, and their sum gives the
 * ring counted from the pole.
 */
static int64_t ang2pix_one(int64_t N, double theta, double phi) {
    const double z = cos(theta), za = fabs(z);
    double t = fmod(phi * (2.0 / M_PI), 4.0);
    if (t < 0.0) t += 4.0;
    const double NN = (double)N;
    if (za <= 2.0 / 3.0) {
        const double a = NN * (0.5 + t), b = 0.75 * NN * z;
        const int64_t jp = (int64_t)floor(a - b), jm = (int64_t)floor(a + b);
        const int64_t ir = N + 1 + jp - jm;            /* 1 .. 2N+1 from z = 2/3 */
        const int64_t odd_shift = 1 - (ir & 1);
        int64_t ip = (jp + jm - N + odd_shift + 1) / 2;
        if (ip >= 4 * N) ip -= 4 * N;
        return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
    }
    const double tp = t - floor(t);
    const double w = NN * sqrt(3.0 * (1.0 - za));
    const int64_t jp = (int64_t)floor(tp * w), jm = (int64_t)floor((1.0 - tp) * w);
    int64_t ir = jp + jm + 1;                          /* 1 .. N from the pole */
    if (ir > N) ir = N;
    int64_t ip = (int64_t)floor(t * (double)ir);
    if (ip >= 4 * ir) ip -= 4 * ir;
    return z > 0.0 ? 2 * ir * (ir - 1) + ip : 12 * N * N - 2 * ir * (ir + 1) + ip;
}

void orc_ang2pix(int64_t N, int64_t m, const double *theta, const double *phi, int64_t *pix) {
    for (int64_t k = 0; k < m; ++k) pix[k] = ang2pix_one(N, theta[k], phi[k]);
}

/* Ring i (1..4N-1, north to south): colatitude, pixel count, first pixel. */
void orc_ring(int64_t N, int64_t i, double *theta, int64_t *count, int64_t *first) {
    const int64_t npix = 12 * N * N;
    if (i < N) {
        *count = 4 * i;
        *first = 2 * i * (i - 1);
    } else if (i <= 3 * N) {
        *count = 4 * N;
        *first = 2 * N * (N - 1) + (i - N) * 4 * N;
    } else {
        const int64_t is = 4 * N - i;
        *count = 4 * is;
        *first = npix - 2 * is * (is + 1);
    }
    double z, s, phi;
    orc_pix2zphi(N, *first, &z, &s, &phi);
    *theta = atan2(s, z);
}

/*
 * A RING map read at (theta, phi) by bilinear interpolation on the sphere (the
 * re-pixelisation of beamsor maps, Sec. 4.2): on each of the two rings whose
 * colatitudes bracket theta, linear in phi between the two pixels whose
 * centres bracket phi (cyclically); between the rings, linear in theta.  Above
 * the first ring the upper "ring" is the north pole, whose value is the mean
 * of the first ring's four pixels; below the last ring, likewise the south pole.
 */
static double ring_value(int64_t N, const double *map, int64_t ring, double phi) {
    double th;
    int64_t cnt, first;
    orc_ring(N, ring, &th, &cnt, &first);
    double z, s, phi0;
    orc_pix2zphi(N, first, &z, &s, &phi0);
    const double dphi = 2.0 * M_PI / (double)cnt;
    const double x = (phi - phi0) / dphi;
    const double fl = floor(x);
    const double w = x - fl;
    int64_t j0 = (int64_t)fl % cnt;
    if (j0 < 0) j0 += cnt;
    const int64_t j1 = (j0 + 1 == cnt) ? 0 : j0 + 1;
    return (1.0 - w) * map[first + j0] + w * map[first + j1];
}

static double ring_theta(int64_t N, int64_t ring) {
    double th;
    int64_t cnt, first;
    orc_ring(N, ring, &th, &cnt, &first);
    return th;
}

double orc_healpix_interp(int64_t N, const double *map, double theta, double phi) {
    const int64_t nring = 4 * N - 1;
    const double th1 = ring_theta(N, 1), thl = ring_theta(N, nring);
    if (theta < th1) {
        const double pole = 0.25 * (map[0] + map[1] + map[2] + map[3]);
        const double t = theta / th1;
        return (1.0 - t) * pole + t * ring_value(N, map, 1, phi);
    }
    if (theta >= thl) {
        const int64_t np = 12 * N * N;
        const double pole = 0.25 * (map[np - 4] + map[np - 3] + map[np - 2] + map[np - 1]);
        const double t = (M_PI - theta) / (M_PI - thl);
        return (1.0 - t) * pole + t * ring_value(N, map, nring, phi);
    }
    /* the ring i with theta_i <= theta < theta_{i+1}, by bisection */
    int64_t lo = 1, hi = nring;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (ring_theta(N, mid) <= theta) lo = mid;
        else hi = mid;
    }
    const double ta = ring_theta(N, lo), tb = ring_theta(N, lo + 1);
    const double t = (theta - ta) / (tb - ta);
    return (1.0 - t) * ring_value(N, map, lo, phi) + t * ring_value(N, map, lo + 1, phi);
}

/* The n x n gnomonic grid over [-T, T]^2 ([v][u]) sampled from a map whose
 * north pole is the boresight: node (u, v) reads the map at theta = rho =
 * atan(sqrt(u^2 + v^2)), phi = sigma = atan2(v, u). */
void orc_healpix_to_grid(int64_t N, const double *map, double T, int n, double *out) {
    const double h = 2.0 * T / (double)(n - 1);
    for (int iv = 0; iv < n; ++iv)
        for (int iu = 0; iu < n; ++iu) {
            const double u = -T + iu * h, v = -T + iv * h;
            out[(int64_t)iv * n + iu] = orc_healpix_interp(N, map, atan(hypot(u, v)), atan2(v, u));
        }
}

/* ------------------------------------------------------------------ */
/* Appendix A: antenna coordinates and polarisation angle               */
/* ------------------------------------------------------------------ */

/*
 * For boresight (theta0, phi0), position angle psi0, detector angle zeta and
 * a sky direction (theta, phi), given by cos/sin of the colatitudes:
 *   rho   = arccos(cos th cos th0 + sin th sin th0 cos dphi)
 *   alpha = angle with sin ~ sin th sin dphi, cos ~ cos th sin th0 - sin th cos th0 cos dphi
 *   sigma = pi - psi0 - alpha
 *   beta  = angle with sin ~ sin th0 sin dphi, cos ~ cos th0 sin th - sin th0 cos th cos dphi
 *   chi   = beta + zeta - sigma
 * The arctangents of Appendix A are taken as two-argument arctangents of the
 * printed sine and cosine numerators (their common 1/sin(rho) is positive);
 * rho is computed as the angle with that cosine and sine |n0 x n|.
 */
static void appA(double z0, double s0, double phi0, double psi0, double zeta,
                 double z, double s, double phi,
                 double *cosrho, double *rho, double *sigma, double *chi) {
    const double dphi = phi - phi0;
    const double cd = cos(dphi), sd = sin(dphi);
    double c = z * z0 + s * s0 * cd;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *cosrho = c;
    /* rho from its sine and cosine together: the cross product of the two unit
     * vectors, in the frame turned by phi0, has components (s sd z0,
     * z s0 - s z0 cd, s s0 sd).  An arccosine of a cosine near 1 keeps only
     * about half the digits of a small rho; the arctangent keeps them all. */
    const double x1 = s * sd * z0, x2 = z * s0 - s * z0 * cd, x3 = s * s0 * sd;
    *rho = atan2(sqrt(x1 * x1 + x2 * x2 + x3 * x3), c);
    const double alpha = atan2(s * sd, z * s0 - s * z0 * cd);
    *sigma = M_PI - psi0 - alpha;
    const double beta = atan2(s0 * sd, z0 * s - s0 * z * cd);
    *chi = beta + zeta - *sigma;
}

void orc_appA(double theta0, double phi0, double psi0, double zeta, double theta, double phi,
              double *rho, double *sigma, double *chi) {
    double cr;
    appA(cos(theta0), sin(theta0), phi0, psi0, zeta, cos(theta), sin(theta), phi, &cr, rho, sigma, chi);
}

/* ------------------------------------------------------------------ */
/* Bilinear re-pixelation of the beamsor on the tangent grid            */
/* ------------------------------------------------------------------ */

/* Grid nodes at -T + i h, h = 2T/(n-1), row-major [iv][iu], 16 Mueller
 * elements per node ([out][in]).  Returns 0 outside the grid. */
static int interp_beamsor(int n, double T, const double *grid, double u, double v, double M[4][4]) {
    const double h = 2.0 * T / (double)(n - 1);
    const double tu = (u + T) / h, tv = (v + T) / h;
    if (!(tu >= 0.0 && tu <= (double)(n - 1) && tv >= 0.0 && tv <= (double)(n - 1))) return 0;
    int iu = (int)floor(tu), iv = (int)floor(tv);
    if (iu > n - 2) iu = n - 2;
    if (iv > n - 2) iv = n - 2;
    const double fu = tu - iu, fv = tv - iv;
    const double w00 = (1.0 - fu) * (1.0 - fv), w10 = fu * (1.0 - fv);
    const double w01 = (1.0 - fu) * fv, w11 = fu * fv;
    const double *g00 = grid + ((int64_t)iv * n + iu) * 16;
    const double *g10 = g00 + 16;
    const double *g01 = g00 + (int64_t)n * 16;
    const double *g11 = g01 + 16;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const int k = a * 4 + b;
            M[a][b] = w00 * g00[k] + w10 * g10[k] + w01 * g01[k] + w11 * g11[k];
        }
    return 1;
}

/* Ideal half-wave plate at angle phi: Lambda(phi) diag(1, 1, -1, -1) Lambda(-phi), formed as that product */
static void lambda_mat(double x, double L[4][4]);
static void hwp_mat(double phi, double H[4][4]) {
    double Lp[4][4], Lm[4][4], P[4][4];
    lambda_mat(phi, Lp);
    lambda_mat(-phi, Lm);
    const double M0[4] = {1.0, 1.0, -1.0, -1.0};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) P[a][b] = M0[a] * Lm[a][b];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            H[a][b] = 0.0;
            for (int c = 0; c < 4; ++c) H[a][b] += Lp[a][c] * P[c][b];
        }
}

/* Lambda(x) of Sec. 4.1 */
static void lambda_mat(double x, double L[4][4]) {
    memset(L, 0, sizeof(double) * 16);
    const double c = cos(2.0 * x), s = sin(2.0 * x);
    L[0][0] = 1.0;
    L[1][1] = c; L[1][2] = -s;
    L[2][1] = s; L[2][2] = c;
    L[3][3] = 1.0;
}

/* ------------------------------------------------------------------ */
/* The convolution                                                      */
/* ------------------------------------------------------------------ */

enum { ORC_NORM_FIXED = 0, ORC_NORM_PER_SAMPLE = 1 };
enum { ORC_OUT_TOD = 0, ORC_OUT_STOKES = 1 };

/*
 * One sample.  out[0] = TOD (OUT_TOD) or out[0..2] = N sum_k B_TT(k) Lambda(-chi_k) S_k
 * restricted to (T, Q, U) (OUT_STOKES: the Stokes pickup of the scalar beam B_TT).
 */
static void one_sample(int64_t N, const double *I, const double *Q, const double *U, const double *V,
                       int n, double T, const double *grid,
                       double zeta, double eps, double s_resp,
                       double rho_min, double rho_max, int norm_mode, double norm_scale,
                       double theta0, double phi0, double psi0, int has_hwp, double hwp_phi, int out_mode,
                       double *out) {
    double H[4][4];
    if (has_hwp) hwp_mat(hwp_phi, H);
    const double z0 = cos(theta0), s0 = sin(theta0);
    const double cmax = cos(rho_max);
    const double cmin = cos(rho_min);
    long double acc[3] = {0.0L, 0.0L, 0.0L};
    long double norm_sum = 0.0L;
    const int64_t nring = 4 * N - 1;
    for (int64_t r = 1; r <= nring; ++r) {
        double th_r;
        int64_t cnt, first;
        orc_ring(N, r, &th_r, &cnt, &first);
        /* a pixel's distance from the boresight is at least |theta - theta0| */
        if (fabs(th_r - theta0) > rho_max + 1e-9) continue;
        for (int64_t p = first; p < first + cnt; ++p) {
            double z, s, phi, cr, rho, sigma, chi;
            orc_pix2zphi(N, p, &z, &s, &phi);
            /* disc membership on the cosine of the angular distance (law of cosines) */
            const double cpre = z * z0 + s * s0 * cos(phi - phi0);
            if (cpre < cmax) continue;                  /* outside rho_max */
            if (rho_min > 0.0 && !(cpre < cmin)) continue; /* inside rho_min */
            appA(z0, s0, phi0, psi0, zeta, z, s, phi, &cr, &rho, &sigma, &chi);
            const double t = tan(rho);
            const double u = t * cos(sigma), v = t * sin(sigma);
            double M[4][4];
            if (!interp_beamsor(n, T, grid, u, v, M)) continue;
            const double S[4] = {I[p], Q[p], U[p], V ? V[p] : 0.0};
            double Lm[4][4], Lp[4][4];
            lambda_mat(-chi, Lm);
            lambda_mat(chi, Lp);
            double rs[4]; /* Lambda(-chi) S, then H(phi_t) Lambda(-chi) S with a plate */
            for (int a = 0; a < 4; ++a) {
                rs[a] = 0.0;
                for (int b = 0; b < 4; ++b) rs[a] += Lm[a][b] * S[b];
            }
            if (has_hwp) {
                double hs[4];
                for (int a = 0; a < 4; ++a) {
                    hs[a] = 0.0;
                    for (int b = 0; b < 4; ++b) hs[a] += H[a][b] * rs[b];
                }
                for (int a = 0; a < 4; ++a) rs[a] = hs[a];
            }
            norm_sum += M[0][0];
            if (out_mode == ORC_OUT_STOKES) {
                for (int a = 0; a < 3; ++a) acc[a] += (long double)(M[0][0] * rs[a]);
                continue;
            }
            double bs[4]; /* B Lambda(-chi) S */
            for (int a = 0; a < 4; ++a) {
                bs[a] = 0.0;
                for (int b = 0; b < 4; ++b) bs[a] += M[a][b] * rs[b];
            }
            double ls[4]; /* Lambda(chi) B Lambda(-chi) S */
            for (int a = 0; a < 4; ++a) {
                ls[a] = 0.0;
                for (int b = 0; b < 4; ++b) ls[a] += Lp[a][b] * bs[b];
            }
            const double D[4] = {0.5 * s_resp * (1.0 + eps), 0.5 * s_resp * (1.0 - eps) * cos(2.0 * chi),
                                 0.5 * s_resp * (1.0 - eps) * sin(2.0 * chi), 0.0};
            double term = 0.0;
            for (int a = 0; a < 4; ++a) term += D[a] * ls[a];
            acc[0] += (long double)term;
        }
    }
    double Nrm = norm_scale;
    if (norm_mode == ORC_NORM_PER_SAMPLE) Nrm = (norm_sum != 0.0L) ? (double)((long double)norm_scale / norm_sum) : 0.0;
    if (out_mode == ORC_OUT_STOKES) {
        for (int a = 0; a < 3; ++a) out[a] = (double)acc[a] * Nrm;
    } else {
        out[0] = (double)acc[0] * Nrm;
    }
}

/*
 * Convolve one detector's pointing stream.
 *   I, Q, U      : RING maps of 12 nside^2 doubles
 *   n, T, grid   : n x n beamsor nodes over u, v in [-T, T], 16 doubles per node
 *   out          : nsamp doubles (OUT_TOD) or 3*nsamp (OUT_STOKES, [t][3])
 *   nthreads     : OpenMP threads (0 = runtime default)
 * Returns 0, or -1 on invalid arguments.
 */
int orc_tod_iquv(int64_t nside, const double *I, const double *Q, const double *U, const double *V,
                 int n, double T, const double *grid,
                 double zeta, double eps, double s_resp,
                 double rho_min, double rho_max, int norm_mode, double norm_scale,
                 int64_t nsamp, const double *theta, const double *phi, const double *psi, const double *hwp,
                 int out_mode, double *out, int nthreads);

int orc_tod(int64_t nside, const double *I, const double *Q, const double *U,
            int n, double T, const double *grid,
            double zeta, double eps, double s_resp,
            double rho_min, double rho_max, int norm_mode, double norm_scale,
            int64_t nsamp, const double *theta, const double *phi, const double *psi,
            int out_mode, double *out, int nthreads) {
    return orc_tod_iquv(nside, I, Q, U, NULL, n, T, grid, zeta, eps, s_resp, rho_min, rho_max, norm_mode,
                        norm_scale, nsamp, theta, phi, psi, NULL, out_mode, out, nthreads);
}

/* As orc_tod with an optional V map and an optional per-sample half-wave-plate
 * angle stream (NULL: none). */
int orc_tod_iquv(int64_t nside, const double *I, const double *Q, const double *U, const double *V,
                 int n, double T, const double *grid,
                 double zeta, double eps, double s_resp,
                 double rho_min, double rho_max, int norm_mode, double norm_scale,
                 int64_t nsamp, const double *theta, const double *phi, const double *psi, const double *hwp,
                 int out_mode, double *out, int nthreads) {
    if (nside < 1 || n < 3 || !(T > 0.0) || !(rho_max > 0.0) || rho_max >= M_PI / 2 || rho_min < 0.0 ||
        rho_min >= rho_max || nsamp < 0)
        return -1;
    const int width = (out_mode == ORC_OUT_STOKES) ? 3 : 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* one sample costs ~1e5-1e7 flops: hand them out one at a time so that
       small calls still spread over every thread */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nsamp; ++t)
        one_sample(nside, I, Q, U, V, n, T, grid, zeta, eps, s_resp, rho_min, rho_max, norm_mode, norm_scale,
                   theta[t], phi[t], psi[t], hwp != NULL, hwp ? hwp[t] : 0.0, out_mode, out + t * width);
    return 0;
}

/* Pixels whose centres lie within rho of (theta0, phi0), ascending; returns the count
 * (writes at most `cap` indices into `pix` when pix != NULL). */
int64_t orc_disc(int64_t N, double theta0, double phi0, double rho, int64_t *pix, int64_t cap) {
    const double z0 = cos(theta0), s0 = sin(theta0), c = cos(rho);
    int64_t k = 0;
    for (int64_t r = 1; r <= 4 * N - 1; ++r) {
        double th_r;
        int64_t cnt, first;
        orc_ring(N, r, &th_r, &cnt, &first);
        if (fabs(th_r - theta0) > rho + 1e-9) continue;
        for (int64_t p = first; p < first + cnt; ++p) {
            double z, s, phi;
            orc_pix2zphi(N, p, &z, &s, &phi);
            const double cr = z * z0 + s * s0 * cos(phi - phi0);
            if (cr >= c) {
                if (pix && k < cap) pix[k] = p;
                ++k;
            }
        }
    }
    return k;
}

/* Disc sizes for many centres at once (OpenMP). */
void orc_disc_counts(int64_t N, int64_t m, const double *theta, const double *phi, double rho, int64_t *counts,
                     int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < m; ++t) counts[t] = orc_disc(N, theta[t], phi[t], rho, NULL, 0);
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
