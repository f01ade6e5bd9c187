/*
 * Seeded-input generator helper: per-ring Fourier coefficients of a real
 * spherical-harmonic expansion, used only to synthesise sky maps from
 * Gaussian a_lm.  This file holds no part of the convolution method.
 *
 * For iso-latitude rings at cos(theta) = z the map is
 *     T(theta, phi) = sum_m F_m(z) e^{i m phi}  (m = -L..L, F_{-m} = conj F_m)
 * with F_m(z) = sum_{l>=m} a_lm lambda_lm(z), lambda_lm the orthonormal
 * associated Legendre functions (Y_lm = lambda_lm e^{i m phi}).
 *
 * lambda_lm is produced by the standard three-term recurrence in l
 * started from lambda_mm.  At large m and small sin(theta) the starting
 * values underflow double precision, so values are carried as v * 2^(400 e)
 * with an integer scale e <= 0; only e == 0 and e == -1 can contribute.
 *
 * Rings come in mirror pairs (z, -z): lambda_lm(-z) = (-1)^(l+m) lambda_lm(z),
 * so the even and odd (l+m) partial sums give both rings at once.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define SC_BIG 0x1p+400
#define SC_SMALL 0x1p-400

static inline int64_t alm_index(int lmax, int l, int m) {
    /* m-major packing: all l for m = 0, then all l for m = 1, ... */
    return (int64_t)m * (lmax + 1) - (int64_t)m * (m - 1) / 2 + (l - m);
}

/*
 * alm_re/alm_im : packed a_lm for 0 <= m <= l <= lmax (m-major, see alm_index)
 * npair         : number of ring pairs
 * z, sth        : cos(theta) and sin(theta) of the northern ring of each pair
 * FN_*, FS_*    : outputs, [npair][lmax+1] coefficients F_m for north / south
 */
void synth_ring_coeffs(int lmax, const double *alm_re, const double *alm_im,
                       int npair, const double *z, const double *sth,
                       double *FN_re, double *FN_im, double *FS_re, double *FS_im) {
    /* recurrence coefficients depend only on (l, m):
       lambda_lm = x A_lm lambda_{l-1,m} - B_lm lambda_{l-2,m},
       A_lm = sqrt((4l^2-1)/(l^2-m^2)),  B_lm = A_lm / A_{l-1,m} */
    const int64_t nalm = alm_index(lmax, lmax, lmax) + 1;
    double *A = (double *)malloc(sizeof(double) * nalm);
    double *B = (double *)malloc(sizeof(double) * nalm);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int m = 0; m <= lmax; ++m) {
        for (int l = m; l <= lmax; ++l) {
            const int64_t k = alm_index(lmax, l, m);
            A[k] = (l == m) ? 0.0 : sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            B[k] = 0.0;
        }
        for (int l = m + 2; l <= lmax; ++l) {
            const int64_t k = alm_index(lmax, l, m);
            B[k] = A[k] / A[k - 1];
        }
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < npair; ++r) {
        const double x = z[r], s = sth[r];
        double vmm = 1.0 / sqrt(4.0 * M_PI); /* lambda_00 */
        int emm = 0;
        for (int m = 0; m <= lmax; ++m) {
            if (m > 0) {
                vmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
                while (fabs(vmm) < SC_SMALL && vmm != 0.0) { vmm *= SC_BIG; emm -= 1; }
            }
            const int64_t k0 = alm_index(lmax, m, m);
            double er = 0, ei = 0, or_ = 0, oi = 0; /* even / odd (l+m) sums */
            double p2 = 0.0, p1 = vmm;               /* lambda_{l-2}, lambda_{l-1} */
            int e = emm;
            for (int l = m; l <= lmax; ++l) {
                const int64_t k = k0 + (l - m);
                double p;
                if (l == m) p = vmm;
                else if (l == m + 1) p = x * A[k] * p1;
                else p = x * A[k] * p1 - B[k] * p2;
                if (l > m) { p2 = p1; p1 = p; }
                if (e < 0 && fabs(p) > SC_BIG) { p *= SC_SMALL; p1 *= SC_SMALL; p2 *= SC_SMALL; e += 1; }
                if (e >= -1) {
                    const double val = (e == 0) ? p : p * SC_SMALL;
                    if (((l + m) & 1) == 0) { er += alm_re[k] * val; ei += alm_im[k] * val; }
                    else { or_ += alm_re[k] * val; oi += alm_im[k] * val; }
                }
            }
            const int64_t o = (int64_t)r * (lmax + 1) + m;
            FN_re[o] = er + or_; FN_im[o] = ei + oi;
            FS_re[o] = er - or_; FS_im[o] = ei - oi;
        }
    }
    free(A); free(B);
}
