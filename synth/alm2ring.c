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

/*
 * Spin-2 counterpart for the Q and U maps of an (E, B) expansion, in the
 * convention of Zaldarriaga & Seljak (1997) with the HEALPix signs: with the
 * spin-2 harmonics of Goldberg et al. (1967) written _{+-2}Y_lm =
 * (W_lm +- X_lm) e^{i m phi},
 *     Q = -sum_{l,m} (aE_lm W_lm + i aB_lm X_lm) e^{i m phi},
 *     U = -sum_{l,m} (aB_lm W_lm - i aE_lm X_lm) e^{i m phi}.
 * W and X follow from lambda_lm and lambda_{l-1,m} (Kamionkowski, Kosowsky &
 * Stebbins 1997):
 *     W = n_l [-((l - m^2)/s^2 + l(l-1)/2) lambda_l + (l+m) c_lm (z/s^2) lambda_{l-1}]
 *     X = n_l (m/s^2) [-(l-1) z lambda_l + (l+m) c_lm lambda_{l-1}]
 * with n_l = 2 / sqrt((l-1) l (l+1) (l+2)), c_lm = sqrt((2l+1)(l-m)/((2l-1)(l+m))).
 * Under z -> -z, W has the parity (-1)^(l+m) of lambda_lm and X the opposite.
 * Outputs as in synth_ring_coeffs, for Q and U.
 */
void synth_ring_coeffs_spin2(int lmax, const double *e_re, const double *e_im, const double *b_re,
                             const double *b_im, int npair, const double *z, const double *sth,
                             double *QN_re, double *QN_im, double *UN_re, double *UN_im,
                             double *QS_re, double *QS_im, double *US_re, double *US_im) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < npair; ++r) {
        const double x = z[r], s = sth[r];
        const double is2 = 1.0 / (s * s);
        double vmm = 1.0 / sqrt(4.0 * M_PI);
        int emm = 0;
        for (int m = 0; m <= lmax; ++m) {
            if (m > 0) {
                vmm *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
                while (fabs(vmm) < SC_SMALL && vmm != 0.0) { vmm *= SC_BIG; emm -= 1; }
            }
            /* [0] = (l+m) even, [1] = odd; W-terms and X-terms kept apart for the mirror ring */
            double qw_r[2] = {0, 0}, qw_i[2] = {0, 0}, qx_r[2] = {0, 0}, qx_i[2] = {0, 0};
            double uw_r[2] = {0, 0}, uw_i[2] = {0, 0}, ux_r[2] = {0, 0}, ux_i[2] = {0, 0};
            double lam_prev = 0.0, lam = vmm;
            int e = emm;
            for (int l = m; l <= lmax; ++l) {
                if (l == m + 1) {
                    lam_prev = lam;
                    lam = sqrt(2.0 * m + 3.0) * x * lam;
                } else if (l > m + 1) {
                    const double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
                    const double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                    const double nxt = a * (x * lam - b * lam_prev);
                    lam_prev = lam;
                    lam = nxt;
                }
                if (e < 0 && fabs(lam) > SC_BIG) { lam *= SC_SMALL; lam_prev *= SC_SMALL; e += 1; }
                if (l < 2 || e < -1) continue;
                const double f = (e == 0) ? 1.0 : SC_SMALL;
                const double L = lam * f, Lp = lam_prev * f;
                const double c = (l > m) ? sqrt((2.0 * l + 1.0) * (l - m) / ((2.0 * l - 1.0) * (l + m))) : 0.0;
                const double nl = 2.0 / sqrt((l - 1.0) * l * (l + 1.0) * (l + 2.0));
                const double W = nl * (-((l - (double)m * m) * is2 + 0.5 * l * (l - 1.0)) * L + (l + m) * c * x * is2 * Lp);
                const double X = nl * m * is2 * (-(l - 1.0) * x * L + (l + m) * c * Lp);
                const int64_t k = alm_index(lmax, l, m);
                const int par = (l + m) & 1;
                qw_r[par] += e_re[k] * W;  qw_i[par] += e_im[k] * W;     /* aE W    */
                qx_r[par] -= b_im[k] * X;  qx_i[par] += b_re[k] * X;     /* i aB X  */
                uw_r[par] += b_re[k] * W;  uw_i[par] += b_im[k] * W;     /* aB W    */
                ux_r[par] += e_im[k] * X;  ux_i[par] -= e_re[k] * X;     /* -i aE X */
            }
            const int64_t o = (int64_t)r * (lmax + 1) + m;
            /* north: all terms; south: W-terms with (-1)^(l+m), X-terms with -(-1)^(l+m) */
            QN_re[o] = -(qw_r[0] + qw_r[1] + qx_r[0] + qx_r[1]);
            QN_im[o] = -(qw_i[0] + qw_i[1] + qx_i[0] + qx_i[1]);
            UN_re[o] = -(uw_r[0] + uw_r[1] + ux_r[0] + ux_r[1]);
            UN_im[o] = -(uw_i[0] + uw_i[1] + ux_i[0] + ux_i[1]);
            QS_re[o] = -(qw_r[0] - qw_r[1] - qx_r[0] + qx_r[1]);
            QS_im[o] = -(qw_i[0] - qw_i[1] - qx_i[0] + qx_i[1]);
            US_re[o] = -(uw_r[0] - uw_r[1] - ux_r[0] + ux_r[1]);
            US_im[o] = -(uw_i[0] - uw_i[1] - ux_i[0] + ux_i[1]);
        }
    }
}
