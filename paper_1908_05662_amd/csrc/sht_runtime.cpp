// C ABI of the harmonic analysis and power spectra (include/pisco.h, "angular
// power spectra" section): argument checks and the launches.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pisco.h"
#include "pisco_internal.h"
#include "sht_internal.h"

namespace {

pisco_status bad(pisco_ctx *c, const char *msg) {
    pisco::set_error(c, msg);
    return PISCO_EINVAL;
}

pisco_status launched(pisco_ctx *c, hipError_t e) {
    if (e == hipSuccess) return PISCO_OK;
    pisco::set_error(c, hipGetErrorString(e));
    return PISCO_EDEVICE;
}

bool nside_ok(int64_t n) { return n >= 1 && n <= pisco::SHT_MAX_NSIDE && (n & (n - 1)) == 0; }
bool lmax_ok(int64_t nside, int64_t lmax) { return lmax >= 0 && lmax <= 4 * nside; }

int64_t fourier_bytes(int64_t nside, int64_t lmax, bool pol) {
    return (pol ? 3 : 1) * (lmax + 1) * (4 * nside - 1) * (int64_t)sizeof(double2);
}

int64_t nalm(int64_t lmax) { return (lmax + 1) * (lmax + 2) / 2; }
int64_t partial_bytes(int64_t lmax) { return (int64_t)pisco::SHT_WAVES * nalm(lmax) * 6 * 8; }
int64_t nfield(bool pol) { return pol ? 3 : 1; }

// ring Fourier sums (or the synthesis' ring coefficients), the a_lm workgroups'
// per-wave partial sums, then for the iterations a residual map and an a_lm
// correction per field
int64_t workspace_bytes(int64_t nside, int64_t lmax, bool pol) {
    return fourier_bytes(nside, lmax, pol) + partial_bytes(lmax) + nfield(pol) * 12 * nside * nside * 8 +
           nfield(pol) * nalm(lmax) * 16;
}

struct Layout {
    double2 *F;
    double *partial, *resid, *dalm;
};

Layout layout(void *ws, int64_t nside, int64_t lmax, bool pol) {
    char *p = static_cast<char *>(ws);
    Layout L;
    L.F = reinterpret_cast<double2 *>(p);
    p += fourier_bytes(nside, lmax, pol);
    L.partial = reinterpret_cast<double *>(p);
    p += partial_bytes(lmax);
    L.resid = reinterpret_cast<double *>(p);
    p += nfield(pol) * 12 * nside * nside * 8;
    L.dalm = reinterpret_cast<double *>(p);
    return L;
}

pisco::ShtArgs base_args(int64_t nside, int32_t lmax, bool pol, const Layout &L) {
    pisco::ShtArgs a{};
    a.nside = (int)nside;
    a.lmax = lmax;
    a.mmax = lmax;
    a.nfields = pol ? 3 : 1;
    a.nrings = (int)(4 * nside - 1);
    a.F = L.F;
    a.partial = L.partial;
    return a;
}

hipError_t analyse(pisco::ShtArgs a, const double *const maps[3], double *const alm[3], hipStream_t st) {
    for (int f = 0; f < 3; ++f) {
        a.map[f] = f < a.nfields ? maps[f] : nullptr;
        a.alm[f] = f < a.nfields ? alm[f] : nullptr;
    }
    hipError_t e = pisco::launch_ring_fourier(a, st);
    return e == hipSuccess ? pisco::launch_alm(a, st) : e;
}

hipError_t synthesise(pisco::ShtArgs a, const double *const alm[3], double *const maps[3], hipStream_t st) {
    for (int f = 0; f < 3; ++f) {
        a.alm_in[f] = f < a.nfields ? alm[f] : nullptr;
        a.map_out[f] = f < a.nfields ? maps[f] : nullptr;
    }
    return pisco::launch_alm2map(a, st);
}

pisco_status check_common(pisco_ctx *ctx, int64_t nside, int32_t lmax, bool pol, void *ws, int64_t ws_bytes) {
    if (!nside_ok(nside)) return bad(ctx, "nside must be a power of two in [1, 1024]");
    if (!lmax_ok(nside, lmax)) return bad(ctx, "lmax must be in [0, 4 nside]");
    if (!ws || ws_bytes < workspace_bytes(nside, lmax, pol)) return bad(ctx, "workspace missing or too small");
    return PISCO_OK;
}

pisco_status map2alm(pisco_ctx *ctx, int64_t nside, int32_t lmax, int32_t iterations, const double *T, const double *Q,
                     const double *U, double *aT, double *aE, double *aB, void *ws, int64_t ws_bytes, hipStream_t st) {
    if (!T || !aT) return bad(ctx, "null T map or a^T");
    if ((Q == nullptr) != (U == nullptr)) return bad(ctx, "Q and U must both be given or both be null");
    const bool pol = Q != nullptr;
    if (pol && (!aE || !aB)) return bad(ctx, "null a^E or a^B");
    if (iterations < 0 || iterations > 16) return bad(ctx, "iterations must be in [0, 16]");
    const pisco_status c = check_common(ctx, nside, lmax, pol, ws, ws_bytes);
    if (c != PISCO_OK) return c;
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    const Layout L = layout(ws, nside, lmax, pol);
    const pisco::ShtArgs a = base_args(nside, lmax, pol, L);
    const int nf = a.nfields;
    const int64_t npix = 12 * nside * nside, na = nalm(lmax);
    const double *maps[3] = {T, Q, U};
    double *alm[3] = {aT, aE, aB};
    double *resid[3] = {L.resid, L.resid + npix, L.resid + 2 * npix};
    double *dalm[3] = {L.dalm, L.dalm + 2 * na, L.dalm + 4 * na};
    hipError_t e = analyse(a, maps, alm, st);
    // Jacobi steps: a <- a + map2alm(m - alm2map(a))
    for (int it = 0; it < iterations && e == hipSuccess; ++it) {
        e = synthesise(a, alm, resid, st);
        for (int f = 0; f < nf && e == hipSuccess; ++f) e = pisco::launch_axpy(resid[f], maps[f], -1.0, npix, true, st);
        const double *rc[3] = {resid[0], resid[1], resid[2]};
        if (e == hipSuccess) e = analyse(a, rc, dalm, st);
        for (int f = 0; f < nf && e == hipSuccess; ++f) e = pisco::launch_axpy(alm[f], dalm[f], 1.0, 2 * na, false, st);
    }
    return launched(ctx, e);
}

}  // namespace

extern "C" {

int64_t pisco_alm_size(int32_t lmax) { return lmax < 0 ? 0 : (int64_t)(lmax + 1) * (lmax + 2) / 2; }

int64_t pisco_map2alm_workspace_bytes(int64_t nside, int32_t lmax, int32_t pol) {
    if (!nside_ok(nside) || !lmax_ok(nside, lmax)) return -1;
    return workspace_bytes(nside, lmax, pol != 0);
}

pisco_status pisco_map2alm(pisco_ctx *ctx, int64_t nside, int32_t lmax, int32_t iterations, const double *T,
                           const double *Q, const double *U, double *alm_T, double *alm_E, double *alm_B,
                           void *workspace, int64_t workspace_bytes, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    return map2alm(ctx, nside, lmax, iterations, T, Q, U, alm_T, alm_E, alm_B, workspace, workspace_bytes,
                   static_cast<hipStream_t>(stream));
}

pisco_status pisco_alm2map(pisco_ctx *ctx, int64_t nside, int32_t lmax, const double *alm_T, const double *alm_E,
                           const double *alm_B, double *T, double *Q, double *U, void *workspace,
                           int64_t workspace_bytes, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (!alm_T || !T) return bad(ctx, "null a^T or T map");
    const bool pol = alm_E != nullptr || alm_B != nullptr || Q != nullptr || U != nullptr;
    if (pol && (!alm_E || !alm_B || !Q || !U)) return bad(ctx, "a^E, a^B, Q and U must all be given or all be null");
    const pisco_status c = check_common(ctx, nside, lmax, pol, workspace, workspace_bytes);
    if (c != PISCO_OK) return c;
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    const Layout L = layout(workspace, nside, lmax, pol);
    const double *alm[3] = {alm_T, alm_E, alm_B};
    double *maps[3] = {T, Q, U};
    return launched(ctx, synthesise(base_args(nside, lmax, pol, L), alm, maps, static_cast<hipStream_t>(stream)));
}

pisco_status pisco_alm2cl(pisco_ctx *ctx, int32_t lmax, const double *alm_x, const double *alm_y, double *cl,
                          void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (lmax < 0 || lmax > 4 * pisco::SHT_MAX_NSIDE) return bad(ctx, "lmax out of range");
    if (!alm_x || !alm_y || !cl) return bad(ctx, "null a_lm or cl");
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    pisco::ClArgs a{};
    a.lmax = lmax;
    a.nspec = 1;
    a.x[0] = alm_x;
    a.y[0] = alm_y;
    a.cl = cl;
    return launched(ctx, pisco::launch_alm2cl(a, static_cast<hipStream_t>(stream)));
}

pisco_status pisco_anafast(pisco_ctx *ctx, int64_t nside, int32_t lmax, int32_t iterations, const double *T,
                           const double *Q, const double *U, double *alm_T, double *alm_E, double *alm_B,
                           void *workspace, int64_t workspace_bytes, double *cl, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (!cl) return bad(ctx, "null cl");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const pisco_status r =
        map2alm(ctx, nside, lmax, iterations, T, Q, U, alm_T, alm_E, alm_B, workspace, workspace_bytes, st);
    if (r != PISCO_OK) return r;
    pisco::ClArgs a{};
    a.lmax = lmax;
    a.cl = cl;
    if (Q) {
        const double *x[6] = {alm_T, alm_E, alm_B, alm_T, alm_E, alm_T};
        const double *y[6] = {alm_T, alm_E, alm_B, alm_E, alm_B, alm_B};
        a.nspec = 6;
        for (int k = 0; k < 6; ++k) {
            a.x[k] = x[k];
            a.y[k] = y[k];
        }
    } else {
        a.nspec = 1;
        a.x[0] = a.y[0] = alm_T;
    }
    return launched(ctx, pisco::launch_alm2cl(a, st));
}

}  // extern "C"
