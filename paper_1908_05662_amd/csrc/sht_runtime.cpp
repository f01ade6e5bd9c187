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

// ring Fourier sums, then the a_lm workgroups' per-wave partial sums
int64_t workspace_bytes(int64_t nside, int64_t lmax, bool pol) {
    return fourier_bytes(nside, lmax, pol) + (int64_t)pisco::SHT_WAVES * (lmax + 1) * (lmax + 2) / 2 * 6 * 8;
}

pisco_status map2alm(pisco_ctx *ctx, int64_t nside, int32_t lmax, const double *T, const double *Q, const double *U,
                     double *aT, double *aE, double *aB, void *ws, int64_t ws_bytes, hipStream_t st) {
    if (!nside_ok(nside)) return bad(ctx, "nside must be a power of two in [1, 1024]");
    if (!lmax_ok(nside, lmax)) return bad(ctx, "lmax must be in [0, 4 nside]");
    if (!T || !aT) return bad(ctx, "null T map or a^T");
    if ((Q == nullptr) != (U == nullptr)) return bad(ctx, "Q and U must both be given or both be null");
    const bool pol = Q != nullptr;
    if (pol && (!aE || !aB)) return bad(ctx, "null a^E or a^B");
    if (!ws || ws_bytes < workspace_bytes(nside, lmax, pol)) return bad(ctx, "workspace missing or too small");
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    pisco::ShtArgs a{};
    a.nside = (int)nside;
    a.lmax = lmax;
    a.mmax = lmax;
    a.nfields = pol ? 3 : 1;
    a.nrings = (int)(4 * nside - 1);
    a.map[0] = T;
    a.map[1] = Q;
    a.map[2] = U;
    a.F = static_cast<double2 *>(ws);
    a.partial = reinterpret_cast<double *>(static_cast<char *>(ws) + fourier_bytes(nside, lmax, pol));
    a.alm[0] = aT;
    a.alm[1] = pol ? aE : nullptr;
    a.alm[2] = pol ? aB : nullptr;
    hipError_t e = pisco::launch_ring_fourier(a, st);
    if (e == hipSuccess) e = pisco::launch_alm(a, st);
    return launched(ctx, e);
}

}  // namespace

extern "C" {

int64_t pisco_alm_size(int32_t lmax) { return lmax < 0 ? 0 : (int64_t)(lmax + 1) * (lmax + 2) / 2; }

int64_t pisco_map2alm_workspace_bytes(int64_t nside, int32_t lmax, int32_t pol) {
    if (!nside_ok(nside) || !lmax_ok(nside, lmax)) return -1;
    return workspace_bytes(nside, lmax, pol != 0);
}

pisco_status pisco_map2alm(pisco_ctx *ctx, int64_t nside, int32_t lmax, const double *T, const double *Q,
                           const double *U, double *alm_T, double *alm_E, double *alm_B, void *workspace,
                           int64_t workspace_bytes, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    return map2alm(ctx, nside, lmax, T, Q, U, alm_T, alm_E, alm_B, workspace, workspace_bytes,
                   static_cast<hipStream_t>(stream));
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

pisco_status pisco_anafast(pisco_ctx *ctx, int64_t nside, int32_t lmax, const double *T, const double *Q,
                           const double *U, double *alm_T, double *alm_E, double *alm_B, void *workspace,
                           int64_t workspace_bytes, double *cl, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (!cl) return bad(ctx, "null cl");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const pisco_status r = map2alm(ctx, nside, lmax, T, Q, U, alm_T, alm_E, alm_B, workspace, workspace_bytes, st);
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
