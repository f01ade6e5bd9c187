// C ABI of the binned map-maker (include/pisco.h, "binned maps" section):
// argument checks and the two launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "map_internal.h"
#include "pisco.h"
#include "pisco_internal.h"

namespace {

pisco_status bad(pisco_ctx *c, const char *msg) {
    pisco::set_error(c, msg);
    return PISCO_EINVAL;
}

bool nside_ok(int64_t n) { return n >= 1 && n <= 8192 && (n & (n - 1)) == 0; }

pisco_status launched(pisco_ctx *c, hipError_t e) {
    if (e == hipSuccess) return PISCO_OK;
    pisco::set_error(c, hipGetErrorString(e));
    return PISCO_EDEVICE;
}

}  // namespace

extern "C" {

pisco_status pisco_map_accumulate(pisco_ctx *ctx, int64_t nside_map, int64_t n, const double *theta, const double *phi,
                                  const double *psi, const double *hwp, const void *tod, int tod_dtype, double zeta,
                                  double eps, double s, double *accum, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (!nside_ok(nside_map)) return bad(ctx, "nside_map must be a power of two in [1, 8192]");
    if (n < 0) return bad(ctx, "negative sample count");
    if (tod_dtype != PISCO_F32 && tod_dtype != PISCO_F64) return bad(ctx, "bad tod dtype");
    if (!std::isfinite(zeta) || !std::isfinite(eps) || !std::isfinite(s)) return bad(ctx, "non-finite zeta, eps or s");
    if (!accum) return bad(ctx, "null accumulator");
    if (n > 0 && (!theta || !phi || !psi || !tod)) return bad(ctx, "null pointing or TOD");
    if (n == 0) return PISCO_OK;
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    pisco::MapAccumArgs a{};
    a.nside = nside_map;
    a.npix = 12 * nside_map * nside_map;
    a.n = n;
    a.theta = theta;
    a.phi = phi;
    a.psi = psi;
    a.hwp = hwp;
    a.zeta = zeta;
    a.c_int = 0.5 * s * (1.0 + eps);
    a.c_pol = 0.5 * s * (1.0 - eps);
    a.accum = accum;
    return launched(ctx, pisco::launch_map_accumulate(a, tod, tod_dtype == PISCO_F64, pisco::ctx_num_cu(ctx),
                                                      static_cast<hipStream_t>(stream)));
}

pisco_status pisco_map_solve(pisco_ctx *ctx, int64_t nside_map, const double *accum, double rcond_min, double *maps,
                             double *rcond, void *stream) {
    if (!ctx) return PISCO_EINVAL;
    if (!nside_ok(nside_map)) return bad(ctx, "nside_map must be a power of two in [1, 8192]");
    if (!accum || !maps) return bad(ctx, "null accumulator or maps");
    if (!(rcond_min >= 0.0 && rcond_min <= 1.0)) return bad(ctx, "rcond_min must be in [0, 1]");
    const hipError_t ed = hipSetDevice(pisco::ctx_device(ctx));
    if (ed != hipSuccess) return launched(ctx, ed);
    pisco::MapSolveArgs a{};
    a.npix = 12 * nside_map * nside_map;
    a.accum = accum;
    a.rcond_min = rcond_min;
    a.maps = maps;
    a.rcond = rcond;
    return launched(ctx, pisco::launch_map_solve(a, pisco::ctx_num_cu(ctx), static_cast<hipStream_t>(stream)));
}

}  // extern "C"
