// Internal declarations of the far-sidelobe training steps (sidelobe_kernel.hip,
// sidelobe_runtime.cpp) and of the fused network epilogue used by convolve.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pisco.h"

namespace pisco {

uint64_t sl_splitmix_at(uint64_t seed, uint64_t k);
hipError_t sl_draw(uint64_t seed, int64_t n, double *th, double *ph, double *ps, hipStream_t s);
hipError_t sl_moments(const float *p, int64_t n, double *out6, hipStream_t s);
hipError_t sl_standardise(const float *p, int64_t n, const double *mom6, float *t, hipStream_t s);
hipError_t sl_gather(const float *x, const float *t, int64_t n, int64_t rows, uint64_t key, float *xs, float *ts,
                     hipStream_t s);

// One training run: `tctx` holds detector 0 set up as the annulus (zeta = 0,
// rho in (r_main, rho_max], FIXED normalisation) whose STOKES pickups are the
// targets.  On success *net holds the trained network and mean/stdv the
// standardisation of its targets; hist one mean loss per epoch.
struct SidelobeRun {
    pisco_ctx *ctx;      // the caller's context (error messages, network device)
    pisco_ctx *tctx;     // target context
    int64_t n_train;
    uint64_t seed;
    int32_t epochs;
    pisco_sidelobe_opts opts;
};
pisco_status sidelobe_train_run(const SidelobeRun &r, pisco_mlp **net, float mean[3], float stdv[3],
                                std::vector<double> &hist);

// tod[t] += sum_c coef[c] (mean[c] + stdv[c] y[t][c]) for the network's output y
// at the n pointings (th, ph, ps): the fused inference kernel, on stream s.
hipError_t mlp_apply_pointing(const pisco_mlp *m, const double *th, const double *ph, const double *ps, int64_t n,
                              const float mean[3], const float stdv[3], const double coef[3], float *tod,
                              hipStream_t s);

}  // namespace pisco
