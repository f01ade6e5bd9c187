// Training the far-sidelobe network behind the C ABI: exact annulus pickups of
// library-drawn pointings (the convolution kernels), standardised targets,
// shuffled Adam epochs with a cosine-decayed rate (the network kernels).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "mlp_internal.h"
#include "pisco.h"
#include "pisco_internal.h"
#include "sidelobe_internal.h"

namespace pisco {
namespace {

struct DevBufs {
    std::vector<void *> ptrs;
    ~DevBufs() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    bool get(T **p, size_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) return false;
        ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return true;
    }
};

pisco_status err(pisco_ctx *c, pisco_status st, const char *what, hipError_t e = hipSuccess) {
    char buf[256];
    if (e != hipSuccess) std::snprintf(buf, sizeof(buf), "sidelobe training: %s: %s", what, hipGetErrorString(e));
    else std::snprintf(buf, sizeof(buf), "sidelobe training: %s", what);
    set_error(c, buf);
    return st;
}

}  // namespace

pisco_status sidelobe_train_run(const SidelobeRun &r, pisco_mlp **net, float mean[3], float stdv[3],
                                std::vector<double> &hist) {
    pisco_ctx *c = r.ctx;
    const int64_t n = r.n_train;
    const int32_t B = r.opts.batch;
    *net = nullptr;
    hist.clear();
    DevBufs buf;
    double *th, *ph, *ps, *mom;
    float *P, *x, *t, *xs, *ts, *losses;
    const int64_t steps = n / B;
    const int64_t rows = steps * B;
    if (!buf.get(&th, n) || !buf.get(&ph, n) || !buf.get(&ps, n) || !buf.get(&mom, 6) || !buf.get(&P, 3 * n) ||
        !buf.get(&x, 5 * n) || !buf.get(&t, 3 * n) || !buf.get(&xs, 5 * rows) || !buf.get(&ts, 3 * rows) ||
        !buf.get(&losses, steps))
        return err(c, PISCO_ENOMEM, "device allocation of the training set failed");

    // training pointings and their exact annulus pickups (zeta = 0 frame)
    hipError_t e = sl_draw(r.seed, n, th, ph, ps, nullptr);
    if (e != hipSuccess) return err(c, PISCO_EDEVICE, "drawing the pointings", e);
    pisco_status st = pisco_set_pointing(r.tctx, 0, n, th, ph, ps, PISCO_DEVICE);
    if (st == PISCO_OK) st = pisco_convolve(r.tctx, 0, PISCO_OUT_STOKES, P, PISCO_DEVICE, nullptr);
    if (st != PISCO_OK) {
        char msg[200];
        std::snprintf(msg, sizeof(msg), "exact targets: %s", pisco_last_error(r.tctx));
        return err(c, st, msg);
    }
    e = mlp_features(th, ph, ps, n, x, nullptr);
    if (e == hipSuccess) e = sl_moments(P, n, mom, nullptr);
    if (e == hipSuccess) e = sl_standardise(P, n, mom, t, nullptr);
    double hm[6];
    if (e == hipSuccess) e = hipMemcpy(hm, mom, sizeof(hm), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return err(c, PISCO_EDEVICE, "standardising the targets", e);
    for (int k = 0; k < 3; ++k) {
        mean[k] = (float)hm[k];
        stdv[k] = (float)std::fmax(hm[3 + k], 1e-300);
    }

    pisco_mlp *m = nullptr;
    st = pisco_mlp_create(c, r.opts.width, r.opts.hidden_layers, B, pisco::sl_splitmix_at(r.seed, 0x5eedULL), &m);
    if (st != PISCO_OK) return st;
    // Adam steps over shuffled epochs; the rate decays from lr to lr_end along a
    // cosine over every step of the run
    const int64_t total = (int64_t)r.epochs * steps;
    std::vector<float> hl((size_t)steps);
    int64_t k = 0;
    for (int32_t ep = 0; ep < r.epochs; ++ep) {
        e = sl_gather(x, t, n, rows, pisco::sl_splitmix_at(r.seed ^ 0xa5a5a5a5a5a5a5a5ULL, (uint64_t)ep), xs, ts,
                      nullptr);
        if (e != hipSuccess) {
            pisco_mlp_destroy(m);
            return err(c, PISCO_EDEVICE, "shuffling the training rows", e);
        }
        for (int64_t i = 0; i < steps; ++i, ++k) {
            const double frac = (double)k / (double)(total > 1 ? total - 1 : 1);
            const float lr = (float)(r.opts.lr_end +
                                     0.5 * ((double)r.opts.lr - r.opts.lr_end) * (1.0 + std::cos(M_PI * frac)));
            st = pisco_mlp_train_step(m, xs + i * B * MLP_IN, ts + i * B * MLP_OUT, B, lr, r.opts.beta1,
                                      r.opts.beta2, r.opts.eps, losses + i, nullptr);
            if (st != PISCO_OK) {
                pisco_mlp_destroy(m);
                return st;
            }
        }
        e = hipMemcpy(hl.data(), losses, sizeof(float) * (size_t)steps, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            pisco_mlp_destroy(m);
            return err(c, PISCO_EDEVICE, "reading the losses", e);
        }
        double s = 0.0;
        for (float v : hl) s += v;
        hist.push_back(s / (double)steps);
    }
    *net = m;
    return PISCO_OK;
}

}  // namespace pisco
