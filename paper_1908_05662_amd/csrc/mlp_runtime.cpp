// C ABI of the far-sidelobe surrogate network (include/pisco.h, "sidelobe
// network" section): parameters, forward, gradients, Adam training steps,
// pointing features and the TOD epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "mlp_internal.h"
#include "pisco.h"
#include "pisco_internal.h"
#include "sidelobe_internal.h"

struct pisco_mlp {
    pisco_ctx *ctx = nullptr;
    int32_t H = 0, L = 0, max_batch = 0;
    std::vector<int32_t> dim;        // d_0 = 5, d_1..d_L = H, d_{L+1} = 3
    std::vector<int64_t> off_w, off_b;
    int64_t nparam = 0;
    int64_t step = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    __bf16 *wb = nullptr;
    int32_t mbp = 0;                 // rows of the activation buffers: max_batch rounded up to 128
    std::vector<float *> z;          // L pre-activations [mbp][H]
    std::vector<__bf16 *> a;         // L activations [mbp][H]
    std::vector<__bf16 *> aT;        // their transposes [H][mbp] (operands of the weight gradients)
    __bf16 *dz[2] = {nullptr, nullptr};      // back-propagated dL/dz [mbp][H]
    __bf16 *dzT[2] = {nullptr, nullptr};     // their transposes [H][mbp]
    __bf16 *wbT = nullptr;           // transposes of the hidden maps' BF16 weights, [L-1][H][H]
    float *y = nullptr, *xbuf = nullptr, *ybuf = nullptr;
    float *dy = nullptr;             // output-layer dL/dy [max_batch][3] (fp32)
    float *part_w = nullptr, *part_b = nullptr, *part_loss = nullptr;
    std::vector<float *> part_map;   // split-K partials of each hidden map's weight gradient
    std::vector<float *> part_bias;  // per-block partial column sums of each hidden layer's dL/dz
    float *part_in = nullptr;        // per-block partials of the input layer's weight gradient
    std::vector<void *> allocs;
};

namespace {

constexpr int ROWS_PER_WAVE = 2;    // output layer
constexpr int ROWS_PER_BLOCK = MLP_WCOL_ROWS;  // weighted column sums (bias, input- and output-layer gradients)

pisco_status mfail(pisco_mlp *m, pisco_status st, const char *msg) {
    if (m && m->ctx) pisco::set_error(m->ctx, msg);
    return st;
}

#define MLP_TRY(m, call)                                                     \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return mfail((m), PISCO_EDEVICE, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
bool alloc(pisco_mlp *m, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    m->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
}

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Split of the batch for a weight gradient of H x H: enough slices that the
// 64 x 64 output tiles times the slices make about 512 workgroups (two per
// CU), each slice a multiple of 64 rows (the GEMM's k step).
int32_t slices_for(int32_t H) {
    const int32_t tiles = (H / 64) * (H / 64);
    return std::max(1, std::min(256, (512 + tiles - 1) / tiles));
}

// Slice groups the reduction adds in parallel: the largest power of two up to
// a quarter of the slices (at most 64).
int32_t groups_for(int32_t slices) {
    int32_t g = 1;
    while (g < 64 && 2 * g * 4 <= slices) g *= 2;
    return g;
}

int32_t k_slice_for(int32_t n, int32_t H) {
    const int32_t want = slices_for(H);
    int32_t ks = ((n + want - 1) / want + 63) / 64 * 64;
    return std::max(64, ks);
}

int32_t round_up(int32_t n, int32_t q) { return (n + q - 1) / q * q; }

// The BF16 transposes of the hidden maps' weights (operands of the backward pass).
hipError_t refresh_wbT(pisco_mlp *m, hipStream_t s) {
    if (m->L < 2) return hipSuccess;
    const int64_t stride = m->off_w[2] - m->off_w[1];
    return pisco::mlp_transpose(m->wb + m->off_w[1], m->H, m->wbT, m->H, m->H, m->H, m->L - 1, stride,
                                (int64_t)m->H * m->H, s);
}

// forward (+ loss and backward when tgt != nullptr) over one chunk of n rows
// (GEMM rows padded to 128; padding rows carry stale values, never read back)
pisco_status run(pisco_mlp *m, const float *x, const float *tgt, int32_t n, float *y, float *grad, float *loss,
                 hipStream_t s) {
    const int32_t H = m->H, L = m->L;
    const int32_t np = round_up(n, 128);
    const int64_t ldt = m->mbp;
    const bool train = tgt != nullptr;
    MLP_TRY(m, pisco::mlp_in_fwd(x, m->wb + m->off_w[0], m->w + m->off_b[0], n, H, m->z[0], m->a[0], s));
    if (train && L > 1) MLP_TRY(m, pisco::mlp_transpose(m->a[0], H, m->aT[0], ldt, np, H, 1, 0, 0, s));
    for (int l = 1; l < L; ++l)
        MLP_TRY(m, pisco::mlp_gemm(pisco::MLP_EPI_FWD, m->a[l - 1], H, m->wb + m->off_w[l], H, np, H, H, H,
                                   m->w + m->off_b[l], m->z[l], m->a[l], (train && l < L - 1) ? m->aT[l] : nullptr,
                                   ldt, nullptr, nullptr, s));
    const int32_t waves = (n + ROWS_PER_WAVE - 1) / ROWS_PER_WAVE;
    int cur = 0;
    MLP_TRY(m, pisco::mlp_out(m->a[L - 1], m->z[L - 1], m->wb + m->off_w[L], m->w + m->off_b[L], n, H, y, tgt,
                              1.0f / (float)(n * MLP_OUT), m->dy, m->dz[cur], m->part_loss, waves, ROWS_PER_WAVE, s));
    if (!train) return PISCO_OK;
    MLP_TRY(m, pisco::mlp_loss_sum(m->part_loss, waves, 1.0f / (float)(n * MLP_OUT), loss, s));
    pisco::MlpReduceList R{};
    auto seg = [&](const float *part, int32_t slices, int64_t count, float *out) {
        pisco::MlpReduceSeg &g = R.seg[R.n++];
        g.part = part;
        g.slices = slices;
        g.count = count;
        g.out = out;
        g.groups = groups_for(slices);
    };
    const int32_t cblocks = (n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
    // output map: dW_out[c][u] = sum_r dY[r][c] A_L[r][u], db_out[c] = sum_r dY[r][c]
    MLP_TRY(m, pisco::mlp_wcolsum(m->a[L - 1], m->dy, MLP_OUT, n, H, m->part_w,
                                  (int64_t)MLP_OUT * H, 1, H, m->part_b, s));
    seg(m->part_w, cblocks, (int64_t)MLP_OUT * H, grad + m->off_w[L]);
    seg(m->part_b, cblocks, MLP_OUT, grad + m->off_b[L]);
    if (L > 1) MLP_TRY(m, pisco::mlp_transpose(m->dz[cur], H, m->dzT[cur], ldt, np, H, 1, 0, 0, s));
    for (int l = L - 1; l >= 1; --l) {
        // weight gradient of map l: dZ_l^T A_{l-1} over the batch, split into slices
        const int32_t ks = k_slice_for(n, H);
        const int32_t slices = (n + ks - 1) / ks;
        MLP_TRY(m, pisco::mlp_gemm(pisco::MLP_EPI_BWD_W, m->dzT[cur], ldt, m->aT[l - 1], ldt, H, H, n, ks, nullptr,
                                   nullptr, nullptr, nullptr, 0, nullptr, m->part_map[l], s));
        seg(m->part_map[l], slices, (int64_t)H * H, grad + m->off_w[l]);
        MLP_TRY(m, pisco::mlp_wcolsum(m->dz[cur], nullptr, 1, n, H, m->part_bias[l], H, 1, 0,
                                      nullptr, s));
        seg(m->part_bias[l], cblocks, H, grad + m->off_b[l]);
        // gradient into the previous layer's pre-activation (and its transpose unless it is layer 0)
        const int nxt = cur ^ 1;
        MLP_TRY(m, pisco::mlp_gemm(pisco::MLP_EPI_BWD_D, m->dz[cur], H, m->wbT + (int64_t)(l - 1) * H * H, H, np, H,
                                   H, H, nullptr, nullptr, m->dz[nxt], l > 1 ? m->dzT[nxt] : nullptr, ldt,
                                   m->z[l - 1], nullptr, s));
        cur = nxt;
    }
    // input map: dW0[u][k] = sum_r dZ_1[r][u] X[r][k], and the first bias
    MLP_TRY(m, pisco::mlp_wcolsum(m->dz[cur], x, MLP_IN, n, H, m->part_in, (int64_t)H * MLP_IN,
                                  MLP_IN, 1, nullptr, s));
    seg(m->part_in, cblocks, (int64_t)H * MLP_IN, grad + m->off_w[0]);
    MLP_TRY(m, pisco::mlp_wcolsum(m->dz[cur], nullptr, 1, n, H, m->part_bias[0], H, 1, 0, nullptr,
                                  s));
    seg(m->part_bias[0], cblocks, H, grad + m->off_b[0]);
    MLP_TRY(m, pisco::mlp_reduce_many(R, s));
    return PISCO_OK;
}

}  // namespace

namespace pisco {
// one fused launch over the whole stream (features, every layer and the
// epilogue on chip); equal bit for bit to features + forward + apply
hipError_t mlp_apply_pointing(const pisco_mlp *m, const double *th, const double *ph, const double *ps, int64_t n,
                              const float mean[3], const float stdv[3], const double coef[3], float *tod,
                              hipStream_t s) {
    MlpInferArgs a{};
    a.th = th;
    a.ph = ph;
    a.ps = ps;
    a.n = n;
    a.H = m->H;
    a.L = m->L;
    a.wb = m->wb;
    a.w = m->w;
    for (int l = 0; l <= m->L; ++l) {
        a.off_w[l] = m->off_w[l];
        a.off_b[l] = m->off_b[l];
    }
    for (int c = 0; c < MLP_OUT; ++c) {
        a.mean[c] = mean[c];
        a.stdv[c] = stdv[c];
        a.coef[c] = coef[c];
    }
    a.tod = tod;
    return mlp_infer_apply(a, s);
}
}  // namespace pisco

extern "C" {

pisco_status pisco_mlp_create(pisco_ctx *ctx, int32_t width, int32_t hidden_layers, int32_t max_batch, uint64_t seed,
                              pisco_mlp **out) {
    if (!ctx || !out) return PISCO_EINVAL;
    *out = nullptr;
    if (width < 64 || width > 512 || width % 64 != 0) {
        pisco::set_error(ctx, "width must be a multiple of 64 in [64, 512]");
        return PISCO_EINVAL;
    }
    if (hidden_layers < 1 || hidden_layers > 16) {
        pisco::set_error(ctx, "hidden_layers must be in [1, 16]");
        return PISCO_EINVAL;
    }
    if (max_batch < 64 || max_batch > (1 << 22) || max_batch % 64 != 0) {
        pisco::set_error(ctx, "max_batch must be a multiple of 64 in [64, 4194304]");
        return PISCO_EINVAL;
    }
    if (hipSetDevice(pisco::ctx_device(ctx)) != hipSuccess) return PISCO_EDEVICE;
    pisco_mlp *m = new pisco_mlp();
    m->ctx = ctx;
    m->H = width;
    m->L = hidden_layers;
    m->max_batch = max_batch;
    m->dim.push_back(MLP_IN);
    for (int l = 0; l < hidden_layers; ++l) m->dim.push_back(width);
    m->dim.push_back(MLP_OUT);
    int64_t o = 0;
    for (int l = 0; l <= hidden_layers; ++l) {
        m->off_w.push_back(o);
        o += (int64_t)m->dim[l + 1] * m->dim[l];
        m->off_b.push_back(o);
        o += m->dim[l + 1];
    }
    m->nparam = o;
    m->mbp = round_up(max_batch, 128);
    const size_t act = (size_t)m->mbp * width;
    const int32_t waves = (max_batch + ROWS_PER_WAVE - 1) / ROWS_PER_WAVE;
    const int32_t cblocks = (max_batch + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
    const int32_t slices = std::max(slices_for(width), (max_batch + k_slice_for(max_batch, width) - 1) /
                                                           k_slice_for(max_batch, width));
    bool ok = alloc(m, &m->w, o) && alloc(m, &m->m, o) && alloc(m, &m->v, o) && alloc(m, &m->g, o) &&
              alloc(m, &m->wb, o) && alloc(m, &m->dz[0], act) && alloc(m, &m->dz[1], act) &&
              alloc(m, &m->dzT[0], act) && alloc(m, &m->dzT[1], act) &&
              alloc(m, &m->wbT, (size_t)std::max(1, hidden_layers - 1) * width * width) &&
              alloc(m, &m->y, (size_t)max_batch * MLP_OUT) && alloc(m, &m->xbuf, (size_t)max_batch * MLP_IN) &&
              alloc(m, &m->ybuf, (size_t)max_batch * MLP_OUT) &&
              alloc(m, &m->dy, (size_t)max_batch * MLP_OUT) &&
              alloc(m, &m->part_w, (size_t)cblocks * MLP_OUT * width) &&
              alloc(m, &m->part_b, (size_t)cblocks * MLP_OUT) && alloc(m, &m->part_loss, waves) &&
              alloc(m, &m->part_in, (size_t)cblocks * width * MLP_IN);
    m->part_map.assign(hidden_layers, nullptr);
    m->part_bias.assign(hidden_layers, nullptr);
    for (int l = 0; l < hidden_layers && ok; ++l) {
        float *zz = nullptr;
        __bf16 *aa = nullptr, *at = nullptr;
        ok = alloc(m, &zz, act) && alloc(m, &aa, act) && alloc(m, &at, act) &&
             alloc(m, &m->part_bias[l], (size_t)cblocks * width) &&
             (l == 0 || alloc(m, &m->part_map[l], (size_t)slices * width * width));
        m->z.push_back(zz);
        m->a.push_back(aa);
        m->aT.push_back(at);
    }
    if (!ok) {
        pisco_mlp_destroy(m);
        pisco::set_error(ctx, "sidelobe network allocation failed");
        return PISCO_ENOMEM;
    }
    // seeded initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0
    std::vector<float> host((size_t)o, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l <= hidden_layers; ++l) {
        const float a = 1.0f / std::sqrt((float)m->dim[l]);
        const int64_t cnt = (int64_t)m->dim[l + 1] * m->dim[l];
        for (int64_t i = 0; i < cnt; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            host[m->off_w[l] + i] = (float)((2.0 * u - 1.0) * a);
        }
    }
    if (pisco_mlp_set_params(m, host.data(), PISCO_HOST) != PISCO_OK) {
        pisco_mlp_destroy(m);
        return PISCO_EDEVICE;
    }
    *out = m;
    return PISCO_OK;
}

void pisco_mlp_destroy(pisco_mlp *m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
}

int64_t pisco_mlp_param_count(const pisco_mlp *m) { return m ? m->nparam : -1; }

pisco_status pisco_mlp_layout(const pisco_mlp *m, int32_t layer, int64_t *w_offset, int64_t *b_offset, int32_t *rows,
                              int32_t *cols) {
    if (!m || layer < 0 || layer > m->L) return PISCO_EINVAL;
    if (w_offset) *w_offset = m->off_w[layer];
    if (b_offset) *b_offset = m->off_b[layer];
    if (rows) *rows = m->dim[layer + 1];
    if (cols) *cols = m->dim[layer];
    return PISCO_OK;
}

pisco_status pisco_mlp_set_params(pisco_mlp *m, const float *params, int mem) {
    if (!m || !params) return PISCO_EINVAL;
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return mfail(m, PISCO_EINVAL, "bad mem");
    const size_t b = sizeof(float) * (size_t)m->nparam;
    MLP_TRY(m, hipMemcpy(m->w, params, b, mem == PISCO_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice));
    MLP_TRY(m, hipMemset(m->m, 0, b));
    MLP_TRY(m, hipMemset(m->v, 0, b));
    MLP_TRY(m, pisco::mlp_to_bf16(m->w, m->wb, m->nparam, nullptr));
    MLP_TRY(m, refresh_wbT(m, nullptr));
    MLP_TRY(m, hipDeviceSynchronize());
    m->step = 0;
    return PISCO_OK;
}

pisco_status pisco_mlp_get_params(const pisco_mlp *m, float *params, int mem) {
    if (!m || !params) return PISCO_EINVAL;
    const size_t b = sizeof(float) * (size_t)m->nparam;
    if (hipDeviceSynchronize() != hipSuccess) return PISCO_EDEVICE;
    if (hipMemcpy(params, m->w, b, mem == PISCO_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice) != hipSuccess)
        return PISCO_EDEVICE;
    return PISCO_OK;
}

pisco_status pisco_mlp_forward(pisco_mlp *m, const float *x, int64_t n, float *y, void *stream) {
    if (!m || (n > 0 && (!x || !y)) || n < 0) return PISCO_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int64_t b = 0; b < n; b += m->max_batch) {
        const int32_t c = (int32_t)std::min<int64_t>(m->max_batch, n - b);
        const pisco_status st = run(m, x + b * MLP_IN, nullptr, c, y + b * MLP_OUT, nullptr, nullptr, s);
        if (st != PISCO_OK) return st;
    }
    return PISCO_OK;
}

pisco_status pisco_mlp_gradient(pisco_mlp *m, const float *x, const float *t, int32_t n, float *grad, float *loss,
                                void *stream) {
    if (!m || !x || !t || !grad || !loss) return PISCO_EINVAL;
    if (n < 64 || n > m->max_batch || n % 64 != 0)
        return mfail(m, PISCO_EINVAL, "batch must be a multiple of 64 and at most max_batch");
    return run(m, x, t, n, m->y, grad, loss, static_cast<hipStream_t>(stream));
}

pisco_status pisco_mlp_train_step(pisco_mlp *m, const float *x, const float *t, int32_t n, float lr, float beta1,
                                  float beta2, float eps, float *loss, void *stream) {
    if (!m || !x || !t || !loss) return PISCO_EINVAL;
    if (n < 64 || n > m->max_batch || n % 64 != 0)
        return mfail(m, PISCO_EINVAL, "batch must be a multiple of 64 and at most max_batch");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return mfail(m, PISCO_EINVAL, "bad Adam hyper-parameters");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pisco_status st = run(m, x, t, n, m->y, m->g, loss, s);
    if (st != PISCO_OK) return st;
    m->step += 1;
    const double bc1 = 1.0 - std::pow((double)beta1, (double)m->step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)m->step);
    // w -= lr * mhat / (sqrt(vhat) + eps), mhat = m / bc1, vhat = v / bc2
    const float lr_t = (float)(lr / bc1);
    const float inv = (float)(1.0 / std::sqrt(bc2));
    MLP_TRY(m, pisco::mlp_adam(m->w, m->m, m->v, m->g, m->wb, m->nparam, lr_t, beta1, beta2, eps, inv, s));
    MLP_TRY(m, refresh_wbT(m, s));
    return PISCO_OK;
}

pisco_status pisco_sidelobe_features(pisco_ctx *ctx, int32_t det, float *x, void *stream) {
    const double *th, *ph, *ps;
    int64_t n = 0;
    if (!ctx || !x) return PISCO_EINVAL;
    if (!pisco::ctx_pointing(ctx, det, &th, &ph, &ps, &n)) {
        pisco::set_error(ctx, "detector has no pointing");
        return PISCO_ESTATE;
    }
    const hipError_t e = pisco::mlp_features(th, ph, ps, n, x, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        pisco::set_error(ctx, hipGetErrorString(e));
        return PISCO_EDEVICE;
    }
    return PISCO_OK;
}

pisco_status pisco_sidelobe_apply(pisco_ctx *ctx, pisco_mlp *m, int32_t det, const float *mean, const float *stdv,
                                  const double *coef, float *tod, void *stream) {
    const double *th, *ph, *ps;
    int64_t n = 0;
    if (!ctx || !m || !mean || !stdv || !coef || !tod) return PISCO_EINVAL;
    if (!pisco::ctx_pointing(ctx, det, &th, &ph, &ps, &n)) {
        pisco::set_error(ctx, "detector has no pointing");
        return PISCO_ESTATE;
    }
    MLP_TRY(m, pisco::mlp_apply_pointing(m, th, ph, ps, n, mean, stdv, coef, tod, static_cast<hipStream_t>(stream)));
    return PISCO_OK;
}

}  // extern "C"
