// Host runtime behind the C ABI declared in include/pisco.h: device buffers,
// validation, the tile plan and work queues, HIP-graph replay of the batched
// launch, and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "pisco.h"
#include "pisco_internal.h"
#include "sidelobe_internal.h"

using pisco::ConvArgs;
using pisco::DetDesc;
using pisco::Tile;

namespace {

// A trained far-sidelobe network and what its outputs mean: the annulus
// (r_main, R] pickups of the training detector's beam at zeta = 0, which
// include that detector's wT and normalisation.  Shared by every detector that
// uses it; released with the last one.
struct SlNet {
    pisco_mlp *net = nullptr;
    float mean[3] = {0.0f, 0.0f, 0.0f}, stdv[3] = {1.0f, 1.0f, 1.0f};
    double r_main = 0.0, wT = 1.0, norm = 1.0;
    std::vector<double> hist;
    SlNet() = default;
    SlNet(const SlNet &) = delete;
    SlNet &operator=(const SlNet &) = delete;
    ~SlNet() {
        if (net) pisco_mlp_destroy(net);
    }
};

struct DetState {
    bool has_beam = false, has_params = false, has_pointing = false;
    void *beam = nullptr;   // device records
    bool beam_owned = false;
    int32_t n = 0;
    double T = 0.0;
    int beam_dtype = -1;
    int beam_kind = pisco::BEAM_FULL;
    double w[4] = {1.0, 1.0, 1.0, 1.0};
    void *beam_v = nullptr;  // full beams: bV cell polynomials (owned with the beam)
    double wv = 0.0;         // scalar beams: V weight
    const double *hwp = nullptr;      // plate angle per sample, or null
    double *owned_hwp = nullptr;
    int64_t hwp_n = 0;
    double zeta = 0.0, rho_min = 0.0, rho_max = 0.0, norm_scale = 1.0;
    int norm_mode = 0;
    int64_t nsamp = 0;
    const double *th = nullptr, *ph = nullptr, *ps = nullptr;
    double *owned_pointing = nullptr;  // one allocation holding th, ph, ps when copied
    int32_t *order = nullptr;          // spatial processing order of the pointing (plan-time), owned
    size_t order_cap = 0;
    std::vector<double> host_pointing;  // pointing kept on the host (memory budget): theta | phi | psi
    std::vector<double> host_hwp;       // plate angles kept on the host (memory budget)
    // far-sidelobe surrogate: a network standing in for the annulus beyond its r_main
    std::shared_ptr<SlNet> sl;
    bool sl_on = false;
};

struct TimedLaunch {
    hipEvent_t a, b;
};

}  // namespace

// A set of work queues: tiles[q * per + i], with 8 counters and 8 lengths in
// the plan's control block.
struct Queues {
    Tile *d_tiles = nullptr;
    size_t cap = 0;
    int32_t per = 1, nq = 1;
    int64_t ntiles = 0;
};

// The fused network epilogue of one surrogate-substituted detector in a launch.
struct SlApply {
    const pisco_mlp *net;
    const double *th, *ph, *ps;
    int64_t n, out_offset;
    float mean[3], stdv[3];
    double coef[3];
};

// A device-side launch plan: detector descriptors, the tile-path and
// pixel-path work queues, and (for the batched plan) the captured graph.  The
// context keeps one plan for single-detector launches and one for the batched
// launch so that eager single-detector calls never invalidate the graph.
struct Plan {
    DetDesc *d_dets = nullptr;
    size_t d_dets_cap = 0;
    Queues tq, pq;              // tile path (coherent 64-sample groups), pixel path
    int32_t *d_ctrl = nullptr;  // [0,8) tq counters, [8,16) tq lengths, [16,24) pq counters, [24,32) pq lengths
    int32_t *d_scratch = nullptr;
    size_t scratch_cap = 0;     // bytes
    uint64_t gen = 0;
    int32_t det = -2;
    int32_t spt = 0, xq = 0, algo = -1;
    double coherence = 0.0;
    int64_t out_samples = 0;
    int32_t beam_kind = 0;
    int32_t per_sample = 0;  // some detector of the plan normalises per sample
    int32_t vbeam = 0;       // some detector of the plan has a full beam with a V column
    int32_t hwp = 0;         // some detector of the plan has a half-wave plate
    int32_t extended = 0;    // some detector has a plate or V terms (not on the matrix-core path)
    int32_t sub = -1;        // TOD plans: surrogate-enabled detectors run their main disc + network
    std::vector<SlApply> sl; // their epilogues
    // captured launch
    hipGraphExec_t gexec = nullptr;
    uint64_t g_gen = 0;
    void *g_out = nullptr;
    hipStream_t g_stream = nullptr;
    int g_mode = -1;
    int32_t g_wpg = 0, g_gpc = 0, g_chunk = 0;
};

struct pisco_ctx {
    int device = 0;
    int num_cu = 256;
    std::string err;
    int64_t nside = 0;
    int sky_dtype = -1;
    void *sky = nullptr;
    std::vector<DetState> dets;
    uint64_t generation = 1;  // bumped whenever anything a launch reads changes

    // launch shape
    int32_t spt = 64, wpg = 4, gpc = 4, xq = 1;
    int32_t algo = PISCO_ALGO_TILE, chunk = 64;
    double coherence = 0.5;
    int32_t ordering = PISCO_ORDER_AUTO;   // processing order of the samples

    Plan plans[3];            // [0] batched (det = -1), [1] single detector, [2] blocks of the budgeted path
    int32_t *d_flag = nullptr;

    // device memory counted against the budget (0: none)
    int64_t budget = 0, in_use = 0;
    std::unordered_map<void *, size_t> dsize;
    bool sky_owned = true;     // false: the sky records are borrowed from another context
    pisco_sidelobe_opts sl_opts = {256, 4, 8192, 2e-3f, 2e-5f, 0.9f, 0.999f, 1e-8f};

    bool timing = false;
    std::vector<TimedLaunch> pending;
    double total_ms = 0.0;
    int64_t launches = 0;
};

namespace {

pisco_status fail(pisco_ctx *c, pisco_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIP_TRY(ctx, call)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail((ctx), PISCO_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

size_t rec_bytes(int dtype) { return dtype == PISCO_F64 ? 32 : 16; }
size_t el_bytes(int dtype) { return dtype == PISCO_F64 ? 8 : 4; }

// Device allocations of a context, counted against its memory budget.
bool dmalloc(pisco_ctx *c, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    if (c->budget > 0 && c->in_use + (int64_t)bytes > c->budget) return false;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return false;
    }
    c->dsize[*p] = bytes;
    c->in_use += (int64_t)bytes;
    return true;
}

void dfree(pisco_ctx *c, void *p) {
    if (!p) return;
    auto it = c->dsize.find(p);
    if (it != c->dsize.end()) {
        c->in_use -= (int64_t)it->second;
        c->dsize.erase(it);
    }
    (void)hipFree(p);
}

DetState *det_slot(pisco_ctx *c, int32_t det) {
    if (det < 0 || det >= PISCO_MAX_DETECTORS) return nullptr;
    if ((size_t)det >= c->dets.size()) c->dets.resize(det + 1);
    return &c->dets[det];
}

bool det_ready(const DetState &d) { return d.has_beam && d.has_params && d.has_pointing; }

// The trained far-sidelobe network of a detector no longer matches once its
// beam or disc changes.
void release_sidelobe(DetState &d) {
    d.sl.reset();
    d.sl_on = false;
}

void release_beam(pisco_ctx *c, int32_t det) {
    DetState &d = c->dets[det];
    if (d.beam_owned && d.beam) {
        // detectors sharing this buffer lose their beam
        for (size_t k = 0; k < c->dets.size(); ++k)
            if ((int32_t)k != det && c->dets[k].beam == d.beam && !c->dets[k].beam_owned) {
                c->dets[k].beam = nullptr;
                c->dets[k].beam_v = nullptr;
                c->dets[k].has_beam = false;
                release_sidelobe(c->dets[k]);
            }
        dfree(c, d.beam);
        dfree(c, d.beam_v);
    }
    d.beam = nullptr;
    d.beam_v = nullptr;
    d.wv = 0.0;
    d.beam_owned = false;
    d.has_beam = false;
    release_sidelobe(d);
}

void release_hwp(pisco_ctx *c, DetState &d) {
    dfree(c, d.owned_hwp);
    d.owned_hwp = nullptr;
    d.hwp = nullptr;
    d.hwp_n = 0;
    std::vector<double>().swap(d.host_hwp);
}

void release_pointing(pisco_ctx *c, DetState &d) {
    dfree(c, d.owned_pointing);
    d.owned_pointing = nullptr;
    dfree(c, d.order);
    std::vector<double>().swap(d.host_pointing);
    d.order = nullptr;
    d.order_cap = 0;
    d.th = d.ph = d.ps = nullptr;
    d.nsamp = 0;
    d.has_pointing = false;
}

void drop_graph(Plan &p) {
    if (p.gexec) (void)hipGraphExecDestroy(p.gexec);
    p.gexec = nullptr;
}

void free_plan(pisco_ctx *c, Plan &p) {
    drop_graph(p);
    dfree(c, p.d_dets);
    dfree(c, p.tq.d_tiles);
    dfree(c, p.pq.d_tiles);
    dfree(c, p.d_ctrl);
    dfree(c, p.d_scratch);
    p = Plan();
}

// Copy a host or device array to a fresh device buffer of `bytes`.
pisco_status to_device(pisco_ctx *c, const void *src, size_t bytes, int mem, void **out) {
    void *p = nullptr;
    if (bytes == 0) {
        *out = nullptr;
        return PISCO_OK;
    }
    if (!dmalloc(c, &p, bytes)) return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", bytes);
    const hipError_t e = hipMemcpy(p, src, bytes, mem == PISCO_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dfree(c, p);
        return fail(c, PISCO_EDEVICE, "copy to device failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return PISCO_OK;
}

// Interleave four n-element channels into n 16/32-byte records on the device.
pisco_status interleave(pisco_ctx *c, const void *a, const void *b, const void *cc, const void *d, int64_t n,
                        int dtype, int mem, void **out) {
    const size_t eb = el_bytes(dtype);
    void *rec = nullptr;
    if (!dmalloc(c, &rec, rec_bytes(dtype) * (size_t)n))
        return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", rec_bytes(dtype) * (size_t)n);
    const void *src[4] = {a, b, cc, d};
    void *tmp[4] = {nullptr, nullptr, nullptr, nullptr};
    pisco_status st = PISCO_OK;
    for (int k = 0; k < 4 && st == PISCO_OK; ++k) {
        if (!src[k]) continue;
        if (mem == PISCO_DEVICE) {
            tmp[k] = const_cast<void *>(src[k]);
        } else {
            st = to_device(c, src[k], eb * (size_t)n, PISCO_HOST, &tmp[k]);
        }
    }
    if (st == PISCO_OK) {
        hipError_t e = pisco::launch_repack4(tmp[0], tmp[1], tmp[2], tmp[3], rec, n, dtype == PISCO_F64, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) st = fail(c, PISCO_EDEVICE, "repack failed: %s", hipGetErrorString(e));
    }
    if (mem == PISCO_HOST)
        for (int k = 0; k < 4; ++k)
            dfree(c, tmp[k]);
    if (st != PISCO_OK) {
        dfree(c, rec);
        return st;
    }
    *out = rec;
    return PISCO_OK;
}

template <typename T>
bool grow(pisco_ctx *c, T **p, size_t *cap, size_t need) {
    if (*cap >= need) return true;
    size_t nc = std::max(need, *cap * 2 + 16);
    void *q = nullptr;
    if (!dmalloc(c, &q, nc * sizeof(T)) && !(nc > need && dmalloc(c, &q, (nc = need) * sizeof(T)))) return false;
    dfree(c, *p);
    *p = static_cast<T *>(q);
    *cap = nc;
    return true;
}

// Split tiles into nq contiguous blocks, one per queue.
void fill_queues(const std::vector<Tile> &tiles, int nq, std::vector<Tile> &qt, int32_t *len, int32_t &per) {
    const size_t ntile = tiles.size();
    per = std::max<int32_t>(1, (int32_t)((ntile + nq - 1) / nq));
    qt.assign((size_t)per * nq, Tile{});
    for (int q = 0; q < 8; ++q) len[q] = 0;
    for (int q = 0; q < nq; ++q) {
        const size_t b = std::min(ntile, (size_t)q * per), e = std::min(ntile, b + per);
        for (size_t i = b; i < e; ++i) qt[(size_t)q * per + (i - b)] = tiles[i];
        len[q] = (int32_t)(e - b);
    }
}

// Weights of the annulus pickup (P_I, P_Q, P_U at zeta = 0) in the TOD of a
// scalar-beam detector at angle zeta: the pixel angle chi grows by zeta, which
// turns the Q, U pickups by 2 zeta.
// The pickups of a network trained on another detector's beam carry that
// detector's wT and normalisation instead of this one's.
void sidelobe_coef(const DetState &d, double coef[3]) {
    const double c2 = std::cos(2.0 * d.zeta), s2 = std::sin(2.0 * d.zeta);
    const double f = d.norm_scale / (d.sl->norm * d.sl->wT);
    coef[0] = f * d.w[0];
    coef[1] = f * (d.w[1] * c2 - d.w[2] * s2);
    coef[2] = f * (d.w[1] * s2 + d.w[2] * c2);
}

// The kernels' description of a detector (pointing and output offset left to
// the caller).  sub: the detector's trained surrogate stands in for the
// annulus, so the exact disc ends at its main radius.
DetDesc make_desc(const DetState &d, bool sub) {
    DetDesc x{};
    const double rho_max = sub ? std::min(d.rho_max, d.sl->r_main) : d.rho_max;
    x.beam = d.beam;
    x.n_samples = d.nsamp;
    x.zeta = d.zeta;
    x.cos_rho_max = std::cos(rho_max);
    x.cos_rho_min = std::cos(d.rho_min);
    x.rho_max = rho_max;
    x.norm_scale = d.norm_scale;
    x.half_span_tan = d.T;
    x.inv_h = (double)(d.n - 1) / (2.0 * d.T);
    x.rot2z[0] = std::cos(2.0 * d.zeta) / (x.inv_h * x.inv_h);
    x.rot2z[1] = std::sin(2.0 * d.zeta) / (x.inv_h * x.inv_h);
    x.omega_max = 2.0 * std::sin(0.5 * rho_max) * std::sin(0.5 * rho_max);
    x.omega_min = 2.0 * std::sin(0.5 * d.rho_min) * std::sin(0.5 * d.rho_min);
    for (int i = 0; i < 4; ++i) x.w[i] = d.w[i];
    x.beam_v = d.beam_v;
    x.wv = d.wv;
    x.hwp = d.hwp;
    // a disc inside the grid's square maps every member into the grid (|u|, |v| <= tan rho)
    x.needs_clip = (std::tan(rho_max) <= d.T * (1.0 + 1e-12)) ? 0 : 1;
    x.n = d.n;
    x.norm_mode = d.norm_mode;
    x.has_inner = d.rho_min > 0.0 ? 1 : 0;
    x.order = nullptr;
    return x;
}

// Upload descriptors, classify their 64-sample groups (tile paths) and fill the
// work queues of plan p.  det_of[i] names the detector of descs[i] (for its
// spatial processing order, taken when may_reorder).
pisco_status build_plan(pisco_ctx *c, Plan &p, std::vector<DetDesc> &descs, const std::vector<int32_t> &det_of,
                        bool may_reorder) {
    p.per_sample = 0;
    p.hwp = 0;
    p.vbeam = 0;
    p.extended = 0;
    int64_t out_end = 0;
    for (const DetDesc &x : descs) {
        if (x.hwp) p.hwp = 1;
        if (x.beam_v) p.vbeam = 1;
        if (x.beam_v || x.wv != 0.0 || x.hwp) p.extended = 1;
        if (x.norm_mode == PISCO_NORM_PER_SAMPLE) p.per_sample = 1;
        out_end = std::max(out_end, x.out_offset + x.n_samples);
    }
    hipError_t e = hipDeviceSynchronize();  // no launch may still read the old plan
    if (e != hipSuccess) return fail(c, PISCO_EDEVICE, "synchronise failed: %s", hipGetErrorString(e));
    p.gen = 0;  // the plan is incomplete until the end of this function
    drop_graph(p);
    if (!p.d_ctrl && !dmalloc(c, reinterpret_cast<void **>(&p.d_ctrl), 32 * sizeof(int32_t)))
        return fail(c, PISCO_ENOMEM, "plan allocation failed");
    if (!grow(c, &p.d_dets, &p.d_dets_cap, std::max<size_t>(descs.size(), 1)))
        return fail(c, PISCO_ENOMEM, "plan allocation failed");
    // the spatial processing order of a descriptor's detector (device sort)
    auto set_order = [&](size_t i) -> pisco_status {
        DetState &d = c->dets[det_of[i]];
        if (!grow(c, &d.order, &d.order_cap, std::max<size_t>((size_t)d.nsamp, 1)))
            return fail(c, PISCO_ENOMEM, "order allocation failed");
        const hipError_t eo = pisco::spatial_order(d.th, d.ph, d.nsamp, d.order, nullptr);
        if (eo != hipSuccess) return fail(c, PISCO_EDEVICE, "spatial ordering failed: %s", hipGetErrorString(eo));
        descs[i].order = d.order;
        return PISCO_OK;
    };
    if (may_reorder && c->ordering == PISCO_ORDER_SPATIAL)
        for (size_t i = 0; i < descs.size(); ++i)
            if (descs[i].n_samples > 64) {
                const pisco_status so = set_order(i);
                if (so != PISCO_OK) return so;
            }
    if (!descs.empty()) HIP_TRY(c, hipMemcpy(p.d_dets, descs.data(), descs.size() * sizeof(DetDesc), hipMemcpyHostToDevice));

    // groups of up to 64 consecutive samples (in processing order); on the tile
    // path each group is classified on the device as coherent (tile kernel) or
    // not (pixel kernel)
    std::vector<Tile> groups;
    for (size_t i = 0; i < descs.size(); ++i)
        for (int64_t b = 0; b < descs[i].n_samples; b += 64) {
            Tile t;
            t.det = (int32_t)i;
            t.begin = b;
            t.count = (int32_t)std::min<int64_t>(64, descs[i].n_samples - b);
            groups.push_back(t);
        }
    std::vector<int32_t> flag(groups.size(), 0);
    const bool tile_path = (c->algo == PISCO_ALGO_TILE || c->algo == PISCO_ALGO_TILE_MX) && (c->sky_dtype == PISCO_F32);
    auto classify = [&]() -> pisco_status {
        if (!tile_path || groups.empty()) return PISCO_OK;
        const size_t need = groups.size() * (sizeof(Tile) + sizeof(int32_t));
        if (p.scratch_cap < need) {
            dfree(c, p.d_scratch);
            p.d_scratch = nullptr;
            p.scratch_cap = 0;
            if (!dmalloc(c, reinterpret_cast<void **>(&p.d_scratch), need))
                return fail(c, PISCO_ENOMEM, "plan scratch allocation failed");
            p.scratch_cap = need;
        }
        Tile *dg = reinterpret_cast<Tile *>(p.d_scratch);
        int32_t *df = reinterpret_cast<int32_t *>(dg + groups.size());
        HIP_TRY(c, hipMemcpy(dg, groups.data(), groups.size() * sizeof(Tile), hipMemcpyHostToDevice));
        HIP_TRY(c, pisco::launch_classify(p.d_dets, dg, (int32_t)groups.size(), c->coherence, df, nullptr));
        HIP_TRY(c, hipMemcpy(flag.data(), df, groups.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        return PISCO_OK;
    };
    pisco_status cs = classify();
    if (cs != PISCO_OK) return cs;
    if (may_reorder && c->ordering == PISCO_ORDER_AUTO && tile_path) {
        // detectors whose given order leaves most groups incoherent are processed in spatial order
        std::vector<int64_t> coherent(descs.size(), 0), total(descs.size(), 0);
        for (size_t g = 0; g < groups.size(); ++g) {
            ++total[groups[g].det];
            coherent[groups[g].det] += flag[g] ? 1 : 0;
        }
        bool any = false;
        for (size_t i = 0; i < descs.size(); ++i)
            if (total[i] >= 2 && 2 * coherent[i] < total[i]) {
                const pisco_status so = set_order(i);
                if (so != PISCO_OK) return so;
                any = true;
            }
        if (any) {
            HIP_TRY(c, hipMemcpy(p.d_dets, descs.data(), descs.size() * sizeof(DetDesc), hipMemcpyHostToDevice));
            cs = classify();
            if (cs != PISCO_OK) return cs;
        }
    }
    // pixel path: runs of incoherent groups of one detector merged, then cut into
    // tiles of at most spt samples, and of fewer when the pixel path has fewer
    // samples than twice the launch's waves hold at spt each (a wave takes one
    // sample at a time, so small tiles spread a few incoherent groups -- scan
    // discontinuities -- over the whole chip instead of a few waves)
    int64_t pix_samples = 0;
    for (size_t g = 0; g < groups.size(); ++g)
        if (!flag[g]) pix_samples += groups[g].count;
    // (under a memory budget at least 16 samples a tile: the block sizing allows
    // about 2 bytes of queues per sample)
    const int64_t waves = std::max<int64_t>(1, (int64_t)c->gpc * c->num_cu * c->wpg);
    const int64_t min_pspt = c->budget > 0 ? 16 : 1;
    const int32_t pspt = (int32_t)std::min<int64_t>(
        c->spt, std::max<int64_t>(min_pspt, (pix_samples + 2 * waves - 1) / (2 * waves)));
    std::vector<Tile> ttiles, ptiles;
    for (size_t g = 0; g < groups.size(); ++g) {
        if (flag[g]) {
            ttiles.push_back(groups[g]);
            continue;
        }
        Tile x = groups[g];
        while (x.count > 0) {
            if (!ptiles.empty() && ptiles.back().det == x.det && ptiles.back().begin + ptiles.back().count == x.begin &&
                ptiles.back().count < pspt) {
                Tile &b = ptiles.back();
                const int32_t take = std::min(pspt - b.count, x.count);
                b.count += take;
                x.begin += take;
                x.count -= take;
            } else {
                Tile t = x;
                t.count = std::min(pspt, x.count);
                ptiles.push_back(t);
                x.begin += t.count;
                x.count -= t.count;
            }
        }
    }
    // each detector's coherent tiles in the Hilbert order of their first samples:
    // tiles that run at the same time then share more of their union caps in
    // L2 (the order of tiles does not change any output)
    if (ttiles.size() > 1) {
        Tile *dg = reinterpret_cast<Tile *>(p.d_scratch);
        uint32_t *dk = reinterpret_cast<uint32_t *>(dg + ttiles.size());
        std::vector<uint32_t> key(ttiles.size());
        HIP_TRY(c, hipMemcpy(dg, ttiles.data(), ttiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
        HIP_TRY(c, pisco::launch_tile_keys(p.d_dets, dg, (int32_t)ttiles.size(), dk, nullptr));
        HIP_TRY(c, hipMemcpy(key.data(), dk, key.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
        std::vector<size_t> idx(ttiles.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
            return ttiles[a].det != ttiles[b].det ? ttiles[a].det < ttiles[b].det : key[a] < key[b];
        });
        std::vector<Tile> sorted(ttiles.size());
        for (size_t i = 0; i < idx.size(); ++i) sorted[i] = ttiles[idx[i]];
        ttiles.swap(sorted);
    }
    const int nq = std::max<int32_t>(1, std::min<int32_t>(c->xq, 8));
    int32_t lens[32] = {0};
    std::vector<Tile> tq, pq;
    fill_queues(ttiles, nq, tq, lens + 8, p.tq.per);
    fill_queues(ptiles, nq, pq, lens + 24, p.pq.per);
    if (!grow(c, &p.tq.d_tiles, &p.tq.cap, tq.size()) || !grow(c, &p.pq.d_tiles, &p.pq.cap, pq.size()))
        return fail(c, PISCO_ENOMEM, "plan allocation failed");
    HIP_TRY(c, hipMemcpy(p.tq.d_tiles, tq.data(), tq.size() * sizeof(Tile), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(p.pq.d_tiles, pq.data(), pq.size() * sizeof(Tile), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(p.d_ctrl, lens, sizeof(lens), hipMemcpyHostToDevice));
    p.tq.nq = p.pq.nq = nq;
    p.tq.ntiles = (int64_t)ttiles.size();
    p.pq.ntiles = (int64_t)ptiles.size();
    p.out_samples = out_end;
    return PISCO_OK;
}

// The surrogate epilogue of detector state d writing from output sample `off`.
SlApply sl_apply_of(const DetState &d, const double *th, const double *ph, const double *ps, int64_t n, int64_t off) {
    SlApply a{};
    a.net = d.sl->net;
    a.th = th;
    a.ph = ph;
    a.ps = ps;
    a.n = n;
    a.out_offset = off;
    for (int k = 0; k < 3; ++k) {
        a.mean[k] = d.sl->mean[k];
        a.stdv[k] = d.sl->stdv[k];
    }
    sidelobe_coef(d, a.coef);
    return a;
}

// Build and upload the plan for `det` (-1 = all ready detectors) and output mode.
pisco_status prepare_plan(pisco_ctx *c, Plan &p, int32_t det, int out_mode) {
    const int32_t sub = out_mode == PISCO_OUT_TOD ? 1 : 0;
    if (p.gen == c->generation && p.det == det && p.spt == c->spt && p.xq == c->xq && p.algo == c->algo &&
        p.coherence == c->coherence && p.sub == sub)
        return PISCO_OK;
    std::vector<DetDesc> descs;
    std::vector<int32_t> det_of;   // detector index of each descriptor
    p.sl.clear();
    int64_t out_off = 0;
    const int32_t lo = det < 0 ? 0 : det, hi = det < 0 ? (int32_t)c->dets.size() - 1 : det;
    for (int32_t k = lo; k <= hi; ++k) {
        const DetState &d = c->dets[k];
        if (!det_ready(d)) continue;
        const bool sl = sub && d.sl_on && d.sl;
        DetDesc x = make_desc(d, sl);
        x.theta = d.th;
        x.phi = d.ph;
        x.psi = d.ps;
        x.out_offset = out_off;
        if (sl) p.sl.push_back(sl_apply_of(d, d.th, d.ph, d.ps, d.nsamp, out_off));
        descs.push_back(x);
        det_of.push_back(k);
        out_off += d.nsamp;
        p.beam_kind = d.beam_kind;
    }
    const pisco_status st = build_plan(c, p, descs, det_of, true);
    if (st != PISCO_OK) return st;
    p.gen = c->generation;
    p.det = det;
    p.spt = c->spt;
    p.xq = c->xq;
    p.algo = c->algo;
    p.coherence = c->coherence;
    p.sub = sub;
    return PISCO_OK;
}

ConvArgs make_args(pisco_ctx *c, const Plan &p, void *out, int out_mode, bool tile) {
    ConvArgs a{};
    const Queues &q = tile ? p.tq : p.pq;
    a.sky = c->sky;
    a.dets = p.d_dets;
    a.tiles = q.d_tiles;
    a.counters = p.d_ctrl + (tile ? 0 : 16);
    a.queue_len = p.d_ctrl + (tile ? 8 : 24);
    a.out = out;
    a.nside = c->nside;
    a.n_queues = q.nq;
    a.tiles_per_queue = q.per;
    a.out_mode = out_mode;
    a.beam_kind = p.beam_kind;
    a.algo = tile ? ((c->algo == PISCO_ALGO_TILE_MX && !p.extended) ? pisco::ALGO_TILE_MX : pisco::ALGO_TILE)
                  : pisco::ALGO_PIXEL;
    a.chunk = c->chunk;
    a.coherence = c->coherence;
    a.per_sample = p.per_sample;
    a.hwp = p.hwp;
    a.vbeam = p.vbeam;
    return a;
}

hipError_t enqueue(pisco_ctx *c, const Plan &p, void *out, int out_mode, hipStream_t s) {
    hipError_t e = pisco::launch_zero_counters(p.d_ctrl, 32, s);
    if (e != hipSuccess) return e;
    const bool f64 = c->sky_dtype == PISCO_F64;
    if (p.tq.ntiles > 0) {
        e = pisco::launch_conv(make_args(c, p, out, out_mode, true), f64, c->wpg, c->gpc * c->num_cu, s);
        if (e != hipSuccess) return e;
    }
    if (p.pq.ntiles > 0) {
        // no more workgroups than the pixel path has tiles for (a wave takes a tile)
        const int64_t g = std::min<int64_t>((int64_t)c->gpc * c->num_cu, (p.pq.ntiles + c->wpg - 1) / c->wpg);
        e = pisco::launch_conv(make_args(c, p, out, out_mode, false), f64, c->wpg, (int)std::max<int64_t>(1, g), s);
        if (e != hipSuccess) return e;
    }
    // far-sidelobe network of surrogate-enabled detectors, added to their TOD
    for (const SlApply &a : p.sl) {
        e = pisco::mlp_apply_pointing(a.net, a.th, a.ph, a.ps, a.n, a.mean, a.stdv, a.coef,
                                      static_cast<float *>(out) + a.out_offset, s);
        if (e != hipSuccess) return e;
    }
    return e;
}

}  // namespace

namespace pisco {
void set_error(pisco_ctx *c, const char *msg) {
    if (c) c->err = msg;
}
int ctx_device(const pisco_ctx *c) { return c->device; }
int ctx_num_cu(const pisco_ctx *c) { return c->num_cu; }
bool ctx_pointing(const pisco_ctx *c, int32_t det, const double **th, const double **ph, const double **ps,
                  int64_t *n) {
    if (det < 0 || (size_t)det >= c->dets.size() || !c->dets[det].has_pointing) return false;
    const DetState &d = c->dets[det];
    if (d.nsamp > 0 && !d.th) return false;  // kept on the host (memory budget)
    *th = d.th;
    *ph = d.ph;
    *ps = d.ps;
    *n = d.nsamp;
    return true;
}
}  // namespace pisco

extern "C" {

int pisco_abi_version(void) { return 100; }

pisco_status pisco_create(int device, pisco_ctx **out) {
    if (!out) return PISCO_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PISCO_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PISCO_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PISCO_EUNSUPPORTED;
    if (hipSetDevice(device) != hipSuccess) return PISCO_EDEVICE;
    pisco_ctx *c = new pisco_ctx();
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    // the device address of the allocation-free entry point's plan array
    if (pisco::static_scratch_init(device) != hipSuccess) {
        delete c;
        return PISCO_EDEVICE;
    }
    if (!dmalloc(c, reinterpret_cast<void **>(&c->d_flag), sizeof(int32_t))) {
        delete c;
        return PISCO_ENOMEM;
    }
    *out = c;
    return PISCO_OK;
}

void pisco_destroy(pisco_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &p : c->plans) free_plan(c, p);
    for (auto &t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (size_t k = 0; k < c->dets.size(); ++k) {
        release_beam(c, (int32_t)k);
        release_pointing(c, c->dets[k]);
        release_hwp(c, c->dets[k]);
        release_sidelobe(c->dets[k]);
    }
    if (c->sky && c->sky_owned) dfree(c, c->sky);
    dfree(c, c->d_flag);
    delete c;
}

const char *pisco_last_error(const pisco_ctx *c) { return c ? c->err.c_str() : "null context"; }

pisco_status pisco_set_sky(pisco_ctx *c, int64_t nside, const void *I, const void *Q, const void *U, int dtype,
                           int mem) {
    return pisco_set_sky_iquv(c, nside, I, Q, U, nullptr, dtype, mem);
}

pisco_status pisco_set_sky_iquv(pisco_ctx *c, int64_t nside, const void *I, const void *Q, const void *U,
                                const void *V, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (!is_pow2(nside) || nside > PISCO_MAX_NSIDE) return fail(c, PISCO_EINVAL, "nside %lld is not a power of two in [1, %d]", (long long)nside, PISCO_MAX_NSIDE);
    if (dtype != PISCO_F32 && dtype != PISCO_F64) return fail(c, PISCO_EINVAL, "bad dtype %d", dtype);
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    if (!I || !Q || !U) return fail(c, PISCO_EINVAL, "null map");
    HIP_TRY(c, hipSetDevice(c->device));
    void *rec = nullptr;
    const pisco_status st = interleave(c, I, Q, U, V, 12 * nside * nside, dtype, mem, &rec);
    if (st != PISCO_OK) return st;
    HIP_TRY(c, hipDeviceSynchronize());
    if (c->sky && c->sky_owned) dfree(c, c->sky);
    c->sky = rec;
    c->sky_owned = true;
    c->nside = nside;
    c->sky_dtype = dtype;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_beam(pisco_ctx *c, int32_t det, int32_t n, double T, const void *bI, const void *bQ,
                            const void *bU, const void *bT, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (n < 3 || n > 4095 || (n % 2) == 0) return fail(c, PISCO_EINVAL, "grid size %d must be odd in [3, 4095]", n);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, PISCO_EINVAL, "half_span_tan must be finite and > 0");
    if (dtype != PISCO_F32 && dtype != PISCO_F64) return fail(c, PISCO_EINVAL, "bad dtype %d", dtype);
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    if (!bI || !bQ || !bU || !bT) return fail(c, PISCO_EINVAL, "null beam channel");
    HIP_TRY(c, hipSetDevice(c->device));
    void *rec = nullptr;
    const pisco_status st = interleave(c, bI, bQ, bU, bT, (int64_t)n * n, dtype, mem, &rec);
    if (st != PISCO_OK) return st;
    HIP_TRY(c, hipDeviceSynchronize());
    release_beam(c, det);
    d = &c->dets[det];
    d->beam = rec;
    d->beam_owned = true;
    d->n = n;
    d->T = T;
    d->beam_dtype = dtype;
    d->beam_kind = pisco::BEAM_FULL;
    for (int i = 0; i < 4; ++i) d->w[i] = 1.0;
    d->has_beam = true;
    ++c->generation;
    return PISCO_OK;
}

// HEALPix beam maps resampled onto a temporary n x n node grid (device arrays
// the caller frees), then uploaded like a node grid.
static pisco_status healpix_nodes(pisco_ctx *c, int64_t nside_b, const void *const *maps, int nch, int32_t n,
                                  double T, int dtype, int mem, void **nodes) {
    if (nside_b < 1 || nside_b > 8192 || !is_pow2(nside_b))
        return fail(c, PISCO_EINVAL, "beam nside %lld must be a power of two in [1, 8192]", (long long)nside_b);
    if (n < 3 || n > 4095 || (n % 2) == 0) return fail(c, PISCO_EINVAL, "grid size %d must be odd in [3, 4095]", n);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, PISCO_EINVAL, "half_span_tan must be finite and > 0");
    if (dtype != PISCO_F32 && dtype != PISCO_F64) return fail(c, PISCO_EINVAL, "bad dtype %d", dtype);
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    for (int k = 0; k < nch; ++k)
        if (!maps[k]) return fail(c, PISCO_EINVAL, "null beam map");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t mbytes = el_bytes(dtype) * (size_t)(12 * nside_b * nside_b);
    const size_t nbytes = el_bytes(dtype) * (size_t)n * (size_t)n;
    pisco::HpxGridArgs a{};
    a.nside = (int32_t)nside_b;
    a.n = n;
    a.nch = nch;
    a.T = T;
    void *staged[4] = {nullptr, nullptr, nullptr, nullptr};
    pisco_status st = PISCO_OK;
    for (int k = 0; k < nch && st == PISCO_OK; ++k) {
        nodes[k] = nullptr;
        if (mem == PISCO_HOST) st = to_device(c, maps[k], mbytes, PISCO_HOST, &staged[k]);
        a.map[k] = mem == PISCO_HOST ? staged[k] : maps[k];
        if (st == PISCO_OK && !dmalloc(c, &nodes[k], nbytes))
            st = fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", nbytes);
        a.out[k] = nodes[k];
    }
    if (st == PISCO_OK) {
        hipError_t e = pisco::launch_healpix_grid(a, dtype == PISCO_F64, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) st = fail(c, PISCO_EDEVICE, "beam map resampling failed: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < nch; ++k)
        dfree(c, staged[k]);
    if (st != PISCO_OK)
        for (int k = 0; k < nch; ++k)
            if (nodes[k]) {
                dfree(c, nodes[k]);
                nodes[k] = nullptr;
            }
    return st;
}

pisco_status pisco_set_beam_healpix(pisco_ctx *c, int32_t det, int64_t nside_beam, const void *bI, const void *bQ,
                                    const void *bU, const void *bT, int32_t n, double T, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (!det_slot(c, det)) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    const void *maps[4] = {bI, bQ, bU, bT};
    void *nodes[4] = {nullptr, nullptr, nullptr, nullptr};
    pisco_status st = healpix_nodes(c, nside_beam, maps, 4, n, T, dtype, mem, nodes);
    if (st != PISCO_OK) return st;
    st = pisco_set_beam(c, det, n, T, nodes[0], nodes[1], nodes[2], nodes[3], dtype, PISCO_DEVICE);
    for (int k = 0; k < 4; ++k) dfree(c, nodes[k]);
    return st;
}

pisco_status pisco_set_beam_healpix_scalar(pisco_ctx *c, int32_t det, int64_t nside_beam, const void *b, double wI,
                                           double wQ, double wU, double wT, int32_t n, double T, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (!det_slot(c, det)) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    const void *maps[1] = {b};
    void *nodes[1] = {nullptr};
    pisco_status st = healpix_nodes(c, nside_beam, maps, 1, n, T, dtype, mem, nodes);
    if (st != PISCO_OK) return st;
    st = pisco_set_beam_scalar(c, det, n, T, nodes[0], wI, wQ, wU, wT, dtype, PISCO_DEVICE);
    dfree(c, nodes[0]);
    return st;
}

pisco_status pisco_set_beam_scalar(pisco_ctx *c, int32_t det, int32_t n, double T, const void *b, double wI,
                                   double wQ, double wU, double wT, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (n < 3 || n > 4095 || (n % 2) == 0) return fail(c, PISCO_EINVAL, "grid size %d must be odd in [3, 4095]", n);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, PISCO_EINVAL, "half_span_tan must be finite and > 0");
    if (!std::isfinite(wI) || !std::isfinite(wQ) || !std::isfinite(wU) || !std::isfinite(wT))
        return fail(c, PISCO_EINVAL, "non-finite beam weight");
    if (dtype != PISCO_F32 && dtype != PISCO_F64) return fail(c, PISCO_EINVAL, "bad dtype %d", dtype);
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    if (!b) return fail(c, PISCO_EINVAL, "null beam");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t nodes = (size_t)n * n, cells = (size_t)(n + 1) * (n + 1);   // grid cells + extrapolated ring
    void *src = nullptr;
    pisco_status st = PISCO_OK;
    if (mem == PISCO_DEVICE) src = const_cast<void *>(b);
    else st = to_device(c, b, el_bytes(dtype) * nodes, PISCO_HOST, &src);
    if (st != PISCO_OK) return st;
    void *rec = nullptr;
    if (!dmalloc(c, &rec, rec_bytes(dtype) * cells)) {
        if (mem == PISCO_HOST) dfree(c, src);
        return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", rec_bytes(dtype) * cells);
    }
    hipError_t e = pisco::launch_repack_cells(src, n, rec, dtype == PISCO_F64, true, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (mem == PISCO_HOST) dfree(c, src);
    if (e != hipSuccess) {
        dfree(c, rec);
        return fail(c, PISCO_EDEVICE, "beam repack failed: %s", hipGetErrorString(e));
    }
    release_beam(c, det);
    d = &c->dets[det];
    d->beam = rec;
    d->beam_owned = true;
    d->n = n;
    d->T = T;
    d->beam_dtype = dtype;
    d->beam_kind = pisco::BEAM_SCALAR;
    d->w[0] = wI;
    d->w[1] = wQ;
    d->w[2] = wU;
    d->w[3] = wT;
    d->has_beam = true;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_share_beam(pisco_ctx *c, int32_t det, int32_t src) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (src < 0 || (size_t)src >= c->dets.size() || !c->dets[src].has_beam || !c->dets[src].beam_owned)
        return fail(c, PISCO_EINVAL, "detector %d has no beam of its own to share", src);
    if (det == src) return PISCO_OK;
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    HIP_TRY(c, hipDeviceSynchronize());
    release_beam(c, det);
    d = &c->dets[det];
    const DetState &s = c->dets[src];
    d->beam = s.beam;
    d->beam_owned = false;
    d->n = s.n;
    d->T = s.T;
    d->beam_dtype = s.beam_dtype;
    d->beam_kind = s.beam_kind;
    for (int i = 0; i < 4; ++i) d->w[i] = s.w[i];
    d->beam_v = s.beam_v;
    d->wv = s.wv;
    d->has_beam = true;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_beam_v(pisco_ctx *c, int32_t det, int32_t n, double T, const void *bI, const void *bQ,
                              const void *bU, const void *bV, const void *bT, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    if (!bV) return pisco_set_beam(c, det, n, T, bI, bQ, bU, bT, dtype, mem);
    pisco_status st = pisco_set_beam(c, det, n, T, bI, bQ, bU, bT, dtype, mem);
    if (st != PISCO_OK) return st;
    const size_t nodes = (size_t)n * n, cells = (size_t)(n - 1) * (n - 1);
    void *src = nullptr;
    if (mem == PISCO_DEVICE) src = const_cast<void *>(bV);
    else if ((st = to_device(c, bV, el_bytes(dtype) * nodes, PISCO_HOST, &src)) != PISCO_OK) return st;
    void *rec = nullptr;
    if (!dmalloc(c, &rec, rec_bytes(dtype) * cells)) {
        if (mem == PISCO_HOST) dfree(c, src);
        return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", rec_bytes(dtype) * cells);
    }
    hipError_t e = pisco::launch_repack_cells(src, n, rec, dtype == PISCO_F64, false, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (mem == PISCO_HOST) dfree(c, src);
    if (e != hipSuccess) {
        dfree(c, rec);
        return fail(c, PISCO_EDEVICE, "beam repack failed: %s", hipGetErrorString(e));
    }
    c->dets[det].beam_v = rec;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_beam_scalar_v(pisco_ctx *c, int32_t det, int32_t n, double T, const void *b, double wI,
                                     double wQ, double wU, double wV, double wT, int dtype, int mem) {
    if (!c) return PISCO_EINVAL;
    if (!std::isfinite(wV)) return fail(c, PISCO_EINVAL, "non-finite beam weight");
    const pisco_status st = pisco_set_beam_scalar(c, det, n, T, b, wI, wQ, wU, wT, dtype, mem);
    if (st != PISCO_OK) return st;
    c->dets[det].wv = wV;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_hwp(pisco_ctx *c, int32_t det, int64_t n, const double *angle, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(c, PISCO_EINVAL, "bad sample count");
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    if (!angle || n == 0) {
        release_hwp(c, *d);
        ++c->generation;
        return PISCO_OK;
    }
    if (mem == PISCO_HOST) {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(angle[i])) return fail(c, PISCO_EINVAL, "plate angle %lld is not finite", (long long)i);
        release_hwp(c, *d);
        void *buf = nullptr;
        if (dmalloc(c, &buf, sizeof(double) * (size_t)n)) {
            const hipError_t e = hipMemcpy(buf, angle, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                dfree(c, buf);
                return fail(c, PISCO_EDEVICE, "plate-angle copy failed: %s", hipGetErrorString(e));
            }
            d->owned_hwp = static_cast<double *>(buf);
            d->hwp = d->owned_hwp;
        } else {
            // over the memory budget: keep the angles on the host, streamed in blocks by convolve
            d->host_hwp.assign(angle, angle + n);
        }
    } else {
        release_hwp(c, *d);
        d->hwp = angle;
    }
    d->hwp_n = n;
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_detector(pisco_ctx *c, int32_t det, double zeta, double rho_min, double rho_max,
                                int norm_mode, double norm_scale) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (!std::isfinite(zeta) || !std::isfinite(norm_scale)) return fail(c, PISCO_EINVAL, "non-finite parameter");
    if (!(rho_min >= 0.0) || !(rho_max > rho_min) || !(rho_max < 0.5 * M_PI))
        return fail(c, PISCO_EINVAL, "need 0 <= rho_min < rho_max < pi/2 (got %g, %g)", rho_min, rho_max);
    if (norm_mode != PISCO_NORM_FIXED && norm_mode != PISCO_NORM_PER_SAMPLE)
        return fail(c, PISCO_EINVAL, "bad norm_mode %d", norm_mode);
    d->zeta = zeta;
    d->rho_min = rho_min;
    d->rho_max = rho_max;
    d->norm_mode = norm_mode;
    d->norm_scale = norm_scale;
    d->has_params = true;
    release_sidelobe(*d);
    ++c->generation;
    return PISCO_OK;
}

pisco_status pisco_set_pointing(pisco_ctx *c, int32_t det, int64_t n, const double *theta, const double *phi,
                                const double *psi, int mem) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    DetState *d = det_slot(c, det);
    if (!d) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(c, PISCO_EINVAL, "bad sample count");
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    if (n > 0 && (!theta || !phi || !psi)) return fail(c, PISCO_EINVAL, "null pointing array");
    HIP_TRY(c, hipSetDevice(c->device));
    if (mem == PISCO_HOST) {
        for (int64_t i = 0; i < n; ++i) {
            const double t = theta[i];
            if (!std::isfinite(t) || t < 0.0 || t > M_PI || !std::isfinite(phi[i]) || !std::isfinite(psi[i]))
                return fail(c, PISCO_EINVAL, "pointing sample %lld is non-finite or has theta outside [0, pi]", (long long)i);
        }
        HIP_TRY(c, hipDeviceSynchronize());
        release_pointing(c, *d);
        void *vb = nullptr;
        if (n > 0 && dmalloc(c, &vb, 3 * sizeof(double) * (size_t)n)) {
            double *buf = static_cast<double *>(vb);
            const size_t b = sizeof(double) * (size_t)n;
            hipError_t e = hipMemcpy(buf, theta, b, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(buf + n, phi, b, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(buf + 2 * n, psi, b, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                dfree(c, buf);
                d->has_pointing = false;
                d->nsamp = 0;
                ++c->generation;
                return fail(c, PISCO_EDEVICE, "pointing copy failed: %s", hipGetErrorString(e));
            }
            d->owned_pointing = buf;
            d->th = buf;
            d->ph = buf + n;
            d->ps = buf + 2 * n;
        } else if (n > 0) {
            // over the memory budget: keep the pointing on the host, streamed in blocks by convolve
            d->host_pointing.resize(3 * (size_t)n);
            std::memcpy(d->host_pointing.data(), theta, sizeof(double) * (size_t)n);
            std::memcpy(d->host_pointing.data() + n, phi, sizeof(double) * (size_t)n);
            std::memcpy(d->host_pointing.data() + 2 * n, psi, sizeof(double) * (size_t)n);
        }
    } else {
        if (n > 0) {
            HIP_TRY(c, hipMemset(c->d_flag, 0, sizeof(int32_t)));
            HIP_TRY(c, pisco::launch_check_pointing(theta, phi, psi, n, c->d_flag, nullptr));
            int32_t bad = 0;
            HIP_TRY(c, hipMemcpy(&bad, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost));
            if (bad) return fail(c, PISCO_EINVAL, "pointing holds non-finite values or theta outside [0, pi]");
        }
        HIP_TRY(c, hipDeviceSynchronize());
        release_pointing(c, *d);
        d->th = theta;
        d->ph = phi;
        d->ps = psi;
    }
    d->nsamp = n;
    d->has_pointing = true;
    ++c->generation;
    return PISCO_OK;
}

int64_t pisco_output_samples(const pisco_ctx *c, int32_t det) {
    if (!c) return -1;
    if (det >= 0) return ((size_t)det < c->dets.size() && det_ready(c->dets[det])) ? c->dets[det].nsamp : 0;
    int64_t s = 0;
    for (const auto &d : c->dets)
        if (det_ready(d)) s += d.nsamp;
    return s;
}

}  // extern "C"

namespace {

// The budgeted path: every ready detector of [lo, hi] streamed in blocks of
// consecutive samples (multiples of 64) through device buffers that fit the
// remaining budget, block after block on stream s.
pisco_status convolve_blocks(pisco_ctx *c, int32_t det, int out_mode, void *out, int mem, hipStream_t s) {
    const size_t el = el_bytes(c->sky_dtype) * (out_mode == PISCO_OUT_STOKES ? 3 : 1);  // bytes per output sample
    const int32_t lo = det < 0 ? 0 : det, hi = det < 0 ? (int32_t)c->dets.size() - 1 : det;
    // the resident plans' buffers make room for the blocks
    for (int i = 0; i < 2; ++i) free_plan(c, c->plans[i]);
    Plan &p = c->plans[2];
    const bool sub = out_mode == PISCO_OUT_TOD;
    int64_t out_base = 0;
    for (int32_t k = lo; k <= hi; ++k) {
        const DetState &d = c->dets[k];
        if (!det_ready(d)) continue;
        const int64_t n = d.nsamp;
        const bool hp = !d.host_pointing.empty(), hh = !d.host_hwp.empty();
        const bool sl = sub && d.sl_on && d.sl;
        // device bytes per sample of a block: staged pointing, plate angles and
        // output, and the queues (tile entries and classification flags of its
        // 64-sample groups); a fixed part for the descriptor and control block
        const int64_t per = (hp ? 24 : 0) + (hh ? 8 : 0) + (mem == PISCO_HOST ? (int64_t)el : 0) + 2;
        const int64_t fixed = 8192;
        const int64_t room = c->budget > 0 ? c->budget - c->in_use - fixed : ((int64_t)1 << 50);
        int64_t C = room > 0 ? room / per : 0;
        C = std::min<int64_t>(C, ((n + 63) / 64) * 64);
        C = (C / 64) * 64;
        void *bp = nullptr, *bh = nullptr, *bo = nullptr;
        for (;;) {
            if (C < 64) {
                free_plan(c, p);
                return fail(c, PISCO_ENOMEM, "detector %d: the device memory budget (%lld bytes, %lld in use) leaves "
                            "no room for a 64-sample block", k, (long long)c->budget, (long long)c->in_use);
            }
            const bool ok = (!hp || dmalloc(c, &bp, 24 * (size_t)C)) && (!hh || dmalloc(c, &bh, 8 * (size_t)C)) &&
                            (mem != PISCO_HOST || dmalloc(c, &bo, el * (size_t)C));
            if (ok) break;
            dfree(c, bp);
            dfree(c, bh);
            dfree(c, bo);
            bp = bh = bo = nullptr;
            C = ((C / 2) / 64) * 64;
        }
        auto release = [&]() {
            dfree(c, bp);
            dfree(c, bh);
            dfree(c, bo);
        };
        for (int64_t b = 0; b < n; b += C) {
            const int64_t m = std::min(C, n - b);
            const double *th = d.th ? d.th + b : nullptr, *ph = d.ph ? d.ph + b : nullptr,
                         *ps = d.ps ? d.ps + b : nullptr, *hw = d.hwp ? d.hwp + b : nullptr;
            hipError_t e = hipSuccess;
            if (hp) {
                double *q = static_cast<double *>(bp);
                const size_t bytes = sizeof(double) * (size_t)m;
                e = hipMemcpy(q, d.host_pointing.data() + b, bytes, hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(q + C, d.host_pointing.data() + n + b, bytes, hipMemcpyHostToDevice);
                if (e == hipSuccess)
                    e = hipMemcpy(q + 2 * C, d.host_pointing.data() + 2 * n + b, bytes, hipMemcpyHostToDevice);
                th = q;
                ph = q + C;
                ps = q + 2 * C;
            }
            if (hh && e == hipSuccess) {
                e = hipMemcpy(bh, d.host_hwp.data() + b, sizeof(double) * (size_t)m, hipMemcpyHostToDevice);
                hw = static_cast<const double *>(bh);
            }
            if (e != hipSuccess) {
                release();
                return fail(c, PISCO_EDEVICE, "block upload failed: %s", hipGetErrorString(e));
            }
            DetDesc x = make_desc(d, sl);
            x.theta = th;
            x.phi = ph;
            x.psi = ps;
            x.hwp = hw;
            x.n_samples = m;
            x.out_offset = 0;
            std::vector<DetDesc> descs{x};
            const std::vector<int32_t> det_of{k};
            p.beam_kind = d.beam_kind;
            p.sl.clear();
            if (sl) p.sl.push_back(sl_apply_of(d, th, ph, ps, m, 0));
            const pisco_status st = build_plan(c, p, descs, det_of, false);
            if (st != PISCO_OK) {
                release();
                return st;
            }
            void *o = mem == PISCO_HOST ? bo : static_cast<void *>(static_cast<char *>(out) + (out_base + b) * el);
            e = enqueue(c, p, o, out_mode, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);   // the staging buffers are reused by the next block
            if (e == hipSuccess && mem == PISCO_HOST)
                e = hipMemcpy(static_cast<char *>(out) + (out_base + b) * el, bo, el * (size_t)m,
                              hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                release();
                return fail(c, PISCO_EDEVICE, "block convolution failed: %s", hipGetErrorString(e));
            }
        }
        release();
        out_base += n;
    }
    free_plan(c, p);
    return PISCO_OK;
}

}  // namespace

extern "C" {

pisco_status pisco_convolve(pisco_ctx *c, int32_t det, int out_mode, void *out, int mem, void *stream) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (!c->sky) return fail(c, PISCO_ESTATE, "no sky set");
    if (out_mode != PISCO_OUT_TOD && out_mode != PISCO_OUT_STOKES && out_mode != PISCO_OUT_COUNT)
        return fail(c, PISCO_EINVAL, "bad out_mode %d", out_mode);
    if (mem != PISCO_HOST && mem != PISCO_DEVICE) return fail(c, PISCO_EINVAL, "bad mem %d", mem);
    if (det < -1) return fail(c, PISCO_EINVAL, "bad detector %d", det);
    if (det >= 0) {
        if ((size_t)det >= c->dets.size() || !det_ready(c->dets[det]))
            return fail(c, PISCO_ESTATE, "detector %d lacks a beam, parameters or pointing", det);
    }
    bool any = false, host_resident = false;
    int first_kind = -1;
    int64_t nall = 0;
    const int32_t lo = det < 0 ? 0 : det, hi = det < 0 ? (int32_t)c->dets.size() - 1 : det;
    for (int32_t k = lo; k <= hi; ++k) {
        const DetState &d = c->dets[k];
        if (!det_ready(d)) continue;
        any = true;
        nall += d.nsamp;
        if (d.beam_dtype != c->sky_dtype)
            return fail(c, PISCO_EINVAL, "detector %d beam dtype differs from the sky dtype", k);
        if ((d.hwp || !d.host_hwp.empty()) && d.hwp_n != d.nsamp)
            return fail(c, PISCO_EINVAL, "detector %d has %lld plate angles for %lld samples", k, (long long)d.hwp_n,
                        (long long)d.nsamp);
        // a V column adds 4 bytes of LDS per staged record and wave on the tile path
        if (d.beam_v && c->algo != PISCO_ALGO_PIXEL && out_mode == PISCO_OUT_TOD &&
            (size_t)c->wpg * (4352 + std::max<size_t>(3840, 48 * (size_t)c->chunk) + 4 * (size_t)c->chunk) >
                160 * 1024)
            return fail(c, PISCO_EINVAL, "detector %d: a V-column beam needs more LDS than chunk %d with %d waves "
                        "per group leaves; use a smaller chunk or fewer waves", k, c->chunk, c->wpg);
        if (d.sl_on && out_mode == PISCO_OUT_TOD && c->sky_dtype != PISCO_F32)
            return fail(c, PISCO_EINVAL, "detector %d: the sidelobe network runs on the FP32 path only", k);
        if (first_kind < 0) first_kind = d.beam_kind;
        if (d.beam_kind != first_kind)
            return fail(c, PISCO_EINVAL, "detectors in one launch must all have full or all scalar beams");
        if (!d.host_pointing.empty() || !d.host_hwp.empty()) host_resident = true;
    }
    if (!any) return fail(c, PISCO_ESTATE, "no detector is ready");
    if (nall > 0 && !out) return fail(c, PISCO_EINVAL, "null output");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (mem == PISCO_HOST) s = nullptr;
    TimedLaunch tl{};
    auto timing_start = [&]() -> pisco_status {
        if (c->timing) {
            HIP_TRY(c, hipEventCreate(&tl.a));
            HIP_TRY(c, hipEventCreate(&tl.b));
            HIP_TRY(c, hipEventRecord(tl.a, s));
        }
        return PISCO_OK;
    };
    auto timing_end = [&]() -> pisco_status {
        if (c->timing) {
            HIP_TRY(c, hipEventRecord(tl.b, s));
            c->pending.push_back(tl);
        }
        return PISCO_OK;
    };
    auto blocks = [&]() -> pisco_status {
        pisco_status st = timing_start();
        if (st == PISCO_OK) st = convolve_blocks(c, det, out_mode, out, mem, s);
        if (st == PISCO_OK) st = timing_end();
        return st;
    };
    if (host_resident) return blocks();
    Plan &p = c->plans[det < 0 ? 0 : 1];
    pisco_status st = prepare_plan(c, p, det, out_mode);
    if (st == PISCO_ENOMEM) {  // the work queues do not fit: run in blocks
        c->err.clear();
        return blocks();
    }
    if (st != PISCO_OK) return st;
    const int64_t nout = p.out_samples * (out_mode == PISCO_OUT_STOKES ? 3 : 1);
    if (nout == 0) return PISCO_OK;
    void *dout = out;
    if (mem == PISCO_HOST && !dmalloc(c, &dout, el_bytes(c->sky_dtype) * (size_t)nout)) return blocks();
    st = timing_start();
    if (st != PISCO_OK) {
        if (mem == PISCO_HOST) dfree(c, dout);
        return st;
    }
    hipError_t e = hipSuccess;
    const bool use_graph = (det < 0) && (s != nullptr);
    if (use_graph) {
        if (!p.gexec || p.g_gen != p.gen || p.g_out != dout || p.g_stream != s || p.g_mode != out_mode ||
            p.g_wpg != c->wpg || p.g_gpc != c->gpc || p.g_chunk != c->chunk) {
            drop_graph(p);
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t e1 = enqueue(c, p, dout, out_mode, s);
                e = hipStreamEndCapture(s, &g);
                if (e1 != hipSuccess) e = e1;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&p.gexec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e == hipSuccess) {
                p.g_gen = p.gen;
                p.g_out = dout;
                p.g_stream = s;
                p.g_mode = out_mode;
                p.g_wpg = c->wpg;
                p.g_gpc = c->gpc;
                p.g_chunk = c->chunk;
            } else {
                p.gexec = nullptr;
            }
        }
        if (e == hipSuccess) e = hipGraphLaunch(p.gexec, s);
    } else {
        e = enqueue(c, p, dout, out_mode, s);
    }
    if (e != hipSuccess) {
        if (mem == PISCO_HOST) dfree(c, dout);
        return fail(c, PISCO_EDEVICE, "convolution launch failed: %s", hipGetErrorString(e));
    }
    st = timing_end();
    if (mem == PISCO_HOST) {
        e = hipMemcpy(out, dout, el_bytes(c->sky_dtype) * (size_t)nout, hipMemcpyDeviceToHost);
        dfree(c, dout);
        if (e != hipSuccess) return fail(c, PISCO_EDEVICE, "output copy failed: %s", hipGetErrorString(e));
    }
    return st;
}

pisco_status pisco_set_ordering(pisco_ctx *c, int32_t mode) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (mode != PISCO_ORDER_GIVEN && mode != PISCO_ORDER_AUTO && mode != PISCO_ORDER_SPATIAL)
        return fail(c, PISCO_EINVAL, "bad ordering mode %d", mode);
    if (mode != c->ordering) {
        c->ordering = mode;
        ++c->generation;
    }
    return PISCO_OK;
}

pisco_status pisco_set_launch(pisco_ctx *c, const pisco_launch *l) {
    if (!c || !l) return PISCO_EINVAL;
    c->err.clear();
    if (l->algorithm != PISCO_ALGO_PIXEL && l->algorithm != PISCO_ALGO_TILE && l->algorithm != PISCO_ALGO_TILE_MX)
        return fail(c, PISCO_EINVAL, "bad algorithm %d", l->algorithm);
    if (l->samples_per_tile < 1 || l->samples_per_tile > 65536) return fail(c, PISCO_EINVAL, "samples_per_tile out of range");
    const int w = l->waves_per_group;
    if (w != 1 && w != 2 && w != 4 && w != 8) return fail(c, PISCO_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
    if (l->groups_per_cu < 1 || l->groups_per_cu > 16) return fail(c, PISCO_EINVAL, "groups_per_cu out of range");
    if (l->xcd_queues != 1 && l->xcd_queues != 8) return fail(c, PISCO_EINVAL, "xcd_queues must be 1 or 8");
    if (l->chunk != 64 && l->chunk != 128 && l->chunk != 256) return fail(c, PISCO_EINVAL, "chunk must be 64, 128 or 256");
    if (!(l->coherence > 0.0 && l->coherence <= 4.0)) return fail(c, PISCO_EINVAL, "coherence must be in (0, 4]");
    // LDS per workgroup must fit the 160 KiB of a compute unit
    // LDS per wave: rings, frames and segment ends, the staged records and, on
    // the matrix-core path, the running sums of TOD launches (Stokes launches
    // split workgroups that would not fit)
    // (tile path: the lane frames share storage with the staged records)
    const size_t tile_slice = l->algorithm == PISCO_ALGO_TILE_MX
                                  ? 64 * 64 + 64 * 60 + 64 * 4 + (size_t)l->chunk * 64 + 4 * 4 * 64 * 4
                                  : 64 * 64 + 64 * 4 + std::max<size_t>(64 * 60, (size_t)l->chunk * 48);
    if (l->algorithm != PISCO_ALGO_PIXEL && tile_slice * (size_t)w > 160 * 1024)
        return fail(c, PISCO_EINVAL, "chunk %d with %d waves per group exceeds the LDS of a compute unit", l->chunk, w);
    c->algo = l->algorithm;
    c->spt = l->samples_per_tile;
    c->wpg = w;
    c->gpc = l->groups_per_cu;
    c->xq = l->xcd_queues;
    c->chunk = l->chunk;
    c->coherence = l->coherence;
    return PISCO_OK;
}

pisco_status pisco_get_launch(const pisco_ctx *c, pisco_launch *l) {
    if (!c || !l) return PISCO_EINVAL;
    l->algorithm = c->algo;
    l->samples_per_tile = c->spt;
    l->waves_per_group = c->wpg;
    l->groups_per_cu = c->gpc;
    l->xcd_queues = c->xq;
    l->chunk = c->chunk;
    l->coherence = c->coherence;
    return PISCO_OK;
}

pisco_status pisco_set_timing(pisco_ctx *c, int on) {
    if (!c) return PISCO_EINVAL;
    c->timing = on != 0;
    return PISCO_OK;
}

pisco_status pisco_kernel_time(pisco_ctx *c, double *total_ms, int64_t *launches, int reset) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    for (auto &t : c->pending) {
        HIP_TRY(c, hipEventSynchronize(t.b));
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, t.a, t.b));
        c->total_ms += ms;
        c->launches += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    c->pending.clear();
    if (total_ms) *total_ms = c->total_ms;
    if (launches) *launches = c->launches;
    if (reset) {
        c->total_ms = 0.0;
        c->launches = 0;
    }
    return PISCO_OK;
}

pisco_status pisco_set_memory_budget(pisco_ctx *c, int64_t bytes) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (bytes < 0) return fail(c, PISCO_EINVAL, "memory budget must be >= 0");
    c->budget = bytes;
    return PISCO_OK;
}

int64_t pisco_memory_in_use(const pisco_ctx *c) { return c ? c->in_use : -1; }

pisco_status pisco_sidelobe_set_options(pisco_ctx *c, const pisco_sidelobe_opts *o) {
    if (!c || !o) return PISCO_EINVAL;
    c->err.clear();
    if (o->width < 64 || o->width > 512 || o->width % 64)
        return fail(c, PISCO_EINVAL, "width must be a multiple of 64 in [64, 512]");
    if (o->hidden_layers < 1 || o->hidden_layers > 16) return fail(c, PISCO_EINVAL, "hidden_layers must be in [1, 16]");
    if (o->batch < 64 || o->batch > (1 << 22) || o->batch % 64)
        return fail(c, PISCO_EINVAL, "batch must be a multiple of 64 in [64, 4194304]");
    if (!(o->lr_end > 0.0f) || !(o->lr >= o->lr_end) || !std::isfinite(o->lr))
        return fail(c, PISCO_EINVAL, "need 0 < lr_end <= lr");
    if (!(o->beta1 >= 0.0f && o->beta1 < 1.0f) || !(o->beta2 >= 0.0f && o->beta2 < 1.0f) || !(o->eps > 0.0f))
        return fail(c, PISCO_EINVAL, "bad Adam hyper-parameters");
    c->sl_opts = *o;
    return PISCO_OK;
}

static pisco_status sidelobe_capable(pisco_ctx *c, int32_t det, const DetState &d);

pisco_status pisco_sidelobe_train(pisco_ctx *c, int32_t det, double r_main, int64_t n_train, uint64_t seed,
                                  int32_t epochs) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (det < 0 || det >= PISCO_MAX_DETECTORS) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (!c->sky) return fail(c, PISCO_ESTATE, "no sky set");
    if ((size_t)det >= c->dets.size() || !c->dets[det].has_beam || !c->dets[det].has_params)
        return fail(c, PISCO_ESTATE, "detector %d lacks a beam or parameters", det);
    DetState &d = c->dets[det];
    {
        const pisco_status cs = sidelobe_capable(c, det, d);
        if (cs != PISCO_OK) return cs;
    }
    if (!(r_main > d.rho_min) || !(r_main < d.rho_max))
        return fail(c, PISCO_EINVAL, "need rho_min < r_main < rho_max (got %g, disc %g..%g)", r_main, d.rho_min,
                    d.rho_max);
    if (n_train < c->sl_opts.batch || n_train > ((int64_t)1 << 31))
        return fail(c, PISCO_EINVAL, "n_train must be in [batch = %d, 2^31]", c->sl_opts.batch);
    if (epochs < 1) return fail(c, PISCO_EINVAL, "epochs must be >= 1");
    HIP_TRY(c, hipSetDevice(c->device));
    // the annulus (r_main, rho_max] at zeta = 0 on a context that borrows the sky and the beam
    pisco_ctx *t = nullptr;
    pisco_status st = pisco_create(c->device, &t);
    if (st != PISCO_OK) return fail(c, st, "target context creation failed");
    t->sky = c->sky;
    t->sky_owned = false;
    t->nside = c->nside;
    t->sky_dtype = c->sky_dtype;
    t->dets.resize(1);
    DetState &td = t->dets[0];
    td.beam = d.beam;
    td.beam_owned = false;
    td.n = d.n;
    td.T = d.T;
    td.beam_dtype = d.beam_dtype;
    td.beam_kind = d.beam_kind;
    for (int i = 0; i < 4; ++i) td.w[i] = d.w[i];
    td.has_beam = true;
    t->algo = c->algo;
    t->spt = c->spt;
    t->wpg = c->wpg;
    t->gpc = c->gpc;
    t->xq = c->xq;
    t->chunk = c->chunk;
    t->coherence = c->coherence;
    t->ordering = PISCO_ORDER_SPATIAL;  // isotropic pointings: tiles of spatially sorted samples
    st = pisco_set_detector(t, 0, 0.0, r_main, d.rho_max, PISCO_NORM_FIXED, d.norm_scale);
    pisco_mlp *net = nullptr;
    float mean[3], stdv[3];
    std::vector<double> hist;
    if (st == PISCO_OK) {
        pisco::SidelobeRun r{c, t, n_train, seed, epochs, c->sl_opts};
        st = pisco::sidelobe_train_run(r, &net, mean, stdv, hist);
    } else {
        fail(c, st, "annulus set-up failed: %s", pisco_last_error(t));
    }
    pisco_destroy(t);
    if (st != PISCO_OK) return st;
    auto sl = std::make_shared<SlNet>();
    sl->net = net;
    for (int k = 0; k < 3; ++k) {
        sl->mean[k] = mean[k];
        sl->stdv[k] = stdv[k];
    }
    sl->r_main = r_main;
    sl->wT = d.w[3];
    sl->norm = d.norm_scale;
    sl->hist = hist;
    d.sl = sl;
    ++c->generation;
    return PISCO_OK;
}

// Whether detector d can take a far-sidelobe network (the split of its TOD into
// disc + annulus pickups holds): a one-grid beam without V terms, no plate,
// FIXED normalisation, wT != 0, FP32 sky.
static pisco_status sidelobe_capable(pisco_ctx *c, int32_t det, const DetState &d) {
    if (c->sky && c->sky_dtype != PISCO_F32)
        return fail(c, PISCO_EINVAL, "the sidelobe network runs on the FP32 path only");
    if (d.beam_kind != pisco::BEAM_SCALAR || d.beam_v || d.wv != 0.0)
        return fail(c, PISCO_EINVAL, "detector %d: the sidelobe split needs a one-grid beam without V terms", det);
    if (d.hwp || !d.host_hwp.empty()) return fail(c, PISCO_EINVAL, "detector %d has a half-wave plate", det);
    if (d.norm_mode != PISCO_NORM_FIXED)
        return fail(c, PISCO_EINVAL, "detector %d: the sidelobe split needs FIXED normalisation", det);
    if (d.w[3] == 0.0) return fail(c, PISCO_EINVAL, "detector %d: wT is zero", det);
    return PISCO_OK;
}

pisco_status pisco_sidelobe_share(pisco_ctx *c, int32_t det, int32_t src) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (det < 0 || det >= PISCO_MAX_DETECTORS || src < 0 || src >= PISCO_MAX_DETECTORS)
        return fail(c, PISCO_EINVAL, "detector out of range");
    if ((size_t)src >= c->dets.size() || !c->dets[src].sl)
        return fail(c, PISCO_ESTATE, "detector %d has no trained sidelobe network", src);
    if ((size_t)det >= c->dets.size() || !c->dets[det].has_beam || !c->dets[det].has_params)
        return fail(c, PISCO_ESTATE, "detector %d lacks a beam or parameters", det);
    DetState &d = c->dets[det];
    const pisco_status st = sidelobe_capable(c, det, d);
    if (st != PISCO_OK) return st;
    if (det != src) {
        d.sl = c->dets[src].sl;
        ++c->generation;
    }
    return PISCO_OK;
}

pisco_status pisco_sidelobe_enable(pisco_ctx *c, int32_t det, int on) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (det < 0 || det >= PISCO_MAX_DETECTORS) return fail(c, PISCO_EINVAL, "detector %d out of range", det);
    if (on && ((size_t)det >= c->dets.size() || !c->dets[det].sl))
        return fail(c, PISCO_ESTATE, "detector %d has no trained sidelobe network", det);
    if ((size_t)det >= c->dets.size()) return PISCO_OK;
    DetState &d = c->dets[det];
    if (d.sl_on != (on != 0)) {
        d.sl_on = on != 0;
        ++c->generation;
    }
    return PISCO_OK;
}

int32_t pisco_sidelobe_history(const pisco_ctx *c, int32_t det, double *loss, int32_t cap) {
    if (!c || det < 0 || det >= PISCO_MAX_DETECTORS) return -1;
    if ((size_t)det >= c->dets.size()) return 0;
    const DetState &d = c->dets[det];
    if (!d.sl) return 0;
    const int32_t n = (int32_t)d.sl->hist.size();
    if (loss)
        for (int32_t i = 0; i < std::min(n, cap); ++i) loss[i] = d.sl->hist[i];
    return n;
}

pisco_status pisco_convolve_static(pisco_ctx *c, int32_t det, int out_mode, void *out, void *stream) {
    if (!c) return PISCO_EINVAL;
    c->err.clear();
    if (!c->sky) return fail(c, PISCO_ESTATE, "no sky set");
    if (out_mode != PISCO_OUT_TOD && out_mode != PISCO_OUT_STOKES && out_mode != PISCO_OUT_COUNT)
        return fail(c, PISCO_EINVAL, "bad out_mode %d", out_mode);
    if (det < 0 || (size_t)det >= c->dets.size() || !det_ready(c->dets[det]))
        return fail(c, PISCO_ESTATE, "detector %d lacks a beam, parameters or pointing", det);
    const DetState &d = c->dets[det];
    if (d.beam_dtype != c->sky_dtype) return fail(c, PISCO_EINVAL, "detector %d beam dtype differs from the sky dtype", det);
    if (!d.host_pointing.empty() || !d.host_hwp.empty())
        return fail(c, PISCO_EINVAL, "detector %d keeps its pointing or plate angles on the host (memory budget)", det);
    if (d.hwp && d.hwp_n != d.nsamp)
        return fail(c, PISCO_EINVAL, "detector %d has %lld plate angles for %lld samples", det, (long long)d.hwp_n,
                    (long long)d.nsamp);
    if (d.beam_v && c->algo != PISCO_ALGO_PIXEL && out_mode == PISCO_OUT_TOD &&
        (size_t)c->wpg * (4352 + std::max<size_t>(3840, 48 * (size_t)c->chunk) + 4 * (size_t)c->chunk) > 160 * 1024)
        return fail(c, PISCO_EINVAL, "detector %d: a V-column beam needs more LDS than chunk %d with %d waves per "
                    "group leaves", det, c->chunk, c->wpg);
    const bool sub = out_mode == PISCO_OUT_TOD && d.sl_on && d.sl;
    if (sub && c->sky_dtype != PISCO_F32)
        return fail(c, PISCO_EINVAL, "detector %d: the sidelobe network runs on the FP32 path only", det);
    if (d.nsamp == 0) return PISCO_OK;
    if (!out) return fail(c, PISCO_EINVAL, "null output");
    if (d.nsamp > pisco::STATIC_MAX_GROUPS * 64)
        return fail(c, PISCO_EINVAL, "detector %d has %lld samples; the allocation-free path takes at most %lld",
                    det, (long long)d.nsamp, (long long)(pisco::STATIC_MAX_GROUPS * 64));
    void *base = pisco::static_scratch(c->device);
    if (!base) return fail(c, PISCO_EDEVICE, "the plan array's device address is unknown");
    HIP_TRY(c, hipSetDevice(c->device));
    DetDesc x = make_desc(d, sub);
    x.theta = d.th;
    x.phi = d.ph;
    x.psi = d.ps;
    x.out_offset = 0;
    ConvArgs a{};
    a.sky = c->sky;
    a.out = out;
    a.nside = c->nside;
    a.out_mode = out_mode;
    a.beam_kind = d.beam_kind;
    a.chunk = c->chunk;
    a.coherence = c->coherence;
    a.per_sample = d.norm_mode == PISCO_NORM_PER_SAMPLE ? 1 : 0;
    a.hwp = d.hwp ? 1 : 0;
    a.vbeam = d.beam_v ? 1 : 0;
    const bool extended = d.beam_v || d.wv != 0.0 || d.hwp;
    ConvArgs tile = a, pix = a;
    tile.algo = (c->algo == PISCO_ALGO_TILE_MX && !extended) ? pisco::ALGO_TILE_MX : pisco::ALGO_TILE;
    pix.algo = pisco::ALGO_PIXEL;
    const bool tile_path = (c->algo == PISCO_ALGO_TILE || c->algo == PISCO_ALGO_TILE_MX) && c->sky_dtype == PISCO_F32;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = pisco::launch_static(tile, pix, x, tile_path, c->sky_dtype == PISCO_F64, c->wpg,
                                        c->gpc * c->num_cu, base, s);
    if (e == hipSuccess && sub) {
        const SlApply ap = sl_apply_of(d, d.th, d.ph, d.ps, d.nsamp, 0);
        e = pisco::mlp_apply_pointing(ap.net, ap.th, ap.ph, ap.ps, ap.n, ap.mean, ap.stdv, ap.coef,
                                      static_cast<float *>(out), s);
    }
    if (e != hipSuccess) return fail(c, PISCO_EDEVICE, "allocation-free convolution launch failed: %s", hipGetErrorString(e));
    return PISCO_OK;
}

}  // extern "C"
