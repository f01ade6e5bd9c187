// Host runtime behind the C ABI declared in include/pisco.h: device buffers,
// validation, the tile plan and work queues, HIP-graph replay of the batched
// launch, and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pisco.h"
#include "pisco_internal.h"

using pisco::ConvArgs;
using pisco::DetDesc;
using pisco::Tile;

namespace {

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

    Plan plans[2];            // [0] batched (det = -1), [1] single detector
    int32_t *d_flag = nullptr;

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

DetState *det_slot(pisco_ctx *c, int32_t det) {
    if (det < 0 || det >= PISCO_MAX_DETECTORS) return nullptr;
    if ((size_t)det >= c->dets.size()) c->dets.resize(det + 1);
    return &c->dets[det];
}

bool det_ready(const DetState &d) { return d.has_beam && d.has_params && d.has_pointing; }

void release_beam(pisco_ctx *c, int32_t det) {
    DetState &d = c->dets[det];
    if (d.beam_owned && d.beam) {
        // detectors sharing this buffer lose their beam
        for (size_t k = 0; k < c->dets.size(); ++k)
            if ((int32_t)k != det && c->dets[k].beam == d.beam && !c->dets[k].beam_owned) {
                c->dets[k].beam = nullptr;
                c->dets[k].beam_v = nullptr;
                c->dets[k].has_beam = false;
            }
        (void)hipFree(d.beam);
        if (d.beam_v) (void)hipFree(d.beam_v);
    }
    d.beam = nullptr;
    d.beam_v = nullptr;
    d.wv = 0.0;
    d.beam_owned = false;
    d.has_beam = false;
}

void release_hwp(DetState &d) {
    if (d.owned_hwp) (void)hipFree(d.owned_hwp);
    d.owned_hwp = nullptr;
    d.hwp = nullptr;
    d.hwp_n = 0;
}

void release_pointing(DetState &d) {
    if (d.owned_pointing) (void)hipFree(d.owned_pointing);
    d.owned_pointing = nullptr;
    if (d.order) (void)hipFree(d.order);
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

void free_plan(Plan &p) {
    drop_graph(p);
    if (p.d_dets) (void)hipFree(p.d_dets);
    if (p.tq.d_tiles) (void)hipFree(p.tq.d_tiles);
    if (p.pq.d_tiles) (void)hipFree(p.pq.d_tiles);
    if (p.d_ctrl) (void)hipFree(p.d_ctrl);
    if (p.d_scratch) (void)hipFree(p.d_scratch);
    p = Plan();
}

// Copy a host or device array to a fresh device buffer of `bytes`.
pisco_status to_device(pisco_ctx *c, const void *src, size_t bytes, int mem, void **out) {
    void *p = nullptr;
    if (bytes == 0) {
        *out = nullptr;
        return PISCO_OK;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", bytes);
    const hipError_t e = hipMemcpy(p, src, bytes, mem == PISCO_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
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
    if (hipMalloc(&rec, rec_bytes(dtype) * (size_t)n) != hipSuccess)
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
            if (tmp[k]) (void)hipFree(tmp[k]);
    if (st != PISCO_OK) {
        (void)hipFree(rec);
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
    if (hipMalloc(&q, nc * sizeof(T)) != hipSuccess) return false;
    if (*p) (void)hipFree(*p);
    *p = static_cast<T *>(q);
    *cap = nc;
    (void)c;
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

// Build and upload the tile plan for `det` (-1 = all ready detectors).
pisco_status prepare_plan(pisco_ctx *c, Plan &p, int32_t det) {
    if (p.gen == c->generation && p.det == det && p.spt == c->spt && p.xq == c->xq && p.algo == c->algo &&
        p.coherence == c->coherence)
        return PISCO_OK;
    std::vector<DetDesc> descs;
    std::vector<int32_t> det_of;   // detector index of each descriptor
    int64_t out_off = 0;
    p.per_sample = 0;
    p.hwp = 0;
    p.vbeam = 0;
    p.extended = 0;
    const int32_t lo = det < 0 ? 0 : det, hi = det < 0 ? (int32_t)c->dets.size() - 1 : det;
    for (int32_t k = lo; k <= hi; ++k) {
        const DetState &d = c->dets[k];
        if (!det_ready(d)) continue;
        DetDesc x{};
        x.beam = d.beam;
        x.theta = d.th;
        x.phi = d.ph;
        x.psi = d.ps;
        x.n_samples = d.nsamp;
        x.out_offset = out_off;
        x.zeta = d.zeta;
        x.cos_rho_max = std::cos(d.rho_max);
        x.cos_rho_min = std::cos(d.rho_min);
        x.rho_max = d.rho_max;
        x.norm_scale = d.norm_scale;
        x.half_span_tan = d.T;
        x.inv_h = (double)(d.n - 1) / (2.0 * d.T);
        x.omega_max = 2.0 * std::sin(0.5 * d.rho_max) * std::sin(0.5 * d.rho_max);
        x.omega_min = 2.0 * std::sin(0.5 * d.rho_min) * std::sin(0.5 * d.rho_min);
        for (int i = 0; i < 4; ++i) x.w[i] = d.w[i];
        x.beam_v = d.beam_v;
        x.wv = d.wv;
        x.hwp = d.hwp;
        if (d.hwp) p.hwp = 1;
        if (d.beam_v) p.vbeam = 1;
        if (d.beam_v || d.wv != 0.0 || d.hwp) p.extended = 1;
        // a disc inside the grid's square maps every member into the grid (|u|, |v| <= tan rho)
        x.needs_clip = (std::tan(d.rho_max) <= d.T * (1.0 + 1e-12)) ? 0 : 1;
        x.n = d.n;
        x.norm_mode = d.norm_mode;
        x.has_inner = d.rho_min > 0.0 ? 1 : 0;
        x.order = nullptr;
        descs.push_back(x);
        det_of.push_back(k);
        out_off += d.nsamp;
        p.beam_kind = d.beam_kind;
        if (d.norm_mode == PISCO_NORM_PER_SAMPLE) p.per_sample = 1;
    }
    hipError_t e = hipDeviceSynchronize();  // no launch may still read the old plan
    if (e != hipSuccess) return fail(c, PISCO_EDEVICE, "synchronise failed: %s", hipGetErrorString(e));
    if (!p.d_ctrl && hipMalloc(&p.d_ctrl, 32 * sizeof(int32_t)) != hipSuccess)
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
    if (c->ordering == PISCO_ORDER_SPATIAL)
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
            if (p.d_scratch) (void)hipFree(p.d_scratch);
            p.d_scratch = nullptr;
            p.scratch_cap = 0;
            if (hipMalloc(&p.d_scratch, need) != hipSuccess) return fail(c, PISCO_ENOMEM, "plan scratch allocation failed");
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
    if (c->ordering == PISCO_ORDER_AUTO && tile_path) {
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
    std::vector<Tile> ttiles, ptiles;
    for (size_t g = 0; g < groups.size(); ++g) {
        if (flag[g]) {
            ttiles.push_back(groups[g]);
            continue;
        }
        // pixel path: merge runs of incoherent groups of one detector, then cut into spt-sample tiles
        const Tile &x = groups[g];
        if (!ptiles.empty() && ptiles.back().det == x.det && ptiles.back().begin + ptiles.back().count == x.begin &&
            ptiles.back().count < c->spt) {
            Tile &b = ptiles.back();
            const int32_t room = c->spt - b.count, take = std::min(room, x.count);
            b.count += take;
            if (take < x.count) {
                Tile t;
                t.det = x.det;
                t.begin = x.begin + take;
                t.count = x.count - take;
                ptiles.push_back(t);
            }
        } else {
            ptiles.push_back(x);
        }
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
    p.gen = c->generation;
    p.det = det;
    p.spt = c->spt;
    p.xq = c->xq;
    p.algo = c->algo;
    p.coherence = c->coherence;
    p.out_samples = out_off;
    drop_graph(p);
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
    if (p.pq.ntiles > 0) e = pisco::launch_conv(make_args(c, p, out, out_mode, false), f64, c->wpg, c->gpc * c->num_cu, s);
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
    if (hipMalloc(&c->d_flag, sizeof(int32_t)) != hipSuccess) {
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
    for (auto &p : c->plans) free_plan(p);
    for (auto &t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (size_t k = 0; k < c->dets.size(); ++k) {
        release_beam(c, (int32_t)k);
        release_pointing(c->dets[k]);
        release_hwp(c->dets[k]);
    }
    if (c->sky) (void)hipFree(c->sky);
    if (c->d_flag) (void)hipFree(c->d_flag);
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
    if (c->sky) (void)hipFree(c->sky);
    c->sky = rec;
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
        if (st == PISCO_OK && hipMalloc(&nodes[k], nbytes) != hipSuccess)
            st = fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", nbytes);
        a.out[k] = nodes[k];
    }
    if (st == PISCO_OK) {
        hipError_t e = pisco::launch_healpix_grid(a, dtype == PISCO_F64, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) st = fail(c, PISCO_EDEVICE, "beam map resampling failed: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < nch; ++k)
        if (staged[k]) (void)hipFree(staged[k]);
    if (st != PISCO_OK)
        for (int k = 0; k < nch; ++k)
            if (nodes[k]) {
                (void)hipFree(nodes[k]);
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
    for (int k = 0; k < 4; ++k) (void)hipFree(nodes[k]);
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
    (void)hipFree(nodes[0]);
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
    if (hipMalloc(&rec, rec_bytes(dtype) * cells) != hipSuccess) {
        if (mem == PISCO_HOST) (void)hipFree(src);
        return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", rec_bytes(dtype) * cells);
    }
    hipError_t e = pisco::launch_repack_cells(src, n, rec, dtype == PISCO_F64, true, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (mem == PISCO_HOST) (void)hipFree(src);
    if (e != hipSuccess) {
        (void)hipFree(rec);
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
    if (hipMalloc(&rec, rec_bytes(dtype) * cells) != hipSuccess) {
        if (mem == PISCO_HOST) (void)hipFree(src);
        return fail(c, PISCO_ENOMEM, "device allocation of %zu bytes failed", rec_bytes(dtype) * cells);
    }
    hipError_t e = pisco::launch_repack_cells(src, n, rec, dtype == PISCO_F64, false, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (mem == PISCO_HOST) (void)hipFree(src);
    if (e != hipSuccess) {
        (void)hipFree(rec);
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
        release_hwp(*d);
        ++c->generation;
        return PISCO_OK;
    }
    if (mem == PISCO_HOST) {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(angle[i])) return fail(c, PISCO_EINVAL, "plate angle %lld is not finite", (long long)i);
        double *buf = nullptr;
        if (hipMalloc(&buf, sizeof(double) * (size_t)n) != hipSuccess)
            return fail(c, PISCO_ENOMEM, "plate-angle allocation failed");
        const hipError_t e = hipMemcpy(buf, angle, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return fail(c, PISCO_EDEVICE, "plate-angle copy failed: %s", hipGetErrorString(e));
        }
        release_hwp(*d);
        d->owned_hwp = buf;
        d->hwp = buf;
    } else {
        release_hwp(*d);
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
        double *buf = nullptr;
        if (n > 0) {
            if (hipMalloc(&buf, 3 * sizeof(double) * (size_t)n) != hipSuccess)
                return fail(c, PISCO_ENOMEM, "pointing allocation failed");
            const size_t b = sizeof(double) * (size_t)n;
            hipError_t e = hipMemcpy(buf, theta, b, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(buf + n, phi, b, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(buf + 2 * n, psi, b, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(buf);
                return fail(c, PISCO_EDEVICE, "pointing copy failed: %s", hipGetErrorString(e));
            }
        }
        HIP_TRY(c, hipDeviceSynchronize());
        release_pointing(*d);
        d->owned_pointing = buf;
        d->th = buf;
        d->ph = buf ? buf + n : nullptr;
        d->ps = buf ? buf + 2 * n : nullptr;
    } else {
        if (n > 0) {
            HIP_TRY(c, hipMemset(c->d_flag, 0, sizeof(int32_t)));
            HIP_TRY(c, pisco::launch_check_pointing(theta, phi, psi, n, c->d_flag, nullptr));
            int32_t bad = 0;
            HIP_TRY(c, hipMemcpy(&bad, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost));
            if (bad) return fail(c, PISCO_EINVAL, "pointing holds non-finite values or theta outside [0, pi]");
        }
        HIP_TRY(c, hipDeviceSynchronize());
        release_pointing(*d);
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
    bool any = false;
    int first_kind = -1;
    const int32_t lo = det < 0 ? 0 : det, hi = det < 0 ? (int32_t)c->dets.size() - 1 : det;
    for (int32_t k = lo; k <= hi; ++k) {
        const DetState &d = c->dets[k];
        if (!det_ready(d)) continue;
        any = true;
        if (d.beam_dtype != c->sky_dtype)
            return fail(c, PISCO_EINVAL, "detector %d beam dtype differs from the sky dtype", k);
        if (d.hwp && d.hwp_n != d.nsamp)
            return fail(c, PISCO_EINVAL, "detector %d has %lld plate angles for %lld samples", k, (long long)d.hwp_n,
                        (long long)d.nsamp);
        // a V column adds 4 bytes of LDS per staged record and wave on the tile path
        if (d.beam_v && c->algo != PISCO_ALGO_PIXEL && out_mode == PISCO_OUT_TOD &&
            (size_t)c->wpg * (4352 + std::max<size_t>(3840, 48 * (size_t)c->chunk) + 4 * (size_t)c->chunk) >
                160 * 1024)
            return fail(c, PISCO_EINVAL, "detector %d: a V-column beam needs more LDS than chunk %d with %d waves "
                        "per group leaves; use a smaller chunk or fewer waves", k, c->chunk, c->wpg);
        if (first_kind < 0) first_kind = d.beam_kind;
        if (d.beam_kind != first_kind)
            return fail(c, PISCO_EINVAL, "detectors in one launch must all have full or all scalar beams");
    }
    if (!any) return fail(c, PISCO_ESTATE, "no detector is ready");
    HIP_TRY(c, hipSetDevice(c->device));
    Plan &p = c->plans[det < 0 ? 0 : 1];
    pisco_status st = prepare_plan(c, p, det);
    if (st != PISCO_OK) return st;
    const int64_t nout = p.out_samples * (out_mode == PISCO_OUT_STOKES ? 3 : 1);
    if (nout == 0) return PISCO_OK;
    if (!out) return fail(c, PISCO_EINVAL, "null output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *dout = out;
    if (mem == PISCO_HOST) {
        s = nullptr;
        if (hipMalloc(&dout, el_bytes(c->sky_dtype) * (size_t)nout) != hipSuccess)
            return fail(c, PISCO_ENOMEM, "output staging allocation failed");
    }
    TimedLaunch tl{};
    if (c->timing) {
        HIP_TRY(c, hipEventCreate(&tl.a));
        HIP_TRY(c, hipEventCreate(&tl.b));
        HIP_TRY(c, hipEventRecord(tl.a, s));
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
        if (mem == PISCO_HOST) (void)hipFree(dout);
        return fail(c, PISCO_EDEVICE, "convolution launch failed: %s", hipGetErrorString(e));
    }
    if (c->timing) {
        HIP_TRY(c, hipEventRecord(tl.b, s));
        c->pending.push_back(tl);
    }
    if (mem == PISCO_HOST) {
        e = hipMemcpy(out, dout, el_bytes(c->sky_dtype) * (size_t)nout, hipMemcpyDeviceToHost);
        (void)hipFree(dout);
        if (e != hipSuccess) return fail(c, PISCO_EDEVICE, "output copy failed: %s", hipGetErrorString(e));
    }
    return PISCO_OK;
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

}  // extern "C"
