// Internal types shared by the runtime and the convolution kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pisco {

enum { MODE_TOD = 0, MODE_STOKES = 1, MODE_COUNT = 2 };
enum { BEAM_FULL = 0, BEAM_SCALAR = 1 };
enum { ALGO_PIXEL = 0, ALGO_TILE = 1, ALGO_TILE_MX = 2 };

// Per-detector description, read by the kernel from device memory.
struct DetDesc {
    const void *beam;      // full: n*n node records (bI, bQ, bU, bT); scalar: (n+1)^2 cell polynomials
                           // (the (n-1)^2 grid cells inside a ring of extrapolated ones)
    const double *theta;   // pointing, SoA
    const double *phi;
    const double *psi;
    int64_t n_samples;
    int64_t out_offset;    // first output sample of this detector
    double zeta;
    double cos_rho_max;    // pixels with cos(rho) >= cos_rho_max ...
    double cos_rho_min;    // ... and (rho_min == 0 or cos(rho) < cos_rho_min)
    double rho_max;
    double norm_scale;
    double half_span_tan;  // T
    double inv_h;          // (n - 1) / (2T)
    double omega_max;      // 1 - cos(rho_max), computed as 2 sin^2(rho_max / 2)
    double omega_min;      // 1 - cos(rho_min)
    double w[4];           // scalar beam weights (wI, wQ, wU, wT); unused for full beams
    const void *beam_v;    // full beams with a V column: (n-1)^2 cell polynomials of bV, else null
    const double *hwp;     // per-sample half-wave-plate angle, or null (no plate)
    const int32_t *order;  // processing order: position t holds the caller's sample order[t]; null = given order
    double wv;             // scalar beam V weight
    double rot2z[2];       // (cos 2 zeta, sin 2 zeta) / inv_h^2: the tile path's turn of the staged Q, U
    int32_t n;             // grid nodes per side
    int32_t norm_mode;     // 0 fixed, 1 per sample
    int32_t has_inner;     // rho_min > 0
    int32_t needs_clip;    // the disc can reach beyond the grid
};

// A tile: `count` consecutive samples of detector `det` starting at `begin`.
struct Tile {
    int32_t det;
    int32_t count;
    int64_t begin;
};

struct ConvArgs {
    const void *sky;         // 12 nside^2 records (float4 / double4): I, Q, U, V
    const DetDesc *dets;
    const Tile *tiles;       // tiles[q * tiles_per_queue + i] for queue q
    int32_t *counters;       // one work counter per queue (zeroed before launch)
    void *out;               // float or double
    int64_t nside;
    int32_t n_queues;        // 1 or 8
    int32_t tiles_per_queue; // padded queue length
    const int32_t *queue_len;
    int32_t out_mode;        // MODE_*
    int32_t beam_kind;       // BEAM_* (uniform over the launch)
    int32_t algo;            // ALGO_*
    int32_t chunk;           // pixel records staged per pass (64, 128, 256)
    double coherence;        // tile path: samples within this many disc radii of the tile centre
    int32_t per_sample;      // some detector of the launch uses per-sample normalisation
    int32_t hwp;             // some detector of the launch has a half-wave plate
    int32_t vbeam;           // some detector of the launch has a full beam with a V column
};

// Launch helpers (conv_kernel.hip).  Return the launch error.
hipError_t launch_zero_counters(int32_t *counters, int n, hipStream_t s);
hipError_t launch_conv(const ConvArgs &a, bool f64, int waves_per_group, int groups, hipStream_t s);
hipError_t launch_repack4(const void *a, const void *b, const void *c, const void *d, void *out, int64_t n,
                          bool f64, hipStream_t s);
hipError_t launch_repack_cells(const void *b, int32_t n, void *out, bool f64, bool padded, hipStream_t s);
// HEALPix beam maps (nside, nch channels) resampled onto an n x n node grid over [-T, T]^2.
struct HpxGridArgs {
    int32_t nside, n, nch;
    double T;
    const void *map[4];
    void *out[4];
};
hipError_t launch_healpix_grid(const HpxGridArgs &a, bool f64, hipStream_t s);
// Spatial processing order (order_kernel.hip): order[t] = the sample at position t when the n samples
// are sorted along a Hilbert curve over (phi, cos theta); synchronises on `s`.
hipError_t spatial_order(const double *theta, const double *phi, int64_t n, int32_t *order, hipStream_t s);
// keys[i] = Hilbert rank (as in spatial_order) of the first sample of tiles[i].
hipError_t launch_tile_keys(const DetDesc *dets, const Tile *tiles, int32_t n, uint32_t *keys, hipStream_t s);
hipError_t launch_classify(const DetDesc *dets, const Tile *groups, int32_t n_groups, double frac, int32_t *flag,
                           hipStream_t s);
hipError_t launch_check_pointing(const double *theta, const double *phi, const double *psi, int64_t n,
                                 int32_t *bad, hipStream_t s);

// Allocation-free single-detector launches (pisco_convolve_static): the plan of
// one call lives in a file-scope device array of conv_kernel.hip, one copy per
// GPU.  Layout: int32 control block [32] at 0 (work counters and queue lengths as
// in a Plan), the DetDesc at STATIC_DESC_OFF, the tile-path and pixel-path
// queues of STATIC_MAX_GROUPS tiles each.
constexpr int64_t STATIC_MAX_GROUPS = 1 << 16;
constexpr size_t STATIC_DESC_OFF = 256;
constexpr size_t STATIC_TQ_OFF = 1024;
constexpr size_t STATIC_PQ_OFF = STATIC_TQ_OFF + sizeof(Tile) * STATIC_MAX_GROUPS;
constexpr size_t STATIC_SCRATCH_BYTES = STATIC_PQ_OFF + sizeof(Tile) * STATIC_MAX_GROUPS;
// Resolves the array's device address on the current device (once per device).
hipError_t static_scratch_init(int device);
// That address, or null before static_scratch_init succeeded on `device`.
void *static_scratch(int device);
// Zero the control block, classify and queue the 64-sample groups of D on the
// device, then run the tile and pixel kernels with args tile / pix (their plan
// pointers are filled in here).
hipError_t launch_static(ConvArgs tile, ConvArgs pix, const DetDesc &D, bool tile_path, bool f64, int waves,
                         int groups, void *base, hipStream_t s);

}  // namespace pisco

// Context accessors for the sidelobe-network and map-making runtimes (runtime.cpp).
struct pisco_ctx;
namespace pisco {
void set_error(pisco_ctx *c, const char *msg);
int ctx_device(const pisco_ctx *c);
int ctx_num_cu(const pisco_ctx *c);
bool ctx_pointing(const pisco_ctx *c, int32_t det, const double **th, const double **ph, const double **ps,
                  int64_t *n);
}  // namespace pisco
