/*
 * pisco.h -- C ABI of the MI355X pixel-space polarised beam convolver.
 *
 * The operation (Fluxa, Brewer & Dunner, "Pixel space convolution for cosmic
 * microwave background experiments", Sec. 4.2, the pixelated convolution
 * equation) turns a pointing stream into a time-ordered data (TOD) stream:
 *
 *   d(theta0, phi0, psi0) = N * sum_k  D(chi_k) Lambda(chi_k) B_k Lambda(-chi_k) S_k
 *
 * over the HEALPix sky pixels k whose centres lie within rho_max of the
 * boresight.  Because D(chi) Lambda(chi) = D(0) (Sec. 4.1, the detector row
 * vector and the rotation matrix), the detector row can be folded into the
 * beamsor once per detector; the library therefore takes three effective
 * beam channels plus the normalising channel:
 *
 *   bI = (s/2)[(1+eps) B_TT + (1-eps) B_TQ]      (D(0) B, column T)
 *   bQ = (s/2)[(1+eps) B_QT + (1-eps) B_QQ]      (D(0) B, column Q)
 *   bU = (s/2)[(1+eps) B_UT + (1-eps) B_UQ]      (D(0) B, column U)
 *   bT = B_TT                                    (normalisation, Sec. 3)
 *
 * and per pair computes bI I + bQ (cos2chi Q + sin2chi U) + bU (-sin2chi Q + cos2chi U).
 * The sky's V is taken as zero (the CMB carries no circular polarisation).
 *
 * Geometry: theta = colatitude, phi = longitude, psi = position angle of the
 * antenna basis (Sec. 2, antenna basis vectors); zeta = detector angle from
 * theta'_0 (Sec. 3, PSB polarisation vectors); chi is the angle from the
 * pixel's theta_hat to the co-polar direction (Sec. 2 and Appendix A, Ludwig's
 * third definition).  The beam is a tangent-plane (gnomonic) grid of the
 * antenna frame: u = tan(rho) cos(sigma), v = tan(rho) sin(sigma).
 *
 * Conventions shared by every call:
 *   - All functions return PISCO_OK or an error code; no exception crosses
 *     the ABI.  After an error, pisco_last_error(ctx) holds a message; the
 *     context stays usable and its previous state is unchanged.
 *   - `mem` says where a caller pointer lives: PISCO_HOST (pageable or pinned
 *     host memory; the library copies synchronously) or PISCO_DEVICE (memory
 *     on the context's device).
 *   - Pointers are borrowed only for the duration of the call unless stated.
 *   - A context is bound to one device and is not thread-safe; use one
 *     context per host thread.  Single-detector launches share one work
 *     counter, and batched launches another: two launches of the same kind
 *     must not overlap in time on different streams.
 */
#ifndef PISCO_H
#define PISCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pisco_ctx pisco_ctx;

typedef enum {
    PISCO_OK = 0,
    PISCO_EINVAL = 1,      /* invalid argument (size, range, non-finite value, dtype mismatch) */
    PISCO_ENOMEM = 2,      /* device or host allocation failed */
    PISCO_EDEVICE = 3,     /* a HIP runtime call failed */
    PISCO_ESTATE = 4,      /* call out of order (e.g. convolve before set_sky) */
    PISCO_EUNSUPPORTED = 5 /* device is not gfx950 or feature not built */
} pisco_status;

enum { PISCO_F32 = 0, PISCO_F64 = 1 };
enum { PISCO_HOST = 0, PISCO_DEVICE = 1 };
enum { PISCO_NORM_FIXED = 0, PISCO_NORM_PER_SAMPLE = 1 };
enum { PISCO_OUT_TOD = 0, PISCO_OUT_STOKES = 1, PISCO_OUT_COUNT = 2 };

#define PISCO_MAX_DETECTORS 4096
#define PISCO_MAX_NSIDE 8192

/* ABI version of this header (major * 100 + minor). */
int pisco_abi_version(void);

/* Create a context on HIP device `device`.  Fails with EUNSUPPORTED unless the
 * device is gfx950.  *out receives the context (owned by the caller; release
 * with pisco_destroy). */
pisco_status pisco_create(int device, pisco_ctx **out);

/* Release every device buffer the context owns.  NULL is accepted. */
void pisco_destroy(pisco_ctx *ctx);

/* Message of the most recent failed call (empty if none); owned by ctx, valid
 * until the next call on ctx. */
const char *pisco_last_error(const pisco_ctx *ctx);

/*
 * Sky maps (Sec. 5.1: Stokes I, Q, U as HEALPix maps; RING order, Gorski et
 * al. 2005).  Each map holds 12 * nside^2 elements of `dtype`.  nside must be
 * a power of two in [1, PISCO_MAX_NSIDE].  The library copies the maps into its
 * own interleaved device layout (one 16-byte (F32) or 32-byte (F64) record
 * per pixel); the caller's buffers are not retained.  The sky's dtype fixes
 * the precision of every later convolve: F64 runs the double-precision
 * kernel, F32 the mixed-precision one.
 */
pisco_status pisco_set_sky(pisco_ctx *ctx, int64_t nside, const void *I, const void *Q, const void *U,
                           int dtype, int mem);

/* As pisco_set_sky with the fourth Stokes map V (circular polarisation; the
 * discrete sum of Sec. 4.2 runs over T, Q, U, V).  V may be NULL (zero). */
pisco_status pisco_set_sky_iquv(pisco_ctx *ctx, int64_t nside, const void *I, const void *Q, const void *U,
                                const void *V, int dtype, int mem);

/*
 * Effective beam of detector `det` (0 <= det < PISCO_MAX_DETECTORS): an n x n
 * grid (n odd, 3..4095) of nodes at u, v in [-T, T] (T = half_span_tan > 0),
 * node (iu, iv) at (-T + iu h, -T + iv h) with h = 2T/(n-1), row-major [iv][iu].
 * bI, bQ, bU, bT are the channels described above, n*n elements of `dtype`
 * each, which must equal the sky's dtype at convolve time.  Between nodes the
 * beam is bilinear; outside the grid it is zero.  Copied into one 16/32-byte
 * record per node.
 */
pisco_status pisco_set_beam(pisco_ctx *ctx, int32_t det, int32_t n, double half_span_tan,
                            const void *bI, const void *bQ, const void *bU, const void *bT,
                            int dtype, int mem);

/*
 * Scalar beam of detector `det`: the Mueller field factors into one n x n grid
 * b(u, v) (same node layout as pisco_set_beam) times constant channel weights,
 * bI = wI b, bQ = wQ b, bU = wU b, bT = wT b -- e.g. an ideal beamsor b (x) I
 * (Sec. 3) folded with the detector row gives wI = (s/2)(1+eps),
 * wQ = (s/2)(1-eps), wU = 0, wT = 1.  Stored as one record per grid cell with
 * the cell's four corners, so each bilinear lookup is a single load.  In
 * STOKES mode the scalar beam is wT b.
 */
pisco_status pisco_set_beam_scalar(pisco_ctx *ctx, int32_t det, int32_t n, double half_span_tan, const void *b,
                                   double wI, double wQ, double wU, double wT, int dtype, int mem);

/*
 * Beams that couple the sky's V into the measurement (the beamsor's V column,
 * Sec. 3 equation beamsor; the detector row of Sec. 4.1 has no V entry, so
 * D(0) B contributes bV = (s/2)[(1+eps) B_TV + (1-eps) B_QV] per pixel):
 * pisco_set_beam_v takes a fifth channel bV on the same node grid (NULL: none;
 * stored as cell polynomials beside the four-channel records);
 * pisco_set_beam_scalar_v a V weight, bV = wV b.  Per pair the term gains
 * bV V (V is not rotated by Lambda).
 */
pisco_status pisco_set_beam_v(pisco_ctx *ctx, int32_t det, int32_t n, double half_span_tan, const void *bI,
                              const void *bQ, const void *bU, const void *bV, const void *bT, int dtype, int mem);
pisco_status pisco_set_beam_scalar_v(pisco_ctx *ctx, int32_t det, int32_t n, double half_span_tan, const void *b,
                                     double wI, double wQ, double wU, double wV, double wT, int dtype, int mem);

/*
 * Rotating half-wave plate: a modulated beamsor (the paper's conclusions note
 * that modulation needs nothing more than a modulated beamsor model).  Sample
 * t of detector `det` uses B(u, v) H(phi_t) with H(phi) = Lambda(phi)
 * diag(1, 1, -1, -1) Lambda(-phi) (Lambda of Sec. 4.1): an ideal plate, sky
 * side of the beam, its axis at angle phi_t (rad) from the antenna frame's
 * reference direction.  Per pair the Stokes rotation angle becomes
 * 2 chi + 4 phi_t and the U-row and V terms change sign.  `angle` holds n
 * values (n must equal the detector's sample count at convolve time); host
 * arrays are copied, device arrays borrowed.  angle = NULL or n = 0 removes
 * the plate.
 */
pisco_status pisco_set_hwp(pisco_ctx *ctx, int32_t det, int64_t n, const double *angle, int mem);

/* Let detector `det` use the beam of detector `src` (no copy; e.g. one shared
 * far-sidelobe grid).  `src` must already have a beam. */
pisco_status pisco_share_beam(pisco_ctx *ctx, int32_t det, int32_t src);
/*
 * Beamsors given as HEALPix maps (the representation the paper stores them
 * in, Sec. 4.2 and Sec. 5.1, "re-pixelated via interpolation"): RING maps of
 * 12 nside_beam^2 values with the boresight at the map's north pole, theta
 * the distance rho from it and phi the antenna-frame azimuth sigma (from
 * theta'_0 toward phi'_0).  The library resamples them once, on the device,
 * onto the n x n gnomonic grid over [-half_span_tan, half_span_tan]^2 of
 * pisco_set_beam: node (u, v) reads the map at theta = atan(sqrt(u^2 + v^2)),
 * phi = atan2(v, u), linearly in phi between the two bracketing pixels of
 * each of the two rings that bracket theta and linearly in theta between the
 * rings (above the first ring the north pole stands in, valued at the mean of
 * that ring's four pixels; likewise the south pole below the last).  The
 * convolution then reads the grid as for pisco_set_beam / pisco_set_beam_scalar.
 * Channels as there (bI, bQ, bU, bT, or one map b with weights); dtype/mem as
 * for the sky; host maps are copied, device maps are read before the call
 * returns.  EINVAL: nside_beam not a power of two in [1, 8192], n not odd in
 * [3, 4095], half_span_tan not finite and > 0, a null map.
 */
pisco_status pisco_set_beam_healpix(pisco_ctx *ctx, int32_t det, int64_t nside_beam, const void *bI, const void *bQ,
                                    const void *bU, const void *bT, int32_t n, double half_span_tan, int dtype,
                                    int mem);
pisco_status pisco_set_beam_healpix_scalar(pisco_ctx *ctx, int32_t det, int64_t nside_beam, const void *b, double wI,
                                           double wQ, double wU, double wT, int32_t n, double half_span_tan,
                                           int dtype, int mem);


/*
 * Detector parameters: zeta (rad, Sec. 3); pixels with rho_min < rho <= rho_max
 * take part (rho_min = 0 selects the whole disc, inclusive of rho = 0;
 * 0 <= rho_min < rho_max < pi/2).  Normalisation N: FIXED -> N = norm_scale;
 * PER_SAMPLE -> N = norm_scale / sum_k bT(k) over the same pixels (0 when the
 * sum is 0).
 */
pisco_status pisco_set_detector(pisco_ctx *ctx, int32_t det, double zeta, double rho_min, double rho_max,
                                int norm_mode, double norm_scale);

/*
 * Pointing stream of detector `det`: n samples of colatitude theta in [0, pi],
 * longitude phi and position angle psi (radians, float64, structure of arrays).
 * mem = HOST: copied to the device (after validation).  mem = DEVICE: the
 * arrays are borrowed and must stay valid, unchanged, until the last convolve
 * that uses them has completed on its stream; they are validated once here.
 * Non-finite values or theta outside [0, pi] give EINVAL.  n may be 0.
 */
pisco_status pisco_set_pointing(pisco_ctx *ctx, int32_t det, int64_t n, const double *theta,
                                const double *phi, const double *psi, int mem);

/*
 * Convolve.  det >= 0: that detector's stream; det = -1: every configured
 * detector in one persistent launch (replayed from a captured HIP graph when
 * the configuration and output buffer are unchanged), outputs concatenated in
 * ascending detector order.  out_mode TOD writes one value per sample;
 * STOKES writes three per sample ([t][3]: N sum bT Lambda(-chi) S restricted
 * to I, Q, U, the detector-frame Stokes pickup of the scalar beam bT);
 * COUNT writes, per sample, the number of sky pixels selected (the pairs the
 * sum runs over, as a floating value), without evaluating them.
 * `out` holds elements of the sky's dtype; mem = DEVICE: written
 * asynchronously on `stream` (a hipStream_t, NULL = default stream);
 * mem = HOST: the call synchronises and copies.
 */
pisco_status pisco_convolve(pisco_ctx *ctx, int32_t det, int out_mode, void *out, int mem, void *stream);

/*
 * Allocation-free convolve of one detector, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts that
 * forbid allocation after start-up.  Same result as pisco_convolve(det, ...)
 * under PISCO_ORDER_GIVEN (samples are processed in the given order), written
 * to `out`, which must be device memory (sky dtype, one value per sample, three
 * for STOKES); asynchronous on `stream`, no host synchronisation.  The call
 * allocates nothing: its plan (descriptor, work counters and queues) is built
 * on the device in one static array of the library, 2 MiB, which each GPU the
 * library runs on holds until the process ends; it takes at most 4,194,304
 * samples per call (EINVAL beyond).  Every call on a GPU shares that array:
 * calls that overlap in time on one GPU (other streams, other contexts, other
 * host threads) race and must be serialised by the caller.  Needs the
 * detector's pointing and plate angles on the device (EINVAL when the memory
 * budget kept them on the host); a surrogate-enabled detector adds its
 * network as in pisco_convolve.  Kernel timing (pisco_set_timing) does not
 * cover these calls.
 */
pisco_status pisco_convolve_static(pisco_ctx *ctx, int32_t det, int out_mode, void *out, void *stream);

/* Number of output samples convolve(det) writes (det = -1: all detectors). */
int64_t pisco_output_samples(const pisco_ctx *ctx, int32_t det);

/*
 * Launch shape of the convolution.
 *   algorithm        PISCO_ALGO_PIXEL: a wavefront takes one sample at a time and
 *                    its lanes stride that sample's disc pixels (used for FP64
 *                    and for incoherent pointing).  PISCO_ALGO_TILE (FP32): the
 *                    lanes of a wavefront take 64 consecutive samples and walk
 *                    the pixels of the union of their discs together; tiles
 *                    whose samples are not within `coherence` disc radii of
 *                    their mean direction fall back to the pixel path.
 *                    PISCO_ALGO_TILE_MX (FP32): the tile path with the
 *                    pixel-linear quantities of every (pixel, sample) pair
 *                    (1 - n.p, the antenna-frame coordinates, the co-polar
 *                    projections) formed by FP32 matrix-core products.
 *                    Launches with a half-wave plate or V terms run the
 *                    PISCO_ALGO_TILE kernels instead.  Kept for comparison:
 *                    on gfx950 it runs about twice as long as PISCO_ALGO_TILE
 *                    (it saves few vector instructions and its vector work
 *                    waits on the matrix results).
 *   samples_per_tile consecutive samples a wavefront takes per queue pop (1..65536)
 *   waves_per_group  wavefronts per workgroup (1, 2, 4 or 8)
 *   groups_per_cu    workgroups launched per compute unit (1..16)
 *   xcd_queues       1: one shared work queue; 8: one queue per accelerator
 *                    die, each holding a contiguous block of tiles (a
 *                    workgroup starts on its die's queue and takes from the
 *                    others once it is empty).  Each detector's tiles are
 *                    queued in the Hilbert order of their first samples, so
 *                    that tiles running together on a die share sky in L2.
 *   chunk            tile paths: union pixels staged in LDS per pass (64, 128, 256)
 *   coherence        tile paths: see algorithm, in (0, 4]
 * A new context starts at {PISCO_ALGO_TILE, 64, 4, 4, 1, 64, 0.5}.
 * Results are bitwise reproducible for a given launch shape.  They do not
 * depend on the shape except through the algorithm (the two paths round
 * differently) and, on the tile path, through samples_per_tile when it is not
 * a multiple of 64 (it decides which samples share a tile frame).
 */
enum { PISCO_ALGO_PIXEL = 0, PISCO_ALGO_TILE = 1, PISCO_ALGO_TILE_MX = 2 };
typedef struct {
    int32_t algorithm;
    int32_t samples_per_tile;
    int32_t waves_per_group;
    int32_t groups_per_cu;
    int32_t xcd_queues;
    int32_t chunk;
    double coherence;
} pisco_launch;
pisco_status pisco_set_launch(pisco_ctx *ctx, const pisco_launch *launch);
/*
 * Processing order of each detector's samples (the output is always in the
 * caller's order).  Tiles group 64 consecutive samples of the processing
 * order; a stream whose consecutive samples are far apart on the sky (random
 * pointings, pixel-centre patterns like the paper's benchmark) gives tiles
 * too spread for the tile path.  PISCO_ORDER_SPATIAL processes every
 * detector's samples sorted along a Hilbert curve over (phi, cos theta) (a
 * device sort at plan time, redone when the pointing changes);
 * PISCO_ORDER_AUTO (the default) does so, on the FP32 tile paths, for a
 * detector whose given order leaves more than half of its 64-sample groups
 * incoherent; PISCO_ORDER_GIVEN keeps the given order.  Results depend on the
 * order only through which samples share a tile (rounding).
 */
enum { PISCO_ORDER_GIVEN = 0, PISCO_ORDER_AUTO = 1, PISCO_ORDER_SPATIAL = 2 };
pisco_status pisco_set_ordering(pisco_ctx *ctx, int32_t mode);
pisco_status pisco_get_launch(const pisco_ctx *ctx, pisco_launch *launch);

/*
 * Kernel timing: when enabled, every convolve brackets its kernel launches
 * with HIP events on the launch stream; pisco_kernel_time reads (and
 * synchronises on) them.  total_ms = summed kernel time of the convolve calls
 * since the last reset, launches = their count.
 */
pisco_status pisco_set_timing(pisco_ctx *ctx, int on);
pisco_status pisco_kernel_time(pisco_ctx *ctx, double *total_ms, int64_t *launches, int reset);

/* ------------------------------------------------------------------------
 * Far-sidelobe surrogate network.
 *
 * The exact wide-disc convolution is the reference for a learned stand-in of
 * the far sidelobe: an MLP maps a pointing (unit vector, sin psi, cos psi) to
 * the detector-frame Stokes pickup (OUT_STOKES) of the sidelobe annulus, so
 * that TOD = exact main-beam TOD + sum_c coef[c] * pickup[c].  Weights are
 * used in BF16 with FP32 accumulation on the matrix cores; FP32 master
 * weights and Adam moments live on the device.
 *
 * Network: 5 -> [width, SiLU] x hidden_layers -> 3.  Parameters are one FP32
 * array: for each linear map l = 0..hidden_layers, W_l (rows x cols,
 * row-major, rows = output units) followed by b_l; pisco_mlp_layout gives the
 * offsets.  All data pointers below are device pointers unless `mem` says
 * otherwise; x is [n][5], targets and outputs [n][3], float32.
 * ------------------------------------------------------------------------ */
typedef struct pisco_mlp pisco_mlp;

/* width: multiple of 64 in [64, 512]; max_batch: multiple of 64 (rows per
 * internal pass); seed: initial weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
 * zero biases.  Errors are reported through pisco_last_error(ctx). */
pisco_status pisco_mlp_create(pisco_ctx *ctx, int32_t width, int32_t hidden_layers, int32_t max_batch, uint64_t seed,
                              pisco_mlp **out);
void pisco_mlp_destroy(pisco_mlp *mlp);
int64_t pisco_mlp_param_count(const pisco_mlp *mlp);
pisco_status pisco_mlp_layout(const pisco_mlp *mlp, int32_t layer, int64_t *w_offset, int64_t *b_offset,
                              int32_t *rows, int32_t *cols);
/* Replace the FP32 master weights (host or device); resets the Adam state. */
pisco_status pisco_mlp_set_params(pisco_mlp *mlp, const float *params, int mem);
pisco_status pisco_mlp_get_params(const pisco_mlp *mlp, float *params, int mem);
/* Inference with the BF16 weights, any n >= 0. */
pisco_status pisco_mlp_forward(pisco_mlp *mlp, const float *x, int64_t n, float *y, void *stream);
/* Mean squared error over the n x 3 outputs and its gradient (FP32, parameter
 * layout) for one batch, without updating; n a multiple of 64, <= max_batch. */
pisco_status pisco_mlp_gradient(pisco_mlp *mlp, const float *x, const float *targets, int32_t n, float *grad,
                                float *loss, void *stream);
/* One Adam step on that loss (bias-corrected; lr, beta1, beta2, eps as usual). */
pisco_status pisco_mlp_train_step(pisco_mlp *mlp, const float *x, const float *targets, int32_t n, float lr,
                                  float beta1, float beta2, float eps, float *loss, void *stream);
/* Features of detector `det`'s pointing: x[t] = (sin th cos ph, sin th sin ph, cos th, sin psi, cos psi). */
pisco_status pisco_sidelobe_features(pisco_ctx *ctx, int32_t det, float *x, void *stream);
/* tod[t] += sum_c coef[c] (mean[c] + stdv[c] y[t][c]) with y the network's
 * output for detector `det`'s pointing; mean, stdv (3 floats) and coef (3
 * doubles) are host arrays, tod a device float array of the detector's samples.
 * One fused launch (features, every layer and the sum on chip, no scratch
 * memory); the result equals features + pisco_mlp_forward + the sum above,
 * bit for bit.  Asynchronous on `stream`. */
pisco_status pisco_sidelobe_apply(pisco_ctx *ctx, pisco_mlp *mlp, int32_t det, const float *mean, const float *stdv,
                                  const double *coef, float *tod, void *stream);

/* ------------------------------------------------------------------------
 * Far-sidelobe surrogate of a detector, trained and used by the library.
 *
 * For a detector with a one-grid (scalar) beam b and FIXED normalisation,
 * the TOD over its disc rho <= rho_max splits exactly into the main disc
 * rho <= r_main and the annulus r_main < rho <= rho_max (Sec. 4.2: the
 * pixelated sum is additive over disjoint pixel sets).  The annulus term is
 *   sum_c coef[c] P[c],  coef = (wI, wQ cos2z - wU sin2z, wQ sin2z + wU cos2z) / wT
 * with P the annulus' Stokes pickup (OUT_STOKES) of the same beam at
 * zeta = 0 and z = zeta (the pixel angle chi grows by zeta, Appendix A).
 * P depends on the pointing only, so a network can stand in for it.
 *
 * pisco_sidelobe_train(ctx, det, r_main_rad, n_train, seed, epochs):
 *   draws n_train pointings (direction uniform on the sphere, psi uniform in
 *   [0, 2 pi), SplitMix64 outputs 3i .. 3i+2 of `seed` for pointing i),
 *   computes their exact annulus pickups P with the convolution kernels,
 *   standardises each channel (mean, sample standard deviation), and trains
 *   a network 5 -> [width, SiLU] x hidden_layers -> 3 (the network
 *   section above) on the standardised targets: `epochs` passes, each over
 *   floor(n_train / batch) * batch rows in a fresh pseudo-random order (a
 *   Feistel bijection keyed by the seed and the epoch), one Adam step per
 *   batch, the learning rate decaying from lr to lr_end along a cosine over
 *   all steps.  Runs synchronously; the detector's previous network, if any,
 *   is replaced.  Needs: a scalar beam without V weight, no plate, FIXED
 *   normalisation, wT != 0, 0 < r_main_rad < rho_max, n_train >= batch,
 *   epochs >= 1 (EINVAL otherwise; ESTATE without sky, beam or parameters).
 *   The pointing of `det` is not used (it may be unset).  Changing the
 *   detector's beam or parameters later drops the network.
 * pisco_sidelobe_enable(ctx, det, on): with on != 0 (ESTATE if untrained),
 *   OUT_TOD convolves of `det` (alone or batched) evaluate the exact sum over
 *   rho <= r_main only and add sum_c coef[c] (mean[c] + std[c] y[c]) with y the
 *   network's output for the sample's pointing (one fused launch per
 *   detector, queued after the convolution on the same stream and captured
 *   in the same graph).  OUT_STOKES and OUT_COUNT stay exact over the whole
 *   disc.  on = 0 restores the exact TOD.
 * pisco_sidelobe_share(ctx, det, src): detector `det` uses the network
 *   trained for `src` (kept alive while any detector uses it): once enabled,
 *   its OUT_TOD is the exact sum over rho <= min(its rho_max, r_main of src)
 *   with its own beam, plus the network's annulus pickup (of src's beam)
 *   weighted by its own (wI, wQ, wU) turned by its zeta, times
 *   N_det / (N_src wT_src) -- e.g. many detectors with their own main beams
 *   sharing one far-sidelobe grid.  det needs what training needs (scalar
 *   beam without V, no plate, FIXED normalisation); ESTATE if src is
 *   untrained.  Enabling stays per detector.
 * pisco_sidelobe_history: copies up to `cap` per-epoch mean training losses
 *   of the last run into `loss` (may be NULL) and returns the epoch count (0
 *   if untrained, -1 for a bad detector).
 * pisco_sidelobe_set_options: network and optimiser of later training runs
 *   (width a multiple of 64 in [64, 512], hidden_layers in [1, 16], batch a
 *   multiple of 64 in [64, 4194304], 0 < lr_end <= lr, 0 <= beta < 1,
 *   eps > 0).  Defaults: {256, 4, 8192, 2e-3, 2e-5, 0.9, 0.999, 1e-8}.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t width;
    int32_t hidden_layers;
    int32_t batch;
    float lr, lr_end;
    float beta1, beta2, eps;
} pisco_sidelobe_opts;
pisco_status pisco_sidelobe_set_options(pisco_ctx *ctx, const pisco_sidelobe_opts *opts);
pisco_status pisco_sidelobe_train(pisco_ctx *ctx, int32_t det, double r_main_rad, int64_t n_train, uint64_t seed,
                                  int32_t epochs);
pisco_status pisco_sidelobe_enable(pisco_ctx *ctx, int32_t det, int on);
pisco_status pisco_sidelobe_share(pisco_ctx *ctx, int32_t det, int32_t src);
int32_t pisco_sidelobe_history(const pisco_ctx *ctx, int32_t det, double *loss, int32_t cap);

/* ------------------------------------------------------------------------
 * Device-memory budget (the paper runs discs that overflow device memory in
 * serial blocks, Sec. 5.3).  pisco_set_memory_budget caps the device memory
 * this context allocates for its sky, beams, pointing and plate copies, work
 * queues and output staging at `bytes` (0: no cap beyond the device's).
 * When a host pointing or plate-angle stream would exceed the budget (or its
 * allocation fails), the context keeps the host copy instead; convolve then
 * streams such detectors -- and every call whose queues or output staging do
 * not fit -- through device buffers sized to the remaining budget, in blocks
 * of consecutive samples (multiples of 64, so every block starts a tile of
 * the given order and the results equal those of the resident path for
 * PISCO_ORDER_GIVEN), block after block on the call's stream, synchronously.
 * PISCO_ENOMEM is returned only when not even a 64-sample block fits.
 * Lowering the budget below what is already allocated is allowed; it applies
 * to later allocations.  pisco_memory_in_use reports the bytes counted
 * against the budget now.
 * ------------------------------------------------------------------------ */
pisco_status pisco_set_memory_budget(pisco_ctx *ctx, int64_t bytes);
int64_t pisco_memory_in_use(const pisco_ctx *ctx);

/* ------------------------------------------------------------------------
 * Binned maps from TOD: the map-making step the TOD are handed to (Sec. 5.1)
 * and from which the validation maps are made (Sec. 6).
 *
 * Measurement model of a sample t of a detector with focal-plane angle zeta,
 * response s and cross-polar leakage eps, its boresight in RING pixel p of a
 * map of nside_map (the detector row D of Sec. 4.1 at one pixel):
 *   d_t = w_t . (I, Q, U)_p,
 *   w_t = (s/2) ((1 + eps), (1 - eps) cos a_t, (1 - eps) sin a_t),
 *   a_t = 2 (psi_t + zeta) + 4 phi_t   (phi_t: half-wave-plate angle, 0 without one).
 *
 * pisco_map_accumulate adds n samples into `accum`, a caller-owned device
 * float64 array [12 nside_map^2][10]: per pixel the six distinct entries of
 * sum w w^T (00, 01, 02, 11, 12, 22), the three of sum w d, and the hit
 * count.  The caller zeroes it before the first call and may add any number of
 * detectors.  theta, phi, psi (radians) and hwp (may be null) are device
 * float64 arrays of n values, tod a device array of n PISCO_F32 or PISCO_F64
 * values (tod_dtype); all are read on `stream` (hipStream_t, NULL = default)
 * and must stay valid until the work there is done.  Samples with a non-finite
 * angle or value are skipped.  The adds are FP64 atomics: each sum is exact up
 * to the order of its additions, which is not fixed.
 *
 * pisco_map_solve: per pixel, rcond = smallest / largest eigenvalue of the
 * 3 x 3 sum.  rcond >= rcond_min: (I, Q, U) solve the 3 x 3 system;
 * 0 <= rcond < rcond_min with hits: intensity only, I = sum w_0 d / sum w_0^2,
 * Q = U = 0; no hits: 0 (rcond 0).  maps: device float64 [3][12 nside_map^2]
 * (I, Q, U rows); rcond: device float64 [12 nside_map^2], or null.
 *
 * Both return PISCO_EINVAL for nside_map not a power of two in [1, 8192], n < 0,
 * a null array that is needed, a bad dtype, non-finite zeta, eps or s, or
 * rcond_min outside [0, 1]; launches are asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
pisco_status pisco_map_accumulate(pisco_ctx *ctx, int64_t nside_map, int64_t n, const double *theta, const double *phi,
                                  const double *psi, const double *hwp, const void *tod, int tod_dtype, double zeta,
                                  double eps, double s, double *accum, void *stream);
pisco_status pisco_map_solve(pisco_ctx *ctx, int64_t nside_map, const double *accum, double rcond_min, double *maps,
                             double *rcond, void *stream);

/* ------------------------------------------------------------------------
 * Angular power spectra of I, Q, U maps: the spectrum estimation the
 * validation maps go through (Sec. 6.2), with the beam-corrected spectra
 * compared with those of the input maps.  FP64 throughout.
 *
 * Definitions.  Y_lm(theta, phi) = lambda_lm(theta) e^{i m phi}, orthonormal,
 * Condon-Shortley phase; _{+-2}Y_lm = (W_lm +- X_lm) e^{i m phi}, the spin-2
 * harmonics of Goldberg et al. (1967).  With w = 4 pi / (12 nside^2) per pixel
 * (one pass of pixel quadrature):
 *   a^T_lm = w sum_p T_p Y*_lm(p),  a^{+-2}_lm = w sum_p (Q +- iU)_p _{+-2}Y*_lm(p),
 *   a^E = -(a^2 + a^-2) / 2,  a^B = i (a^2 - a^-2) / 2
 * (Zaldarriaga & Seljak 1997; the HEALPix sign convention), and
 *   C^XY_l = (2l + 1)^-1 [Re(a^X_l0 a^Y*_l0) + 2 sum_{m=1..l} Re(a^X_lm a^Y*_lm)].
 *
 * a_lm arrays: device float64, complex interleaved (re, im), m-major packing:
 * index(l, m) = m (2 lmax + 1 - m) / 2 + l for 0 <= m <= l <= lmax,
 * pisco_alm_size(lmax) = (lmax + 1)(lmax + 2) / 2 complex values.
 *
 * pisco_map2alm: T, Q, U are device float64 RING maps of 12 nside^2 pixels
 * (Q and U both null: temperature only; alm_E and alm_B are then not
 * written and may be null).  iterations (0..16) Jacobi steps refine the pixel
 * quadrature: a <- a + map2alm(m - alm2map(a)) (each step costs one synthesis
 * and one analysis; 0 = one pass of quadrature).  `workspace` is caller-owned
 * device memory of at least pisco_map2alm_workspace_bytes(nside, lmax, pol)
 * bytes (ring Fourier sums, partial sums of the a_lm, and a residual map and
 * a_lm correction per field for the iterations: about 2.9 GB at nside 1024,
 * lmax 3071); it must not be shared by calls in flight.  mmax = lmax.
 *
 * pisco_alm2map: the synthesis T = sum a^T_lm Y_lm, Q + iU = -sum (a^E + i a^B)_lm
 * _2Y_lm over m = -l..l (a_{l,-m} = (-1)^m a*_lm) at every RING pixel centre,
 * into device float64 maps (alm_E, alm_B, Q, U all null: T only).  Same
 * workspace as pisco_map2alm.
 *
 * pisco_alm2cl: cl[l] = C^XY_l for l = 0..lmax (device float64, lmax + 1).
 *
 * pisco_anafast: pisco_map2alm into the caller's alm arrays, then the six
 * spectra TT, EE, BB, TE, EB, TB into cl [6][lmax + 1] (TT only, cl [1][lmax + 1],
 * without Q and U).
 *
 * All return PISCO_EINVAL for nside not a power of two in [1, 1024], lmax
 * outside [0, 4 nside], iterations outside [0, 16], a null array that is
 * needed, or a workspace smaller than required; launches are asynchronous on
 * `stream` (hipStream_t, NULL = default) and every array must stay valid until
 * the work there is done.
 * ------------------------------------------------------------------------ */
int64_t pisco_alm_size(int32_t lmax);
int64_t pisco_map2alm_workspace_bytes(int64_t nside, int32_t lmax, int32_t pol);
pisco_status pisco_map2alm(pisco_ctx *ctx, int64_t nside, int32_t lmax, int32_t iterations, const double *T,
                           const double *Q, const double *U, double *alm_T, double *alm_E, double *alm_B,
                           void *workspace, int64_t workspace_bytes, void *stream);
pisco_status pisco_alm2map(pisco_ctx *ctx, int64_t nside, int32_t lmax, const double *alm_T, const double *alm_E,
                           const double *alm_B, double *T, double *Q, double *U, void *workspace,
                           int64_t workspace_bytes, void *stream);
pisco_status pisco_alm2cl(pisco_ctx *ctx, int32_t lmax, const double *alm_x, const double *alm_y, double *cl,
                          void *stream);
pisco_status pisco_anafast(pisco_ctx *ctx, int64_t nside, int32_t lmax, int32_t iterations, const double *T,
                           const double *Q, const double *U, double *alm_T, double *alm_E, double *alm_B,
                           void *workspace, int64_t workspace_bytes, double *cl, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PISCO_H */
