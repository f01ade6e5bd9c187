// Far-sidelobe surrogate network on gfx950: BF16 weights and activations,
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Network: x (5) -> [Linear + SiLU] x L -> Linear -> y (3), hidden width H.
// Input features are the pointing unit vector and (sin psi, cos psi); the
// outputs are the standardised Stokes pickup of the far sidelobe.
//
// Kernels
//   in_fwd      layer 0 (K = 5) on the vector ALU: Z1 = X W0^T + b0, A1 = SiLU(Z1)
//   gemm        H x H layers on MFMA, three operand layouts:
//                 FWD   Z = A W^T + b -> Z (fp32), SiLU(Z) (bf16)
//                 BWD_D dZ_prev = (dZ W) * SiLU'(Z_prev)   (bf16)
//                 BWD_W partial dW = dZ^T A over one batch slice (fp32, split-K)
//   out_rows    output layer (N = 3): Y, MSE loss, dY, dZ_L = (dY W_out) * SiLU'(Z_L)
//   wcolsum     per-block partial weighted column sums: the bias gradients,
//               dW0 = dZ1^T X and dW_out = dY^T A_L (with db_out)
//   reduce_many fixed-order sums of the partials (deterministic gradients)
//   adam        Adam on FP32 master weights, refreshing the BF16 copy
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mlp_internal.h"

namespace pisco {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// SiLU and its derivative with the hardware exponential and reciprocal
// (about 1 ulp); z -> -inf gives -0, z -> +inf gives z.
__device__ inline float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float silu_grad(float z) {
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// ----------------------------------------------------------------------
// GEMM: C[M x N] = A[M x K] B[K x N] with both operands k-contiguous: A[m][k]
// at a[m*lda + k] and B given by rows n, B(k, n) at b[n*ldb + k] (so the
// layers' backward passes read transposed copies the forward epilogues,
// the output layer and Adam keep).  M, N multiples of the tile (64 or 128),
// K of 32.  Workgroup: four waves as 2 x 2, each (BM/2) x (BN/2) of
// v_mfma_f32_16x16x32_bf16 tiles; 64-wide k steps staged in LDS, double
// buffered (the next step's tiles are fetched into registers while the
// current step's MFMAs run; k past the end of the slice reads as zero and its
// MFMAs are skipped).  Every output element is one MFMA chain over k0 = 0, 32,
// 64, ... with lane l holding k0 + 8 (l / 16) .. + 7 of row l % 16: the
// fragments and order of the fused inference kernel.
// ----------------------------------------------------------------------
constexpr int TK = 32;                 // k per MFMA
constexpr int KS = 64, LDK = KS + 8;   // k per staged step; LDS rows padded by 16 bytes

enum { EPI_FWD = MLP_EPI_FWD, EPI_BWD_D = MLP_EPI_BWD_D, EPI_BWD_W = MLP_EPI_BWD_W };

struct GemmArgs {
    const __bf16 *a;
    const __bf16 *b;
    int64_t lda, ldb;
    int32_t M, N, K;
    int32_t k_slice;       // split-K slice length (multiple of 32)
    const float *bias;     // FWD
    float *z_out;          // FWD: pre-activation (ldc = N)
    __bf16 *a_out;         // FWD: SiLU(Z); BWD_D: dZ_prev (ldc = N)
    __bf16 *t_out;         // optional transposed copy of a_out: t_out[n * ldt + m]
    int64_t ldt;
    const float *z_prev;   // BWD_D: pre-activation of the previous layer
    float *partial;        // BWD_W: [slice][M][N]
};

// Rows [r0, r0 + R) x k [k0, k0 + KS) of a k-contiguous operand: R * KS / 8
// chunks of 16 bytes, CH per thread of 256; chunks at k >= ke read as zero.
template <int R>
struct TileRegs {
    static constexpr int CPR = KS / 8;            // chunks per row
    static constexpr int CH = R * CPR / 256;
    bf16x8 v[CH];
    __device__ inline void load(const __bf16 *__restrict__ p, int64_t ld, int r0, int k0, int ke, int tid) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int idx = tid + 256 * c, r = idx / CPR, kk = (idx % CPR) * 8;
            if (k0 + kk < ke) v[c] = *reinterpret_cast<const bf16x8 *>(p + (int64_t)(r0 + r) * ld + (k0 + kk));
            else v[c] = bf16x8{};
        }
    }
    __device__ inline void store(__bf16 (*dst)[LDK], int tid) const {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int idx = tid + 256 * c, r = idx / CPR, kk = (idx % CPR) * 8;
            *reinterpret_cast<bf16x8 *>(&dst[r][kk]) = v[c];
        }
    }
};

template <int EPI, int BM, int BN>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    constexpr int WM = BM / 2, WN = BN / 2, FI = WM / 16, FJ = WN / 16;
    __shared__ __align__(16) __bf16 As[2][BM][LDK];
    __shared__ __align__(16) __bf16 Bs[2][BN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kb = blockIdx.z * g.k_slice, ke = min(g.K, kb + g.k_slice);
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[FI][FJ];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    TileRegs<BM> ra;
    TileRegs<BN> rb;
    if (kb < ke) {
        ra.load(g.a, g.lda, m0, kb, ke, tid);
        rb.load(g.b, g.ldb, n0, kb, ke, tid);
        ra.store(As[0], tid);
        rb.store(Bs[0], tid);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += KS) {
        const bool more = k0 + KS < ke;
        if (more) {
            ra.load(g.a, g.lda, m0, k0 + KS, ke, tid);
            rb.load(g.b, g.ldb, n0, k0 + KS, ke, tid);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ks += TK) {
            if (k0 + ks >= ke) break;
            bf16x8 af[FI], bfr[FJ];
#pragma unroll
            for (int i = 0; i < FI; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(&As[cur][wm + 16 * i + r][ks + kq]);
#pragma unroll
            for (int j = 0; j < FJ; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][wn + 16 * j + r][ks + kq]);
#pragma unroll
            for (int i = 0; i < FI; ++i)
#pragma unroll
                for (int j = 0; j < FJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            ra.store(As[cur ^ 1], tid);
            rb.store(Bs[cur ^ 1], tid);
        }
        __syncthreads();
        cur ^= 1;
    }

    // epilogue: lane holds C[row0 + 4 (lane/16) + q][col0 + lane%16], q = 0..3
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int rowb = m0 + wm + 16 * i + 4 * (lane >> 4);
            const int col = n0 + wn + 16 * j + (lane & 15);
            __bf16 t4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = rowb + q;
                const float v = acc[i][j][q];
                const int64_t o = (int64_t)row * g.N + col;
                if (EPI == EPI_FWD) {
                    const float z = v + g.bias[col];
                    g.z_out[o] = z;
                    t4[q] = (__bf16)silu(z);
                    g.a_out[o] = t4[q];
                } else if (EPI == EPI_BWD_D) {
                    t4[q] = (__bf16)(v * silu_grad(g.z_prev[o]));
                    g.a_out[o] = t4[q];
                } else {
                    g.partial[(int64_t)blockIdx.z * g.M * g.N + o] = v;
                }
            }
            // four consecutive rows of one column: one 8-byte store into the transposed copy
            if (EPI != EPI_BWD_W && g.t_out) {
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                *reinterpret_cast<bf16x4 *>(g.t_out + (int64_t)col * g.ldt + rowb) = bf16x4{t4[0], t4[1], t4[2], t4[3]};
            }
        }
}

// dst[c * ldd + r] = src[r * lds + c] for an R x C bf16 matrix (both multiples of
// 64), 64 x 64 tiles through LDS; grid.z walks a batch of matrices (strides sz, dz).
__global__ void __launch_bounds__(256) transpose_kernel(const __bf16 *src, int64_t lds, __bf16 *dst, int64_t ldd,
                                                        int64_t sz, int64_t dz) {
    __shared__ __bf16 t[64][66];
    src += blockIdx.z * sz;
    dst += blockIdx.z * dz;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 16; ++k) t[ty * 16 + k][tx] = src[(int64_t)(r0 + ty * 16 + k) * lds + c0 + tx];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[(int64_t)(c0 + ty * 16 + k) * ldd + r0 + tx] = t[tx][ty * 16 + k];
}

// ----------------------------------------------------------------------
// Small layers and reductions
// ----------------------------------------------------------------------
// Layer 0: one thread per (row, unit).  W0 is [H][5] (bf16-rounded).
__global__ void in_fwd_kernel(const float *x, const __bf16 *w0, const float *b0, int32_t n, int32_t H, float *z,
                              __bf16 *a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * H) return;
    const int64_t r = i / H;
    const int u = (int)(i % H);
    float s = b0[u];
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) s = fmaf(x[r * MLP_IN + k], (float)w0[u * MLP_IN + k], s);
    if (z) z[i] = s;
    a[i] = (__bf16)silu(s);
}

// Output layer: `rows` consecutive rows per wave, lanes over the H units
// (H % 64 == 0, H <= 512).  Per row, y_c = sum_u a_u W_out[c][u] + b_c as a
// per-lane FMA chain over u = lane + 64 k followed by an xor butterfly (the
// order the fused inference kernel repeats).  With targets it also writes
// dY = 2 (y - t) / count (fp32, for the weight-gradient sums), dZ_L =
// (dY W_out) * SiLU'(Z_L) (bf16) and the wave's sum of squared errors.
__global__ void out_rows_kernel(const __bf16 *a, const float *zL, const __bf16 *wout, const float *bout, int32_t n,
                                int32_t H, float *y, const float *tgt, float inv_count, float *dy_out, __bf16 *dz,
                                float *part_loss, int32_t waves, int32_t rows) {
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wv >= waves) return;
    const int per = H / 64;
    float gl = 0.0f;
    for (int64_t r = wv * rows; r < min((int64_t)n, (wv + 1) * rows); ++r) {
        float av[8], s[MLP_OUT] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < per; ++k) {
            const int u = lane + 64 * k;
            av[k] = (float)a[r * H + u];
#pragma unroll
            for (int c = 0; c < MLP_OUT; ++c) s[c] = fmaf(av[k], (float)wout[c * H + u], s[c]);
        }
#pragma unroll
        for (int c = 0; c < MLP_OUT; ++c) {
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) s[c] += __shfl_xor(s[c], m, 64);
            s[c] += bout[c];
        }
        if (lane == 0)
            for (int c = 0; c < MLP_OUT; ++c) y[r * MLP_OUT + c] = s[c];
        if (!tgt) continue;
        float dy[MLP_OUT];
#pragma unroll
        for (int c = 0; c < MLP_OUT; ++c) {
            const float e = s[c] - tgt[r * MLP_OUT + c];
            gl += e * e;
            dy[c] = 2.0f * e * inv_count;
        }
        if (lane == 0)
            for (int c = 0; c < MLP_OUT; ++c) dy_out[r * MLP_OUT + c] = dy[c];
        for (int k = 0; k < per; ++k) {
            const int u = lane + 64 * k;
            float da = 0.0f;
#pragma unroll
            for (int c = 0; c < MLP_OUT; ++c) da = fmaf(dy[c], (float)wout[c * H + u], da);
            dz[r * H + u] = (__bf16)(da * silu_grad(zL[r * H + u]));
        }
    }
    if (tgt && lane == 0) part_loss[wv] = gl;  // lane 0 saw every row's error (the sums were reduced)
}

// Weighted column sums over blocks of MLP_WCOL_ROWS rows.  Block (b, slab)
// writes, for the columns u of its 512-column slab (thread t: u = 512 slab +
// 2t, 2t + 1),
//   part[b * stride + u * su + k * sk] = sum_r w(r, k) m[r][u]   (rows in order)
// with w(r, k) = wt[r K + k], or 1 when wt is null (K = 1); with `ones` set,
// block b also writes ones[b K + k] = sum_r w(r, k).  The block's rows are
// loaded before any is added, so their loads are in flight together.
template <int K>
__global__ void __launch_bounds__(256) wcolsum_kernel(const __bf16 *m, const float *wt, int32_t n, int32_t H,
                                                      float *part, int64_t stride, int32_t su, int32_t sk,
                                                      float *ones) {
    constexpr int R = MLP_WCOL_ROWS;
    const int u0 = blockIdx.y * 512 + 2 * threadIdx.x;
    const bool act = u0 < H;   // H is even
    const int64_t r0 = (int64_t)blockIdx.x * R;
    uint32_t mv[R];   // two bf16 per row, low half first
#pragma unroll
    for (int q = 0; q < R; ++q)
        mv[q] = (act && r0 + q < n) ? *reinterpret_cast<const uint32_t *>(m + (r0 + q) * H + u0) : 0u;
    float s0[K], s1[K], so[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s0[k] = s1[k] = so[k] = 0.0f;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (r0 + q >= n) break;
        float w[K];
#pragma unroll
        for (int k = 0; k < K; ++k) w[k] = wt ? wt[(r0 + q) * K + k] : 1.0f;
        const float m0 = __uint_as_float(mv[q] << 16), m1 = __uint_as_float(mv[q] & 0xffff0000u);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            s0[k] = fmaf(w[k], m0, s0[k]);
            s1[k] = fmaf(w[k], m1, s1[k]);
            so[k] += w[k];
        }
    }
    float *pb = part + (int64_t)blockIdx.x * stride;
    if (act) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pb[(int64_t)u0 * su + (int64_t)k * sk] = s0[k];
            pb[(int64_t)(u0 + 1) * su + (int64_t)k * sk] = s1[k];
        }
    }
    if (ones && blockIdx.y == 0 && threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) ones[(int64_t)blockIdx.x * K + k] = so[k];
    }
}

// Fixed-order sums of several partial arrays in one launch: out[i] = sum over
// slices j = 0, 1, ... of part[j * count + i], for the segment blockIdx.y.  A
// segment with G slice groups (G divides 256) gives each block 256 / G outputs;
// thread (o, g) adds slices g, g + G, ... in order, then group 0 adds the G
// group sums in order g = 0, 1, ...: the same result on every run.
__global__ void __launch_bounds__(256) reduce_many_kernel(MlpReduceList L) {
    __shared__ float red[256];
    const MlpReduceSeg &sg = L.seg[blockIdx.y];
    const int G = sg.groups, OB = 256 / G;
    const int o = threadIdx.x % OB, g = threadIdx.x / OB;
    const int64_t chunks = (sg.count + OB - 1) / OB;
    for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const int64_t i = c * OB + o;
        float s = 0.0f;
        if (i < sg.count)
            for (int j = g; j < sg.slices; j += G) s += sg.part[(int64_t)j * sg.count + i];
        red[threadIdx.x] = s;
        __syncthreads();
        if (g == 0 && i < sg.count) {
            float t = red[o];
            for (int q = 1; q < G; ++q) t += red[q * OB + o];
            sg.out[i] = t;
        }
        __syncthreads();
    }
}

// Adam on FP32 master weights (bias-corrected step size given), BF16 copy refreshed.
__global__ void adam_kernel(float *w, float *m, float *v, const float *g, __bf16 *wb, int64_t count, float lr_t,
                            float b1, float b2, float eps, float inv_bc2_sqrt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr_t * mi / (sqrtf(vi) * inv_bc2_sqrt + eps);
    w[i] = wi;
    wb[i] = (__bf16)wi;
}

__global__ void to_bf16_kernel(const float *w, __bf16 *wb, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) wb[i] = (__bf16)w[i];
}

// Sum of the per-wave squared errors in a fixed order: thread t adds entries
// t, t + 256, ... in order, then a tree over the 256 partial sums.
__global__ void __launch_bounds__(256) loss_sum_kernel(const float *part, int32_t count, float inv_count, float *loss) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    float s = 0.0f;
    for (int i = t; i < count; i += 256) s += part[i];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) *loss = red[0] * inv_count;
}

// Features of a pointing stream: (sin th cos ph, sin th sin ph, cos th, sin psi, cos psi).
__global__ void features_kernel(const double *th, const double *ph, const double *ps, int64_t n, float *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double st, ct, sf, cf, sp, cp;
    sincos(th[i], &st, &ct);
    sincos(ph[i], &sf, &cf);
    sincos(ps[i], &sp, &cp);
    x[i * 5 + 0] = (float)(st * cf);
    x[i * 5 + 1] = (float)(st * sf);
    x[i * 5 + 2] = (float)ct;
    x[i * 5 + 3] = (float)sp;
    x[i * 5 + 4] = (float)cp;
}

// tod[i] += sum_c coef[c] (mean[c] + std[c] y[i][c])
__global__ void apply_kernel(const float *y, int64_t n, float m0, float m1, float m2, float s0, float s1, float s2,
                             double c0, double c1, double c2, float *tod) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p0 = m0 + (double)s0 * y[i * 3 + 0];
    const double p1 = m1 + (double)s1 * y[i * 3 + 1];
    const double p2 = m2 + (double)s2 * y[i * 3 + 2];
    tod[i] = (float)((double)tod[i] + c0 * p0 + c1 * p1 + c2 * p2);
}

// ----------------------------------------------------------------------
// Fused inference with the TOD epilogue: 64 RB pointings per workgroup of H/64
// waves, wave w owning units 64 w .. 64 w + 63 of every hidden layer.
// Features, layer 0, the H x H layers, the output layer and
// tod += sum_c coef_c (mean_c + std_c y_c) stay on chip: one activation
// buffer in LDS, updated in place (each layer's products are formed in
// registers, then, after a barrier, its activations overwrite its input),
// weights read from L2.  At most 128 registers per lane, so that four waves
// share a SIMD.  The H x H layers use the operand fragments and K order of
// gemm_kernel, layer 0 the FMA chain of in_fwd_kernel, the output layer the
// per-lane order and butterfly of out_rows_kernel and the epilogue
// apply_kernel's arithmetic, so the result equals the layer-by-layer forward
// pass followed by apply, bit for bit.
// ----------------------------------------------------------------------
constexpr int XLD = 8;        // feature row stride in LDS (floats)
constexpr int WD = 2;         // k steps of weight fragments in flight

__device__ inline void features_of(const double *th, const double *ph, const double *ps, int64_t i, float *f) {
    double st, ct, sf, cf, sp, cp;
    sincos(th[i], &st, &ct);
    sincos(ph[i], &sf, &cf);
    sincos(ps[i], &sp, &cp);
    f[0] = (float)(st * cf);
    f[1] = (float)(st * sf);
    f[2] = (float)ct;
    f[3] = (float)sp;
    f[4] = (float)cp;
}

// The wave's 64 units of an H x H layer for the 64 RB rows in LDS, as Z^T = W A^T:
// the weights are the MFMA's first operand (lane l: unit u0 + 16 i + l % 16,
// k0 + 8 (l / 16) .. + 7, from L2), the activations its second (row 16 j +
// l % 16, the same k, from LDS), so each output element is the training
// GEMM's product chain over k0 = 0, 32, ... with the operands exchanged.  The
// weight fragments of WD k steps are in flight (a ring of register slots,
// refilled as each is used); every weight fragment serves 4 RB row tiles, so
// more rows per workgroup read the weights from L2 fewer times per row.
// acc[i][j]: lane l holds units u0 + 16 i + 4 (l / 16) .. + 3 of row 16 j + l % 16.
template <int RB>
__device__ inline void hxh_products(const __bf16 *__restrict__ W, const __bf16 *act, int H, int LD, int u0, int lane,
                                    f32x4 (&acc)[4][4 * RB]) {
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4 * RB; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const __bf16 *wrow = W + (int64_t)(u0 + r16) * H + kq;
    bf16x8 wf[WD][4];
#pragma unroll
    for (int sl = 0; sl < WD; ++sl)
#pragma unroll
        for (int i = 0; i < 4; ++i) wf[sl][i] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * i * H + 32 * sl);
    for (int k0 = 0; k0 < H; k0 += WD * 32) {
#pragma unroll
        for (int sl = 0; sl < WD; ++sl) {
            const int kc = k0 + 32 * sl;
#pragma unroll
            for (int j = 0; j < 4 * RB; ++j) {
                const bf16x8 af = *reinterpret_cast<const bf16x8 *>(act + (16 * j + r16) * LD + kc + kq);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[sl][i], af, acc[i][j], 0, 0, 0);
            }
            const int kn = kc + WD * 32;
            if (kn < H) {
#pragma unroll
                for (int i = 0; i < 4; ++i) wf[sl][i] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * i * H + kn);
            }
        }
    }
}

// bias, SiLU and the wave's activations into the buffer (one 8-byte store
// per four consecutive units of a row)
template <int RB>
__device__ inline void hxh_store(const float *__restrict__ bias, __bf16 *act, int LD, int u0, int lane,
                                 const f32x4 (&acc)[4][4 * RB]) {
    const int r16 = lane & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int ub = u0 + 16 * i + 4 * (lane >> 4);   // this lane's four units
        const float4 bq = *reinterpret_cast<const float4 *>(bias + ub);
#pragma unroll
        for (int j = 0; j < 4 * RB; ++j) {
            const int row = 16 * j + r16;
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const bf16x4 o = bf16x4{(__bf16)silu(acc[i][j][0] + bq.x), (__bf16)silu(acc[i][j][1] + bq.y),
                                    (__bf16)silu(acc[i][j][2] + bq.z), (__bf16)silu(acc[i][j][3] + bq.w)};
            *reinterpret_cast<bf16x4 *>(act + row * LD + ub) = o;
        }
    }
}

// NW = H / 64 waves (and 64-unit groups) per workgroup, 64 RB rows.  RB = 1:
// at most 128 registers per lane (four waves per SIMD); RB = 2: 256 (two).
template <int NW, int RB>
__global__ void __launch_bounds__(64 * NW, RB == 1 ? 4 : 2) infer_kernel(MlpInferArgs g) {
    constexpr int H = 64 * NW, LD = H + 8, IR = 64 * RB;
    extern __shared__ __align__(16) unsigned char lds[];
    float *X = reinterpret_cast<float *>(lds);
    __bf16 *act = reinterpret_cast<__bf16 *>(lds + IR * XLD * sizeof(float));
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int u0 = 64 * wave;
    const int64_t r0 = (int64_t)blockIdx.x * IR;

    for (int r = tid; r < IR; r += 64 * NW) {
        float f[MLP_IN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (r0 + r < g.n) features_of(g.th, g.ph, g.ps, r0 + r, f);
#pragma unroll
        for (int k = 0; k < MLP_IN; ++k) X[r * XLD + k] = f[k];
    }
    __syncthreads();

    // layer 0 (K = 5) on the vector ALU: lane r of wave w forms rows r, r + 64, ..
    // of units 64 w .. 64 w + 63 (wave-uniform weights), eight units per 16-byte store
    for (int rb = 0; rb < RB; ++rb) {
        const int row = 64 * rb + lane;
        float xr[MLP_IN];
#pragma unroll
        for (int k = 0; k < MLP_IN; ++k) xr[k] = X[row * XLD + k];
        // the wave's 320 BF16 weights as 32-bit words (wave-uniform, so scalar
        // loads; the offset of layer 0 and 5 u0 are even): BF16 k of unit u is
        // the high or low half of word (5 u + k) / 2
        const uint32_t *__restrict__ w0 =
            reinterpret_cast<const uint32_t *>(g.wb + g.off_w[0] + (int64_t)u0 * MLP_IN);
        const float *__restrict__ b0 = g.w + g.off_b[0] + u0;
        for (int q = 0; q < 8; ++q) {
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int u = 8 * q + e;
                float sv = b0[u];
#pragma unroll
                for (int k = 0; k < MLP_IN; ++k) {
                    const int i = u * MLP_IN + k;
                    const uint32_t wd = w0[i >> 1];
                    sv = fmaf(xr[k], __uint_as_float((i & 1) ? (wd & 0xffff0000u) : (wd << 16)), sv);
                }
                o[e] = (__bf16)silu(sv);
            }
            *reinterpret_cast<bf16x8 *>(act + row * LD + u0 + 8 * q) = o;
        }
    }
    __syncthreads();

    // H x H layers, in place: every wave's products from the whole input,
    // then (after the barrier) its units' activations over that input
    for (int l = 1; l < g.L; ++l) {
        f32x4 acc[4][4 * RB];
        hxh_products<RB>(g.wb + g.off_w[l], act, H, LD, u0, lane, acc);
        __syncthreads();
        hxh_store<RB>(g.w + g.off_b[l], act, LD, u0, lane, acc);
        __syncthreads();
    }

    // output layer (N = 3): wave w takes rows 4 w .. 4 w + 3, 4 (w + NW) ..,
    // four at a time; lanes over units, the weights held in registers
    const __bf16 *__restrict__ Wo = g.wb + g.off_w[g.L];
    const float *__restrict__ bo = g.w + g.off_b[g.L];
    float wo[NW][MLP_OUT];
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
        for (int c = 0; c < MLP_OUT; ++c) wo[k][c] = (float)Wo[c * H + lane + 64 * k];
    for (int rb = 4 * wave; rb < IR; rb += 4 * NW) {
        float sc[4][MLP_OUT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < MLP_OUT; ++c) sc[q][c] = 0.0f;
#pragma unroll
        for (int k = 0; k < NW; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float av = (float)act[(rb + q) * LD + lane + 64 * k];
#pragma unroll
                for (int c = 0; c < MLP_OUT; ++c) sc[q][c] = fmaf(av, wo[k][c], sc[q][c]);
            }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < MLP_OUT; ++c) sc[q][c] += __shfl_xor(sc[q][c], m, 64);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = r0 + rb + q;
                if (i < g.n) {
                    const double p0 = g.mean[0] + (double)g.stdv[0] * (sc[q][0] + bo[0]);
                    const double p1 = g.mean[1] + (double)g.stdv[1] * (sc[q][1] + bo[1]);
                    const double p2 = g.mean[2] + (double)g.stdv[2] * (sc[q][2] + bo[2]);
                    g.tod[i] = (float)((double)g.tod[i] + g.coef[0] * p0 + g.coef[1] * p1 + g.coef[2] * p2);
                }
            }
        }
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ----------------------------------------------------------------------
// Launch wrappers
// ----------------------------------------------------------------------
hipError_t mlp_in_fwd(const float *x, const __bf16 *w0, const float *b0, int32_t n, int32_t H, float *z, __bf16 *a,
                      hipStream_t s) {
    const int64_t tot = (int64_t)n * H;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(in_fwd_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, s, x, w0, b0, n, H, z, a);
    return hipGetLastError();
}

// 128 x 128 tiles only when they still give two workgroups per CU (512);
// otherwise 64 x 64 tiles, four times as many workgroups to hide the load
// latency of these short-K products.
template <int EPI>
static void gemm_launch(const GemmArgs &g, hipStream_t s) {
    const int64_t z = (g.K + g.k_slice - 1) / g.k_slice;
    const bool big = g.M % 128 == 0 && g.N % 128 == 0 && (int64_t)(g.M / 128) * (g.N / 128) * z >= 512;
    const int t = big ? 128 : 64;
    const dim3 grid(g.N / t, g.M / t, (unsigned)z);
    if (big) hipLaunchKernelGGL((gemm_kernel<EPI, 128, 128>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_kernel<EPI, 64, 64>), grid, dim3(256), 0, s, g);
}

hipError_t mlp_gemm(int epi, const __bf16 *a, int64_t lda, const __bf16 *b, int64_t ldb, int32_t M, int32_t N,
                    int32_t K, int32_t k_slice, const float *bias, float *z_out, __bf16 *a_out, __bf16 *t_out,
                    int64_t ldt, const float *z_prev, float *partial, hipStream_t s) {
    if (M % 64 || N % 64 || K % TK || k_slice % KS || k_slice <= 0) return hipErrorInvalidValue;
    GemmArgs g;
    g.a = a;
    g.b = b;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.k_slice = k_slice;
    g.bias = bias;
    g.z_out = z_out;
    g.a_out = a_out;
    g.t_out = t_out;
    g.ldt = ldt;
    g.z_prev = z_prev;
    g.partial = partial;
    if (epi == EPI_FWD) gemm_launch<EPI_FWD>(g, s);
    else if (epi == EPI_BWD_D) gemm_launch<EPI_BWD_D>(g, s);
    else gemm_launch<EPI_BWD_W>(g, s);
    return hipGetLastError();
}

hipError_t mlp_transpose(const __bf16 *src, int64_t lds, __bf16 *dst, int64_t ldd, int32_t R, int32_t C,
                         int32_t batch, int64_t src_stride, int64_t dst_stride, hipStream_t s) {
    if (R % 64 || C % 64) return hipErrorInvalidValue;
    if (R == 0 || C == 0 || batch == 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_kernel, dim3(C / 64, R / 64, batch), dim3(256), 0, s, src, lds, dst, ldd,
                       src_stride, dst_stride);
    return hipGetLastError();
}

hipError_t mlp_reduce_many(const MlpReduceList &l, hipStream_t s) {
    if (l.n <= 0) return hipSuccess;
    int64_t mx = 0;
    for (int i = 0; i < l.n; ++i) {
        const int G = l.seg[i].groups;
        if (G < 1 || G > 256 || 256 % G || l.seg[i].slices < 0) return hipErrorInvalidValue;
        mx = std::max<int64_t>(mx, (l.seg[i].count + 256 / G - 1) / (256 / G));
    }
    if (mx == 0) return hipSuccess;
    const unsigned bx = (unsigned)std::min<int64_t>(4096, mx);
    hipLaunchKernelGGL(reduce_many_kernel, dim3(bx, l.n), dim3(256), 0, s, l);
    return hipGetLastError();
}

hipError_t mlp_out(const __bf16 *a, const float *zL, const __bf16 *wout, const float *bout, int32_t n, int32_t H,
                   float *y, const float *tgt, float inv_count, float *dy, __bf16 *dz, float *part_loss,
                   int32_t waves, int32_t rows_per_wave, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (H % 64 || H > 512) return hipErrorInvalidValue;
    const int wpb = 4;
    hipLaunchKernelGGL(out_rows_kernel, dim3((unsigned)((waves + wpb - 1) / wpb)), dim3(64 * wpb), 0, s, a, zL, wout,
                       bout, n, H, y, tgt, inv_count, dy, dz, part_loss, waves, rows_per_wave);
    return hipGetLastError();
}

hipError_t mlp_wcolsum(const __bf16 *m, const float *wt, int32_t K, int32_t n, int32_t H, float *part, int64_t stride,
                       int32_t su, int32_t sk, float *ones, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (H % 2 || (!wt && K != 1)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + MLP_WCOL_ROWS - 1) / MLP_WCOL_ROWS), (unsigned)((H + 511) / 512));
    switch (K) {
    case 1: hipLaunchKernelGGL(wcolsum_kernel<1>, grid, dim3(256), 0, s, m, wt, n, H, part, stride, su, sk, ones);
        break;
    case 3: hipLaunchKernelGGL(wcolsum_kernel<3>, grid, dim3(256), 0, s, m, wt, n, H, part, stride, su, sk, ones);
        break;
    case 5: hipLaunchKernelGGL(wcolsum_kernel<5>, grid, dim3(256), 0, s, m, wt, n, H, part, stride, su, sk, ones);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t mlp_adam(float *w, float *m, float *v, const float *g, __bf16 *wb, int64_t count, float lr_t, float b1,
                    float b2, float eps, float inv_bc2_sqrt, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, w, m, v, g, wb, count, lr_t, b1, b2,
                       eps, inv_bc2_sqrt);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float *w, __bf16 *wb, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, w, wb, count);
    return hipGetLastError();
}

hipError_t mlp_loss_sum(const float *part, int32_t count, float inv_count, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, part, count, inv_count, loss);
    return hipGetLastError();
}

hipError_t mlp_features(const double *th, const double *ph, const double *ps, int64_t n, float *x, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, th, ph, ps, n, x);
    return hipGetLastError();
}

// rows per workgroup: 128 from width 256 up (each weight fragment then serves
// eight row tiles, halving the L2 reads per row: 8.35 -> 6.0 ms at 512 x 10 and
// 0.92 -> 0.84 ms at 256 x 4 over 1e6 pointings), 64 below
template <int NW>
static hipError_t infer_launch(const MlpInferArgs &a, hipStream_t s) {
    constexpr int RB = NW >= 4 ? 2 : 1, IR = 64 * RB;
    const size_t lds = (size_t)IR * XLD * sizeof(float) + (size_t)IR * (64 * NW + 8) * sizeof(__bf16);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&infer_kernel<NW, RB>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((infer_kernel<NW, RB>), dim3(blocks_for(a.n, IR)), dim3(64 * NW), lds, s, a);
    return hipGetLastError();
}

hipError_t mlp_infer_apply(const MlpInferArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (a.off_w[0] % 2) return hipErrorInvalidValue;   // layer 0 is read as 32-bit words
    switch (a.H) {
    case 64: return infer_launch<1>(a, s);
    case 128: return infer_launch<2>(a, s);
    case 192: return infer_launch<3>(a, s);
    case 256: return infer_launch<4>(a, s);
    case 320: return infer_launch<5>(a, s);
    case 384: return infer_launch<6>(a, s);
    case 448: return infer_launch<7>(a, s);
    case 512: return infer_launch<8>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t mlp_apply(const float *y, int64_t n, const float *mean, const float *stdv, const double *coef, float *tod,
                     hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(apply_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, y, n, mean[0], mean[1], mean[2],
                       stdv[0], stdv[1], stdv[2], coef[0], coef[1], coef[2], tod);
    return hipGetLastError();
}

}  // namespace pisco
