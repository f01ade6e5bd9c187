// Internal declarations of the sidelobe-network kernels (mlp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_IN 5
#define MLP_OUT 3

namespace pisco {

enum { MLP_EPI_FWD = 0, MLP_EPI_BWD_D = 1, MLP_EPI_BWD_W = 2 };
#define MLP_MAX_L 16

// Fused inference + TOD epilogue over a pointing stream (infer_kernel).
struct MlpInferArgs {
    const double *th, *ph, *ps;  // pointing, n samples
    int64_t n;
    int32_t H, L;                // width, hidden layers
    const __bf16 *wb;            // bf16 parameter copy (weights used from it)
    const float *w;              // fp32 parameters (biases used from it)
    int64_t off_w[MLP_MAX_L + 1], off_b[MLP_MAX_L + 1];
    float mean[3], stdv[3];
    double coef[3];
    float *tod;
};

hipError_t mlp_in_fwd(const float *x, const __bf16 *w0, const float *b0, int32_t n, int32_t H, float *z, __bf16 *a,
                      hipStream_t s);
// C = A B with A[m][k] at a[m*lda + k] and B(k, n) at b[n*ldb + k]; epilogues as
// in mlp_kernels.hip (t_out, if not null, receives the transposed bf16 output).
hipError_t mlp_gemm(int epi, const __bf16 *a, int64_t lda, const __bf16 *b, int64_t ldb, int32_t M, int32_t N,
                    int32_t K, int32_t k_slice, const float *bias, float *z_out, __bf16 *a_out, __bf16 *t_out,
                    int64_t ldt, const float *z_prev, float *partial, hipStream_t s);
// dst[c * ldd + r] = src[r * lds + c] (R, C multiples of 64), for `batch` matrices.
hipError_t mlp_transpose(const __bf16 *src, int64_t lds, __bf16 *dst, int64_t ldd, int32_t R, int32_t C,
                         int32_t batch, int64_t src_stride, int64_t dst_stride, hipStream_t s);
// Fixed-order sums of several partial arrays in one launch.
#define MLP_MAX_SEGS 40
struct MlpReduceSeg {
    const float *part;
    float *out;
    int64_t count;
    int32_t slices;
    int32_t groups;   // slices summed in parallel groups (divides 256), combined in order
};
struct MlpReduceList {
    MlpReduceSeg seg[MLP_MAX_SEGS];
    int32_t n;
};
hipError_t mlp_reduce_many(const MlpReduceList &l, hipStream_t s);
hipError_t mlp_out(const __bf16 *a, const float *zL, const __bf16 *wout, const float *bout, int32_t n, int32_t H,
                   float *y, const float *tgt, float inv_count, float *dy, __bf16 *dz, float *part_loss,
                   int32_t waves, int32_t rows_per_wave, hipStream_t s);
// part[b * stride + u * su + k * sk] = sum over the rows r of block b (MLP_WCOL_ROWS
// rows each) of w(r, k) m[r][u], w(r, k) = wt[r K + k] or 1 (wt null, K = 1);
// ones[b K + k] = sum_r w(r, k) when given.  K in {1, 3, 5}.
#define MLP_WCOL_ROWS 32
hipError_t mlp_wcolsum(const __bf16 *m, const float *wt, int32_t K, int32_t n, int32_t H, float *part, int64_t stride,
                       int32_t su, int32_t sk, float *ones, hipStream_t s);
hipError_t mlp_adam(float *w, float *m, float *v, const float *g, __bf16 *wb, int64_t count, float lr_t, float b1,
                    float b2, float eps, float inv_bc2_sqrt, hipStream_t s);
hipError_t mlp_to_bf16(const float *w, __bf16 *wb, int64_t count, hipStream_t s);
hipError_t mlp_loss_sum(const float *part, int32_t count, float inv_count, float *loss, hipStream_t s);
hipError_t mlp_features(const double *th, const double *ph, const double *ps, int64_t n, float *x, hipStream_t s);
hipError_t mlp_infer_apply(const MlpInferArgs &a, hipStream_t s);
hipError_t mlp_apply(const float *y, int64_t n, const float *mean, const float *stdv, const double *coef, float *tod,
                     hipStream_t s);

}  // namespace pisco
