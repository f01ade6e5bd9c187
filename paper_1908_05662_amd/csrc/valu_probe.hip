// Issue-rate probe of the vector ALU on gfx950 (a measurement program, not
// part of the library): wave64 instructions per second for independent
// chains of one instruction kind, eight chains per lane, at 16 waves per
// SIMD.  Prints one JSON object.  The plain (non-packed) FP32 FMA, add and
// multiply are measured with operands that repeat across instructions and
// with distinct operands; conversions, fract and compares, the other kinds
// of the convolution's pair loop, once each; and the FMA with one operand a
// scalar register or an inline constant (two vector-register reads instead of
// three), and in its two-operand accumulating form.  ALU-only inline assembly: no
// memory operation is issued inside an asm statement.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CH8(S) S(0) S(1) S(2) S(3) S(4) S(5) S(6) S(7)

template <int OP>
__global__ void __launch_bounds__(256) probe(float *out, int iters, float su) {
    float x[8], y[8], z[8];
    int xi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = 0.5f + k * 0.01f + threadIdx.x * 1e-6f;
        y[k] = 1.0000001f + k * 1e-9f;
        z[k] = 1e-7f * (k + 1);
        xi[k] = k + threadIdx.x;
    }
    const float a = 1.0000001f + threadIdx.x * 1e-9f, b = 1e-7f;
    for (int i = 0; i < iters; ++i) {
#define FMA_SAME(k) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[k]) : "v"(a), "v"(b));
#define FMA_DIST(k) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[k]) : "v"(y[k]), "v"(z[k]));
#define MUL(k) asm volatile("v_mul_f32 %0, %1, %0" : "+v"(x[k]) : "v"(y[k]));
#define ADD(k) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x[k]) : "v"(b));
#define CVT(k) asm volatile("v_cvt_i32_f32 %0, %1" : "=v"(xi[k]) : "v"(x[k]));
#define FRACT(k) asm volatile("v_fract_f32 %0, %0" : "+v"(x[k]));
#define CMP(k) asm volatile("v_cmp_le_f32 vcc, %0, %1" ::"v"(x[k]), "v"(a) : "vcc");
#define FMA_SGPR(k) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x[k]) : "s"(su), "v"(z[k]));
#define FMA_CONST(k) asm volatile("v_fma_f32 %0, %0, %1, 0.5" : "+v"(x[k]) : "v"(z[k]));
#define FMAC(k) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(x[k]) : "v"(y[k]), "v"(z[k]));
        if (OP == 0) { CH8(FMA_SAME) }
        if (OP == 1) { CH8(FMA_DIST) }
        if (OP == 2) { CH8(MUL) }
        if (OP == 3) { CH8(ADD) }
        if (OP == 4) { CH8(CVT) }
        if (OP == 5) { CH8(FRACT) }
        if (OP == 6) { CH8(CMP) }
        if (OP == 7) { CH8(FMA_SGPR) }
        if (OP == 8) { CH8(FMA_CONST) }
        if (OP == 9) { CH8(FMAC) }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k] + y[k] + z[k] + (float)xi[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int OP>
static double rate(float *out, int blocks, int iters) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0000001f);  // warm-up
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0000001f);  // su: an SGPR operand
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)blocks * 4 * iters * 8 / (ms * 1e-3);
}

int main() {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
    const int simds = p.multiProcessorCount * 4;
    const int blocks = simds * 16 / 4;  // 16 waves per SIMD, four waves per block
    const int iters = 50000;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * 256) != hipSuccess) return 1;
    const double clk = p.clockRate * 1e3;
    const double per4 = simds * clk / 4.0;  // one wave64 instruction per four clocks per SIMD
    const char *names[] = {"fma_repeated_operands", "fma_distinct_operands", "mul", "add", "cvt_i32_f32", "fract",
                           "cmp", "fma_sgpr_operand", "fma_inline_constant", "fmac_distinct_operands"};
    const double r[] = {rate<0>(out, blocks, iters), rate<1>(out, blocks, iters), rate<2>(out, blocks, iters),
                        rate<3>(out, blocks, iters), rate<4>(out, blocks, iters), rate<5>(out, blocks, iters),
                        rate<6>(out, blocks, iters), rate<7>(out, blocks, iters), rate<8>(out, blocks, iters),
                        rate<9>(out, blocks, iters)};
    printf("{\"device\": \"%s\", \"simds\": %d, \"clock_hz\": %.4g, \"waves_per_simd\": 16, "
           "\"unit\": \"wave64 instructions/s\", \"one_per_4_clocks\": %.4g",
           p.gcnArchName, simds, clk, per4);
    for (int i = 0; i < 10; ++i) printf(", \"%s\": [%.4g, %.3f]", names[i], r[i], r[i] / per4);
    printf("}\n");
    (void)hipFree(out);
    return 0;
}
