// Microbenchmark behind the contraction's roofline notes: the rate of back-to-back
// v_mfma_f32_32x32x16_f16 chains on gfx950, and how much FP64 or FP32 vector work on
// other waves of the same SIMDs slows them.  Registers only (one store per lane at the
// end, inside a buffer of grid x 512 floats).
//
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       -o mfma_coexec mfma_coexec.hip && ./mfma_coexec
//
// Workgroups of 8 waves, two per CU (512 workgroups): the hardware places wave w of a
// workgroup on SIMD w % 4, so waves 0-3 and waves 4-7 share the four SIMDs.
#include <hip/hip_runtime.h>
#include <cstdio>

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

enum { kMfmaLow = 1, kMfmaHigh = 2, kF64 = 4, kF32 = 8 };

// waves 0-3: MFMA chains if kMfmaLow; waves 4-7: MFMA chains if kMfmaHigh, else FP64
// (kF64) or FP32 (kF32) fused multiply-adds, 8 independent chains per lane
template <int MODE>
__global__ __launch_bounds__(512) void k_coexec(float* out, int iters, float seed)
{
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool mfma = wave < 4 ? (MODE & kMfmaLow) != 0 : (MODE & kMfmaHigh) != 0;
    float res = 0.0f;
    if (mfma) {
        half8_t a, b;
        for (int j = 0; j < 8; ++j) {
            a[j] = (_Float16)(seed * (lane + j));
            b[j] = (_Float16)(seed * (j - lane));
        }
        floatx16 z0 = {}, z1 = {};
        for (int i = 0; i < iters; ++i) {
            z0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, z0, 0, 0, 0);
            z1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(b, a, z1, 0, 0, 0);
        }
        for (int r = 0; r < 16; ++r) res += z0[r] + z1[r];
    } else if (wave >= 4 && (MODE & kF64)) {
        double x[8];
        for (int c = 0; c < 8; ++c) x[c] = seed * (lane + c);
        const double m = 1.0 - 1e-9 * seed, d = 1e-9;
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < 8; ++c) x[c] = fma(x[c], m, d);
        for (int c = 0; c < 8; ++c) res += (float)x[c];
    } else if (wave >= 4 && (MODE & kF32)) {
        float x[8];
        for (int c = 0; c < 8; ++c) x[c] = seed * (lane + c);
        const float m = 1.0f - 1e-6f * seed, d = 1e-6f;
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], m, d);
        for (int c = 0; c < 8; ++c) res += x[c];
    }
    out[(size_t)blockIdx.x * blockDim.x + tid] = res;
}

template <int MODE>
static float time_ms(float* out, int grid, int iters)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
    k_coexec<MODE><<<grid, 512>>>(out, iters, 0.001f);
    (void)hipEventRecord(e0);
    for (int r = 0; r < 5; ++r) k_coexec<MODE><<<grid, 512>>>(out, iters, 0.001f);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / 5.0f;
}

int main()
{
    const int grid = 512, iters = 4000;
    float* out = nullptr;
    if (hipMalloc(&out, sizeof(float) * grid * 512) != hipSuccess) return 1;
    const double mf = 2.0 * iters * 32768.0 * 64 / 64;      // flops of one MFMA wave (two chains)
    const double vf = 8.0 * iters * 2.0 * 64;                // flops of one vector wave
    const float m4 = time_ms<kMfmaLow>(out, grid, iters);
    const float m8 = time_ms<kMfmaLow | kMfmaHigh>(out, grid, iters);
    const float d = time_ms<kF64>(out, grid, iters), f = time_ms<kF32>(out, grid, iters);
    const float md = time_ms<kMfmaLow | kF64>(out, grid, iters), mf32 = time_ms<kMfmaLow | kF32>(out, grid, iters);
    const double w4 = grid * 4.0;
    printf("MFMA chains, 2 waves per SIMD: %.3f ms, %.1f TFLOP/s\n", m4, w4 * mf / (m4 * 1e-3) / 1e12);
    printf("MFMA chains, 4 waves per SIMD: %.3f ms, %.1f TFLOP/s\n", m8, 2 * w4 * mf / (m8 * 1e-3) / 1e12);
    printf("FP64 FMA, 2 waves per SIMD: %.3f ms, %.1f TFLOP/s\n", d, w4 * vf / (d * 1e-3) / 1e12);
    printf("FP32 FMA, 2 waves per SIMD: %.3f ms, %.1f TFLOP/s\n", f, w4 * vf / (f * 1e-3) / 1e12);
    printf("MFMA + FP64 on the same SIMDs: %.3f ms (alone %.3f + %.3f)\n", md, m4, d);
    printf("MFMA + FP32 on the same SIMDs: %.3f ms (alone %.3f + %.3f)\n", mf32, m4, f);
    (void)hipFree(out);
    return 0;
}
