// Contraction kernels: Y_o(c) = sum_{p<=q} Tf[o][p][q] g_p(c) g_q(c) for every cell
// (the raw flux vector of Sec. 3.3, a quadratic form in the Legendre coefficients).
//
//     Z_p(c)[o] = sum_{q>=p} Tf[o][p][q] g_q(c)     MFMA: A = T (rows o), B = cells
//     Y_o(c)   += w_p(c) Z_p(c)[o]                  VALU, FP64 accumulation
//
// A workgroup (4 waves) shares one schedule of iterations; every iteration stages
// the T fragments of two p values in LDS (double buffered, prefetched one
// iteration ahead into registers) and every wave applies them to its own tiles of
// cells, whose B operands stay in registers for the whole launch.
#include "gd_internal.h"

namespace gd {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Split FP16: 32x32x16 MFMA, tiles of 32 slots, row blocks of 32, K steps of 16.
// A lane l holds T[o = l%32][q = 16ks + 8(l/32) + j]; B lane l holds
// m[slot = l%32][q = 16ks + 8(l/32) + j]; D register r of lane l holds
// row 8(r/4) + 4(l/32) + r%4, column l%32.
template <int KSMAX, int NT>
__global__ __launch_bounds__(256) void k_contract_mixed(MixedArgs a)
{
    extern __shared__ uint4 lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile0 = (blockIdx.x * 4 + wave) * NT;
    constexpr int BUF = 2 * KSMAX * 128;   // uint4 per buffer: up to 2*KSMAX fragments of 2 KB
    const int level = a.slot_level ? a.slot_level[blockIdx.x * 4 * NT * 32] : 0;
    const IterDesc* its = a.iters + a.iter_off[level];
    const int n_it = a.iter_cnt[level];

    half8_t bh[NT][KSMAX], bl[NT][KSMAX];
    double th[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const bool tv = tile0 + t < a.n_tiles;
        const int slot = (tile0 + t) * 32 + (lane & 31);
        th[t] = (tv && a.theta && slot < a.n_slots) ? a.theta[slot] : 0.0;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            uint4 vh = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
            if (tv && ks < a.KS) {
                const size_t base = ((size_t)((tile0 + t) * a.KS + ks) * 2) * 64 + lane;
                vh = a.mfrag[base];
                vl = a.mfrag[base + 64];
            }
            bh[t][ks] = *reinterpret_cast<half8_t*>(&vh);
            bl[t][ks] = *reinterpret_cast<half8_t*>(&vl);
        }
    }

    uint4 pre[KSMAX];
    auto fetch = [&](int i) {
        const int f0 = its[i].frag, nf = its[i].nfrag;
        const uint4* src = a.frag + (size_t)f0 * 128;
#pragma unroll
        for (int r = 0; r < KSMAX; ++r) {
            const int idx = tid + 256 * r;
            if (idx < nf * 128) pre[r] = src[idx];
        }
        return nf;
    };
    auto store = [&](int buf, int nf) {
#pragma unroll
        for (int r = 0; r < KSMAX; ++r) {
            const int idx = tid + 256 * r;
            if (idx < nf * 128) lds[buf * BUF + idx] = pre[r];
        }
    };

    if (n_it > 0) store(0, fetch(0));
    __syncthreads();

    double Y[NT][16];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) Y[t][r] = 0.0;

    for (int i = 0; i < n_it; ++i) {
        const IterDesc d = its[i];
        const int buf = i & 1;
        int nf_next = 0;
        if (i + 1 < n_it) nf_next = fetch(i + 1);
        const uint4* B = lds + buf * BUF;
        int f = 0;
#pragma unroll
        for (int seg = 0; seg < 2; ++seg) {
            const int p = seg ? d.pb : d.pa;
            const unsigned long long m = seg ? d.mb : d.ma;
            if (p < 0 || m == 0) continue;
            double wp[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float mp = (tile0 + t < a.n_tiles) ? a.mt[((size_t)(tile0 + t) * a.P + p) * 32 + (lane & 31)] : 0.0f;
                wp[t] = (double)mp * (d.delta ? th[t] : 1.0);
            }
            floatx16 Z[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) Z[t][r] = 0.0f;
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks) {
                if ((m >> ks) & 1ull) {
                    uint4 uh = B[f * 128 + lane];
                    uint4 ul = B[f * 128 + 64 + lane];
                    ++f;
                    const half8_t ah = *reinterpret_cast<half8_t*>(&uh);
                    const half8_t al = *reinterpret_cast<half8_t*>(&ul);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh[t][ks], Z[t], 0, 0, 0);
                        Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl[t][ks], Z[t], 0, 0, 0);
                        Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh[t][ks], Z[t], 0, 0, 0);
                    }
                }
            }
            const double sc = a.scale[d.scale + p];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double w = wp[t] * sc;
#pragma unroll
                for (int r = 0; r < 16; ++r) Y[t][r] = fma(w, (double)Z[t][r], Y[t][r]);
            }
        }
        if (i + 1 < n_it) store(buf ^ 1, nf_next);
        __syncthreads();
        if (i + 1 == n_it || its[i + 1].ob != d.ob) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int slot = (tile0 + t) * 32 + (lane & 31);
                if (tile0 + t < a.n_tiles && slot < a.n_slots) {
                    float* dst = a.Y + (size_t)slot * a.ystride + d.ob * 32 + 4 * (lane >> 5);
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) {
                        float4 v = make_float4((float)Y[t][4 * r4], (float)Y[t][4 * r4 + 1],
                                               (float)Y[t][4 * r4 + 2], (float)Y[t][4 * r4 + 3]);
                        *reinterpret_cast<float4*>(dst + 8 * r4) = v;
                    }
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) Y[t][r] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64: 16x16x4 MFMA, tiles of 16 slots, row blocks of 16, K steps of 4.
// A lane l holds T[o = l%16][q = 4ks + l/16]; B lane l holds g[slot = l%16][q = 4ks + l/16];
// D register r of lane l holds row 4r + l/16, column l%16.
template <int KSMAX, int NT>
__global__ __launch_bounds__(256) void k_contract_fp64(F64Args a)
{
    extern __shared__ uint4 lds4[];
    double* lds = reinterpret_cast<double*>(lds4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile0 = (blockIdx.x * 4 + wave) * NT;
    constexpr int BUF = 2 * KSMAX * 64;                                 // doubles per buffer
    constexpr int PRE = (2 * KSMAX * 64 + 2 * 256 - 1) / (2 * 256);     // double2 per thread
    const int level = a.slot_level ? a.slot_level[blockIdx.x * 4 * NT * 16] : 0;
    const IterDesc* its = a.iters + a.iter_off[level];
    const int n_it = a.iter_cnt[level];

    double b[NT][KSMAX];
    double th[NT];
    int cell[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int slot = (tile0 + t) * 16 + (lane & 15);
        int c = -1;
        if (tile0 + t < a.n_tiles && slot < a.n_slots) c = a.perm ? a.perm[slot] : slot;
        cell[t] = c;
        th[t] = (c >= 0 && a.theta) ? a.theta[slot] : 0.0;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            const int q = ks * 4 + (lane >> 4);
            b[t][ks] = (c >= 0 && q < a.P) ? a.g[(size_t)c * a.P + q] : 0.0;
        }
    }

    double2 pre[PRE];
    auto fetch = [&](int i) {
        const int f0 = its[i].frag, nf = its[i].nfrag;
        const double2* src = reinterpret_cast<const double2*>(a.frag + (size_t)f0 * 64);
#pragma unroll
        for (int r = 0; r < PRE; ++r) {
            const int idx = tid + 256 * r;
            if (idx < nf * 32) pre[r] = src[idx];
        }
        return nf;
    };
    auto store = [&](int buf, int nf) {
        double2* dst = reinterpret_cast<double2*>(lds + buf * BUF);
#pragma unroll
        for (int r = 0; r < PRE; ++r) {
            const int idx = tid + 256 * r;
            if (idx < nf * 32) dst[idx] = pre[r];
        }
    };

    if (n_it > 0) store(0, fetch(0));
    __syncthreads();

    doublex4 Y[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Y[t] = doublex4{0.0, 0.0, 0.0, 0.0};

    for (int i = 0; i < n_it; ++i) {
        const IterDesc d = its[i];
        const int buf = i & 1;
        int nf_next = 0;
        if (i + 1 < n_it) nf_next = fetch(i + 1);
        const double* B = lds + buf * BUF;
        int f = 0;
#pragma unroll
        for (int seg = 0; seg < 2; ++seg) {
            const int p = seg ? d.pb : d.pa;
            const unsigned long long m = seg ? d.mb : d.ma;
            if (p < 0 || m == 0) continue;
            double gp[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gp[t] = (cell[t] >= 0) ? a.g[(size_t)cell[t] * a.P + p] : 0.0;
                if (d.delta) gp[t] *= th[t];
            }
            doublex4 Z[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) Z[t] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks) {
                if ((m >> ks) & 1ull) {
                    const double av = B[f * 64 + lane];
                    ++f;
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        Z[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[t][ks], Z[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) Y[t][r] = fma(gp[t], Z[t][r], Y[t][r]);
        }
        if (i + 1 < n_it) store(buf ^ 1, nf_next);
        __syncthreads();
        if (i + 1 == n_it || its[i + 1].ob != d.ob) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int slot = (tile0 + t) * 16 + (lane & 15);
                if (tile0 + t < a.n_tiles && slot < a.n_slots) {
                    double* dst = a.Y + (size_t)slot * a.ystride + d.ob * 16 + (lane >> 4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) dst[4 * r] = Y[t][r];
                }
                Y[t] = doublex4{0.0, 0.0, 0.0, 0.0};
            }
        }
    }
}

// ---------------------------------------------------------------------------
template <int KSMAX, int NT>
static int launch_mixed_t(const MixedArgs& a, hipStream_t s)
{
    const int blocks = cdiv(cdiv(a.n_tiles, NT), 4);
    const size_t lds = size_t(2) * 2 * KSMAX * 128 * sizeof(uint4);
    static bool attr = false;
    if (!attr && lds > 65536) {
        HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_contract_mixed<KSMAX, NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        attr = true;
    }
    if (blocks == 0) return GD_OK;
    hipLaunchKernelGGL((k_contract_mixed<KSMAX, NT>), dim3(blocks), dim3(256), lds, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

// tile shapes: NT tiles of 32 cells per wave; 2 tiles while the K steps fit the registers
int slots_per_wg_mixed(int KS) { return 4 * 32 * (KS <= 8 ? 2 : 1); }
int slots_per_wg_fp64(int KS4) { return 4 * 16 * (KS4 <= 24 ? 2 : 1); }

int launch_contract_mixed(const MixedArgs& a, hipStream_t s)
{
    if (a.KS <= 2) return launch_mixed_t<2, 2>(a, s);
    if (a.KS <= 4) return launch_mixed_t<4, 2>(a, s);
    if (a.KS <= 6) return launch_mixed_t<6, 2>(a, s);
    if (a.KS <= 8) return launch_mixed_t<8, 2>(a, s);
    if (a.KS <= 12) return launch_mixed_t<12, 1>(a, s);
    return fail(GD_EUNSUPPORTED, "P too large for the mixed contraction");
}

template <int KSMAX, int NT>
static int launch_f64_t(const F64Args& a, hipStream_t s)
{
    const int blocks = cdiv(cdiv(a.n_tiles, NT), 4);
    const size_t lds = size_t(2) * 2 * KSMAX * 64 * sizeof(double);
    static bool attr = false;
    if (!attr && lds > 65536) {
        HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_contract_fp64<KSMAX, NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        attr = true;
    }
    if (blocks == 0) return GD_OK;
    hipLaunchKernelGGL((k_contract_fp64<KSMAX, NT>), dim3(blocks), dim3(256), lds, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_contract_fp64(const F64Args& a, hipStream_t s)
{
    if (a.KS <= 8) return launch_f64_t<8, 2>(a, s);
    if (a.KS <= 16) return launch_f64_t<16, 2>(a, s);
    if (a.KS <= 24) return launch_f64_t<24, 2>(a, s);
    if (a.KS <= 32) return launch_f64_t<32, 1>(a, s);
    if (a.KS <= 48) return launch_f64_t<48, 1>(a, s);
    return fail(GD_EUNSUPPORTED, "P too large for the FP64 contraction");
}

} // namespace gd
