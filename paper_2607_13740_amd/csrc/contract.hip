// Contraction kernels: Y_o(c) = sum_{p<=q} Tf[o][p][q] g_p(c) g_q(c) for every cell
// (the raw flux vector of Sec. 3.3, a quadratic form in the Legendre coefficients).
//
//     Z_p(c)[o] = sum_{q>=p} Tf[o][p][q] g_q(c)     MFMA: A = T (rows o), B = cells
//     Y_o(c)   += w_p(c) Z_p(c)[o]                  VALU, FP64 accumulation
//
// A workgroup (8 waves) walks one schedule of iterations.  Each iteration carries up
// to SEG p values of one row block.  Its T fragments (2 KB each) are copied
// global -> LDS by the LDS-DMA path (global_load_lds_dwordx4) one iteration ahead
// into the other of two static LDS buffers, together with the next descriptor and
// stage-2 weights, while the waves run the current iteration.  The two buffers are
// distinct LDS objects so that reads of one are not ordered after the DMA into the
// other.  Each wave keeps the B operands of its tile of cells in registers for
// the whole launch.  A segment covers the K steps lo..KS-1 of one p; every lo has
// its own straight-line MFMA chain, selected by uniform branches, so that
// accumulators never cross a branch.  Workgroups are numbered XCD by XCD so
// that the cells of one XCD (and the tensor levels they use) share one L2.
#include "gd_internal.h"

namespace gd {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// Hardware dispatches workgroup b to XCD b % 8.  Renumber so that XCD x runs a
// contiguous range of logical workgroups.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int xcd = b & 7, idx = b >> 3;
    const int q = n >> 3, r = n & 7;
    return xcd * q + min(xcd, r) + idx;
}

// copy nfrag 2 KB fragments into LDS as 1 KB chunks shared out over the waves
__device__ __forceinline__ void dma_frags(const uint4* src, uint4* dst, int nfrag, int wave, int lane, int nwaves)
{
    for (int c = wave; c < 2 * nfrag; c += nwaves)
        __builtin_amdgcn_global_load_lds((gbl_ptr_t)(src + c * 64 + lane), (lds_ptr_t)(dst + c * 64), 16, 0, 0);
}

// Uniform dispatch on lo to a compile-time chain F::run<LO> (segments run to the last K step).
template <int KS, int LO, class F>
__device__ __forceinline__ void pick_lo(int lo, F& f)
{
    if constexpr (LO < KS) {
        if (lo == LO) f.template run<LO>();
        else pick_lo<KS, LO + 1>(lo, f);
    }
}

constexpr int kWaves = 8;   // waves per workgroup, one tile of cells each

// ---------------------------------------------------------------------------
// Split FP16: 32x32x16 MFMA, tiles of 32 slots, row blocks of 32, K steps of 16.
// A lane l holds T[o = l%32][q = 16ks + 8(l/32) + j]; B lane l holds
// m[slot = l%32][q = 16ks + 8(l/32) + j]; D register r of lane l holds
// row 8(r/4) + 4(l/32) + r%4, column l%32.  A fragment: hi halves of the 64 lanes,
// then lo halves.
template <int KS>
struct MixedSeg {
    const uint4* A;                 // first fragment of the segment in LDS, + lane
    const uint4* bh;                // [KS]
    const uint4* bl;
    double w;                       // stage-2 weight of the lane's cell
    double* Y;                      // [16]
    template <int LO>
    __device__ __forceinline__ void run()
    {
        floatx16 Z;
#pragma unroll
        for (int r = 0; r < 16; ++r) Z[r] = 0.0f;
#pragma unroll
        for (int ks = LO; ks < KS; ++ks) {
            const half8_t xh = __builtin_bit_cast(half8_t, A[(ks - LO) * 128]);
            const half8_t xl = __builtin_bit_cast(half8_t, A[(ks - LO) * 128 + 64]);
            const half8_t mh = __builtin_bit_cast(half8_t, bh[ks]);
            const half8_t ml = __builtin_bit_cast(half8_t, bl[ks]);
            Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(xh, mh, Z, 0, 0, 0);
            Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(xh, ml, Z, 0, 0, 0);
            Z = __builtin_amdgcn_mfma_f32_32x32x16_f16(xl, mh, Z, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Y[r] = fma(w, (double)Z[r], Y[r]);
    }
};

template <int KS>
__global__ __launch_bounds__(64 * kWaves) void k_contract_mixed(MixedArgs a)
{
    constexpr int SEG = (KS <= 8) ? 4 : 2;
    constexpr int BUF = SEG * KS * 128;   // uint4 per buffer
    __shared__ uint4 buf0[BUF];
    __shared__ uint4 buf1[BUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = wg * kWaves + wave;
    const int level = a.slot_level ? a.slot_level[wg * kWaves * 32] : 0;
    const IterDesc* its = a.iters + a.iter_off[level];
    const int n_it = a.iter_cnt[level];

    const bool tv = tile < a.n_tiles;
    const int tcl = min(tile, a.n_tiles - 1);
    const int slot = tile * 32 + (lane & 31);
    const double th = (tv && a.theta && slot < a.n_slots) ? a.theta[slot] : 0.0;
    uint4 bh[KS], bl[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const size_t base = ((size_t)(tcl * KS + ks) * 2) * 64 + lane;
        bh[ks] = a.mfrag[base];
        bl[ks] = a.mfrag[base + 64];
    }
    const float* mtile = a.mt + (size_t)tcl * a.P * 32 + (lane & 31);

    double Y[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) Y[r] = 0.0;

    // raw stage-2 inputs of an iteration (loads only, consumed one iteration later)
    auto prefetch_w = [&](const IterDesc& d, float (&mp)[SEG], float (&sc)[SEG]) {
#pragma unroll
        for (int s = 0; s < SEG; ++s) {
            const int p = (s < d.nseg) ? d.p[s] : 0;
            sc[s] = a.scale[d.scale + p];
            mp[s] = mtile[(size_t)p * 32];
        }
    };

    // one iteration: compute d from rd while the fragments of dn stream into wr
    auto body = [&](const IterDesc& d, const IterDesc& dn, const float (&mp)[SEG], const float (&sc)[SEG],
                    float (&mpn)[SEG], float (&scn)[SEG], const uint4* rd, uint4* wr) {
        dma_frags(a.frag + (size_t)dn.frag * 128, wr, dn.nfrag, wave, lane, kWaves);
        prefetch_w(dn, mpn, scn);
        int f = 0;
#pragma unroll
        for (int s = 0; s < SEG; ++s) {
            if (s >= d.nseg) break;
            MixedSeg<KS> seg{rd + f * 128 + lane, bh, bl,
                             (double)mp[s] * (double)sc[s] * (d.delta ? th : 1.0), Y};
            pick_lo<KS, 0>(d.lo[s], seg);
            f += KS - d.lo[s];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (dn.ob != d.ob) {
            if (tv && slot < a.n_slots) {
                float* dst = a.Y + (size_t)slot * a.ystride + d.ob * 32 + 4 * (lane >> 5);
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    float4 v = make_float4((float)Y[4 * r4], (float)Y[4 * r4 + 1], (float)Y[4 * r4 + 2],
                                           (float)Y[4 * r4 + 3]);
                    *reinterpret_cast<float4*>(dst + 8 * r4) = v;
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) Y[r] = 0.0;
        }
    };

    // descriptors are loaded two iterations ahead (each level ends with two sentinels)
    IterDesc dA = its[0], dB = its[1];
    float mp0[SEG], sc0[SEG], mp1[SEG], sc1[SEG];
    dma_frags(a.frag + (size_t)dA.frag * 128, buf0, dA.nfrag, wave, lane, kWaves);
    prefetch_w(dA, mp0, sc0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int i = 0; i < n_it; i += 2) {
        const IterDesc dC = its[i + 2];
        body(dA, dB, mp0, sc0, mp1, sc1, buf0, buf1);
        if (i + 1 >= n_it) break;
        const IterDesc dD = its[i + 3];
        body(dB, dC, mp1, sc1, mp0, sc0, buf1, buf0);
        dA = dC;
        dB = dD;
    }
}

// ---------------------------------------------------------------------------
// FP64: 16x16x4 MFMA, tiles of 16 slots, row blocks of 16.  A fragment covers 16
// rows and one 16-column K step as four 4-column sub-steps: lane l, sub-step j holds
// T[o = l%16][q = 16ks + 4j + l/16] (2 KB).  B lane l holds g[slot = l%16][q = 4k + l/16];
// D register r of lane l holds row 4r + l/16, column l%16.
template <int KS>
struct F64Seg {
    const double* A;                 // first fragment of the segment in LDS, + lane
    const double* b;                 // [4 KS]
    double w;
    doublex4* Y;
    template <int LO>
    __device__ __forceinline__ void run()
    {
        doublex4 Z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = LO; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                Z = __builtin_amdgcn_mfma_f64_16x16x4f64(A[((ks - LO) * 4 + j) * 64], b[ks * 4 + j], Z, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) (*Y)[r] = fma(w, Z[r], (*Y)[r]);
    }
};

template <int KS>
__global__ __launch_bounds__(64 * kWaves) void k_contract_fp64(F64Args a)
{
    constexpr int SEG = (KS <= 8) ? 4 : 2;
    constexpr int BUF = SEG * KS * 128;   // uint4 per buffer
    __shared__ uint4 buf0[BUF];
    __shared__ uint4 buf1[BUF];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = wg * kWaves + wave;
    const int level = a.slot_level ? a.slot_level[wg * kWaves * 16] : 0;
    const IterDesc* its = a.iters + a.iter_off[level];
    const int n_it = a.iter_cnt[level];

    const int slot = tile * 16 + (lane & 15);
    int cell = -1;
    if (tile < a.n_tiles && slot < a.n_slots) cell = a.perm ? a.perm[slot] : slot;
    const int ccl = cell >= 0 ? cell : 0;
    const double th = (cell >= 0 && a.theta) ? a.theta[slot] : 0.0;
    double b[4 * KS];
#pragma unroll
    for (int k4 = 0; k4 < 4 * KS; ++k4) {
        const int q = k4 * 4 + (lane >> 4);
        b[k4] = (cell >= 0 && q < a.P) ? a.g[(size_t)cell * a.P + q] : 0.0;
    }
    const double* gcell = a.g + (size_t)ccl * a.P;

    doublex4 Y = {0.0, 0.0, 0.0, 0.0};

    auto prefetch_w = [&](const IterDesc& d, double (&gp)[SEG]) {
#pragma unroll
        for (int s = 0; s < SEG; ++s) gp[s] = gcell[(s < d.nseg) ? d.p[s] : 0];
    };

    auto body = [&](const IterDesc& d, const IterDesc& dn, const double (&gp)[SEG], double (&gpn)[SEG],
                    const uint4* rd, uint4* wr) {
        dma_frags(a.frag + (size_t)dn.frag * 128, wr, dn.nfrag, wave, lane, kWaves);
        prefetch_w(dn, gpn);
        const double* rdd = reinterpret_cast<const double*>(rd);
        int f = 0;
#pragma unroll
        for (int s = 0; s < SEG; ++s) {
            if (s >= d.nseg) break;
            F64Seg<KS> seg{rdd + f * 256 + lane, b, (cell >= 0) ? gp[s] * (d.delta ? th : 1.0) : 0.0, &Y};
            pick_lo<KS, 0>(d.lo[s], seg);
            f += KS - d.lo[s];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (dn.ob != d.ob) {
            if (cell >= 0) {
                double* dst = a.Y + (size_t)slot * a.ystride + d.ob * 16 + (lane >> 4);
#pragma unroll
                for (int r = 0; r < 4; ++r) dst[4 * r] = Y[r];
            }
            Y = doublex4{0.0, 0.0, 0.0, 0.0};
        }
    };

    IterDesc dA = its[0], dB = its[1];
    double gp0[SEG], gp1[SEG];
    dma_frags(a.frag + (size_t)dA.frag * 128, buf0, dA.nfrag, wave, lane, kWaves);
    prefetch_w(dA, gp0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int i = 0; i < n_it; i += 2) {
        const IterDesc dC = its[i + 2];
        body(dA, dB, gp0, gp1, buf0, buf1);
        if (i + 1 >= n_it) break;
        const IterDesc dD = its[i + 3];
        body(dB, dC, gp1, gp0, buf1, buf0);
        dA = dC;
        dB = dD;
    }
}

// ---------------------------------------------------------------------------
int segs_per_iter(int KS) { return KS <= 8 ? 4 : 2; }
int slots_per_wg(int rows) { return kWaves * (rows == 32 ? 32 : 16); }

template <class Args, class Kern>
static int launch_generic(Kern kern, const Args& a, hipStream_t s)
{
    const int blocks = cdiv(a.n_tiles, kWaves);
    if (blocks == 0) return GD_OK;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * kWaves), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

#define GD_KS_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

int launch_contract_mixed(const MixedArgs& a, hipStream_t s)
{
    switch (a.KS) {
#define GD_CASE(K) case K: return launch_generic(&k_contract_mixed<K>, a, s);
        GD_KS_CASES(GD_CASE)
#undef GD_CASE
    }
    return fail(GD_EUNSUPPORTED, "P too large for the mixed contraction");
}

int launch_contract_fp64(const F64Args& a, hipStream_t s)
{
    switch (a.KS) {
#define GD_CASE(K) case K: return launch_generic(&k_contract_fp64<K>, a, s);
        GD_KS_CASES(GD_CASE)
#undef GD_CASE
    }
    return fail(GD_EUNSUPPORTED, "P too large for the FP64 contraction");
}

} // namespace gd
