// Split-FP16 contraction: T and the scaled state are each carried as FP16 hi + lo
// halves; three 32x32x16 MFMA products (hi*hi, hi*lo, lo*hi) accumulate in FP32 per
// segment, and the segment sums are weighted and accumulated in FP64.
//
// Tiles of 32 slots, row blocks of 32, K steps of 16.  A lane l holds
// T[o = l%32][q = 16ks + 8(l/32) + j]; B lane l holds m[slot = l%32][q = 16ks + 8(l/32) + j];
// D register r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32.  An A
// fragment holds the hi halves of the 64 lanes, then the lo halves.
#include "contract_common.h"

namespace gd {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// One segment: the chain over the K steps LO..KS-1 for T tiles of cells at once (the
// A fragment read from LDS once per K step feeds T independent accumulators), then
// Y += w Z per tile in FP64.
template <int KS, int T>
struct MixedSeg {
    const uint4* A;                 // first fragment of the segment in LDS, + lane
    const uint4 (*bh)[KS];          // [T][KS]
    const uint4 (*bl)[KS];
    const double* w;                // [T] stage-2 weight of the lane's cell
    double (*Y)[16];                // [T][16]
    template <int LO>
    __device__ __forceinline__ void run()
    {
        floatx16 Z[T];
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) Z[t][r] = 0.0f;
#pragma unroll
        for (int ks = LO; ks < KS; ++ks) {
            const half8_t xh = __builtin_bit_cast(half8_t, A[(ks - LO) * 128]);
            const half8_t xl = __builtin_bit_cast(half8_t, A[(ks - LO) * 128 + 64]);
#pragma unroll
            for (int t = 0; t < T; ++t)
                Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xh, __builtin_bit_cast(half8_t, bh[t][ks]), Z[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < T; ++t)
                Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xh, __builtin_bit_cast(half8_t, bl[t][ks]), Z[t], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < T; ++t)
                Z[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xl, __builtin_bit_cast(half8_t, bh[t][ks]), Z[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) Y[t][r] = fma(w[t], (double)Z[t][r], Y[t][r]);
    }
};

// W waves, T consecutive tiles of 32 slots per wave.
template <int W, int T>
struct MixedItem {
    const GD_CONST GroupDev* gp;
    int r, ob0, ob1, tile0, ntile;   // ntile: tiles of the item inside its bracket
    uint4* buf0;
    uint4* buf1;

    // device checks (GD_CHECKS) of an iteration descriptor before its fragments are
    // fetched; uniform over the workgroup, as the descriptors are
    template <int KS>
    __device__ __forceinline__ bool desc_ok(const IterDesc& d) const
    {
        bool ok = d.nseg >= 0 && d.nseg <= kSegMax && d.nfrag >= 0 && d.nfrag <= frag_budget(KS) && d.frag >= 0 &&
                  (long long)d.frag + d.nfrag <= gp->n_frag;
        for (int s = 0; s < kSegMax; ++s)
            if (s < d.nseg) ok = ok && d.p[s] >= 0 && d.p[s] < gp->P && d.lo[s] >= 0 && d.lo[s] < KS;
        if (!ok && threadIdx.x == 0) check_fail(gp->checks, kCheckDesc);
        return ok;
    }

    template <int KS>
    __device__ __forceinline__ void item()
    {
        constexpr int SEG = kSegMax;
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        if constexpr (kChecks) {
            if (!(r >= 0 && r < gp->R && ob0 >= 0 && ob0 < ob1 && ob1 <= gp->NOB && tile0 >= 0 && ntile >= 0 &&
                  ntile <= W * T && KS == gp->KS)) {
                if (tid == 0) check_fail(gp->checks, kCheckItem);
                return;
            }
        }
        bool bad = false;   // a failed device check (GD_CHECKS): the item stops, nothing is stored
        const GD_GLOBAL uint4* frag = gptr(gp->frag);
        const GD_CONST IterDesc* iters = cptr(gp->iters);
        const GD_CONST float* scale = cptr(gp->scale);
        const GD_GLOBAL uint4* mfrag = gptr(gp->mfrag);
        const GD_GLOBAL double* theta = gptr(gp->theta);
        const int n_tiles = gp->tiles32, n_slots = gp->n_slots, P = gp->P;
        int slot[T];
        bool sv[T];
        double th[T];
        uint4 bh[T][KS], bl[T][KS];
        const GD_GLOBAL float* mtile[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int tile = tile0 + wave * T + t;
            const bool tv = wave * T + t < ntile && tile < n_tiles;
            const int tcl = tv ? tile : n_tiles - 1;
            slot[t] = tile * 32 + (lane & 31);
            sv[t] = tv && slot[t] < n_slots;
            th[t] = (sv[t] && theta) ? theta[slot[t]] : 0.0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const size_t base = ((size_t)(tcl * KS + ks) * 2) * 64 + lane;
                bh[t][ks] = mfrag[base];
                bl[t][ks] = mfrag[base + 64];
            }
            mtile[t] = gptr(gp->mt) + (size_t)tcl * P * 32 + (lane & 31);
        }
        double Y[T][16];

        // raw stage-2 inputs of an iteration (loads only, consumed one iteration later)
        auto prefetch_w = [&](const IterDesc& d, float (&mp)[T][SEG], float (&sc)[SEG]) {
#pragma unroll
            for (int s = 0; s < SEG; ++s) {
                const int p = (s < d.nseg) ? d.p[s] : 0;
                sc[s] = scale[d.scale + p];
#pragma unroll
                for (int t = 0; t < T; ++t) mp[t][s] = mtile[t][(size_t)p * 32];
            }
        };

        // one iteration: compute d from rd while the fragments of dn stream into wr
        auto body = [&](const IterDesc& d, const IterDesc& dn, const float (&mp)[T][SEG], const float (&sc)[SEG],
                        float (&mpn)[T][SEG], float (&scn)[SEG], const uint4* rd, uint4* wr) {
            if constexpr (kChecks) {
                if (!desc_ok<KS>(dn)) {
                    bad = true;
                    return;
                }
            }
            dma_frags<W>(frag + (size_t)dn.frag * 128, wr, dn.nfrag, wave, lane);
            prefetch_w(dn, mpn, scn);
            int f = 0;
#pragma unroll
            for (int s = 0; s < SEG; ++s) {
                if (s >= d.nseg) break;
                double w[T];
#pragma unroll
                for (int t = 0; t < T; ++t) w[t] = (double)mp[t][s] * (double)sc[s] * (d.delta ? th[t] : 1.0);
                MixedSeg<KS, T> seg{rd + f * 128 + lane, bh, bl, w, Y};
                pick_lo<KS, 0>(d.lo[s], seg);
                f += KS - d.lo[s];
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        };

        for (int ob = ob0; ob < ob1; ++ob) {
            const int list = r * gp->NOB + ob;
            const GD_CONST IterDesc* its = iters + cptr(gp->list_off)[list];
            const int n_it = cptr(gp->list_cnt)[list];
            if constexpr (kChecks) {
                // the list and the two descriptors read past its end lie inside the schedule
                const long long off = cptr(gp->list_off)[list];
                if (!(n_it >= 1 && off >= 0 && off + n_it + 2 <= gp->n_iters && desc_ok<KS>(its[0]))) {
                    if (tid == 0 && n_it >= 1) check_fail(gp->checks, kCheckDesc);
                    return;
                }
            }
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) Y[t][i] = 0.0;
            // descriptors are read two iterations ahead (every list ends with two sentinels)
            IterDesc dA = its[0], dB = its[1];
            float mp0[T][SEG], sc0[SEG], mp1[T][SEG], sc1[SEG];
            dma_frags<W>(frag + (size_t)dA.frag * 128, buf0, dA.nfrag, wave, lane);
            prefetch_w(dA, mp0, sc0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int i = 0; i < n_it; i += 2) {
                const IterDesc dC = its[i + 2];
                body(dA, dB, mp0, sc0, mp1, sc1, buf0, buf1);
                if (i + 1 >= n_it || bad) break;
                const IterDesc dD = its[i + 3];
                body(dB, dC, mp1, sc1, mp0, sc0, buf1, buf0);
                if (bad) break;
                dA = dC;
                dB = dD;
            }
            if (bad) return;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                if (!sv[t]) continue;
                GD_GLOBAL float* dst = gptr(gp->Yf) + (size_t)slot[t] * gp->ystride + ob * 32 + 4 * (lane >> 5);
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    float4 v = make_float4((float)Y[t][4 * r4], (float)Y[t][4 * r4 + 1], (float)Y[t][4 * r4 + 2],
                                           (float)Y[t][4 * r4 + 3]);
                    *reinterpret_cast<GD_GLOBAL float4*>(dst + 8 * r4) = v;
                }
            }
        }
    }
};

// two tiles per wave need ~250 registers: ask for two waves per SIMD
template <int KSMAX, int W, int T>
__global__ __launch_bounds__(64 * W, T == 2 ? 2 : 1) void k_contract_mixed(ContractArgs a)
{
    __shared__ uint4 buf0[frag_budget(KSMAX) * 128];
    __shared__ uint4 buf1[frag_budget(KSMAX) * 128];
    const int4 it = cptr(a.items)[blockIdx.x];
    if (it.x < 0) return;   // padding of an XCD's range
    MixedItem<W, T> f{cptr(a.groups) + it.x, it.y, it.z & 0x3ff, (it.z >> 10) & 0x3ff, it.w, it.z >> 20, buf0, buf1};
    dispatch_ks<KSMAX>(f.gp->KS, f);
}

template <int KSMAX, int W, int T>
static int launch(const ContractArgs& a, hipStream_t s)
{
    if (a.n_items == 0) return GD_OK;
    hipLaunchKernelGGL((k_contract_mixed<KSMAX, W, T>), dim3(a.n_items), dim3(64 * W), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

template <int KSMAX>
static int launch_ks(const ContractArgs& a, int waves, int tpw, hipStream_t s)
{
    if (waves == 4 && tpw == 1) return launch<KSMAX, 4, 1>(a, s);
    if (waves == 8 && tpw == 1) return launch<KSMAX, 8, 1>(a, s);
    if constexpr (KSMAX <= 6)
        if (waves == 4 && tpw == 2) return launch<KSMAX, 4, 2>(a, s);
    return fail(GD_EINVAL, "split contraction variants: 4 or 8 waves with 1 tile per wave, or 4 waves with 2 "
                           "(P <= 96)");
}

int launch_contract_mixed(const ContractArgs& a, int ksmax, int waves, int tpw, hipStream_t s)
{
    if (ksmax <= 4) return launch_ks<4>(a, waves, tpw, s);
    if (ksmax <= 6) return launch_ks<6>(a, waves, tpw, s);
    if (ksmax <= 8) return launch_ks<8>(a, waves, tpw, s);
    if (ksmax <= 12) return launch_ks<12>(a, waves, tpw, s);
    if (ksmax <= kMaxKS) return launch_ks<kMaxKS>(a, waves, tpw, s);
    return fail(GD_EUNSUPPORTED, "P too large for the mixed contraction");
}

} // namespace gd
