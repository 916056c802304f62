// FP64 contraction: the plain double-precision form of the same contraction, on the
// 16x16x4 FP64 MFMA.
//
// Tiles of 16 slots, row blocks of 16.  A fragment covers 16 rows and one
// 16-column K step as four 4-column sub-steps: lane l, sub-step j holds
// T[o = l%16][q = 16ks + 4j + l/16] (2 KB).  B lane l holds g[slot = l%16][q = 4k + l/16];
// D register r of lane l holds row 4r + l/16, column l%16.
#include "contract_common.h"

namespace gd {

typedef double doublex4 __attribute__((ext_vector_type(4)));

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

template <int W>
struct F64Item {
    const GD_CONST GroupDev* gp;
    const double* gplan;
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
                  ntile <= W && KS == gp->KS)) {
                if (tid == 0) check_fail(gp->checks, kCheckItem);
                return;
            }
        }
        bool bad = false;   // a failed device check (GD_CHECKS): the item stops, nothing is stored
        const GD_GLOBAL uint4* frag = gptr(gp->frag);
        const GD_CONST IterDesc* iters = cptr(gp->iters);
        const GD_GLOBAL int* perm = gptr(gp->perm);
        const GD_GLOBAL double* theta = gptr(gp->theta);
        const int P = gp->P;
        const int tile = tile0 + wave;
        const int slot = tile * 16 + (lane & 15);
        int cell = -1;
        if (wave < ntile && tile < gp->tiles16 && slot < gp->n_slots) cell = perm ? perm[slot] : slot;
        if constexpr (kChecks) {
            if (cell >= gp->n_cells) {
                check_fail(gp->checks, kCheckSlot);
                cell = -1;
            }
        }
        const int ccl = cell >= 0 ? cell : 0;
        const double th = (cell >= 0 && theta) ? theta[slot] : 0.0;
        const GD_GLOBAL double* gg = gptr(gplan) + gp->val0;
        double b[4 * KS];
#pragma unroll
        for (int k4 = 0; k4 < 4 * KS; ++k4) {
            const int q = k4 * 4 + (lane >> 4);
            b[k4] = (cell >= 0 && q < P) ? gg[(size_t)cell * P + q] : 0.0;
        }
        const GD_GLOBAL double* gcell = gg + (size_t)ccl * P;
        doublex4 Y;

        auto prefetch_w = [&](const IterDesc& d, double (&gp_)[SEG]) {
#pragma unroll
            for (int s = 0; s < SEG; ++s) gp_[s] = gcell[(s < d.nseg) ? d.p[s] : 0];
        };

        auto body = [&](const IterDesc& d, const IterDesc& dn, const double (&gw)[SEG], double (&gwn)[SEG],
                        const uint4* rd, uint4* wr) {
            if constexpr (kChecks) {
                if (!desc_ok<KS>(dn)) {
                    bad = true;
                    return;
                }
            }
            dma_frags<W>(frag + (size_t)dn.frag * 128, wr, dn.nfrag, wave, lane);
            prefetch_w(dn, gwn);
            const double* rdd = reinterpret_cast<const double*>(rd);
            int f = 0;
#pragma unroll
            for (int s = 0; s < SEG; ++s) {
                if (s >= d.nseg) break;
                F64Seg<KS> seg{rdd + f * 256 + lane, b, (cell >= 0) ? gw[s] * (d.delta ? th : 1.0) : 0.0, &Y};
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
            Y = doublex4{0.0, 0.0, 0.0, 0.0};
            IterDesc dA = its[0], dB = its[1];
            double gw0[SEG], gw1[SEG];
            dma_frags<W>(frag + (size_t)dA.frag * 128, buf0, dA.nfrag, wave, lane);
            prefetch_w(dA, gw0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int i = 0; i < n_it; i += 2) {
                const IterDesc dC = its[i + 2];
                body(dA, dB, gw0, gw1, buf0, buf1);
                if (i + 1 >= n_it || bad) break;
                const IterDesc dD = its[i + 3];
                body(dB, dC, gw1, gw0, buf1, buf0);
                if (bad) break;
                dA = dC;
                dB = dD;
            }
            if (bad) return;
            if (cell >= 0) {
                GD_GLOBAL double* dst = gptr(gp->Yd) + (size_t)slot * gp->ystride + ob * 16 + (lane >> 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) dst[4 * q] = Y[q];
            }
        }
    }
};

template <int KSMAX, int W>
__global__ __launch_bounds__(64 * W) void k_contract_fp64(ContractArgs a)
{
    __shared__ uint4 buf0[frag_budget(KSMAX) * 128];
    __shared__ uint4 buf1[frag_budget(KSMAX) * 128];
    const int4 it = cptr(a.items)[blockIdx.x];
    if (it.x < 0) return;   // padding of an XCD's range
    F64Item<W> f{cptr(a.groups) + it.x, a.g, it.y, it.z & 0x3ff, (it.z >> 10) & 0x3ff, it.w, it.z >> 20, buf0, buf1};
    dispatch_ks<KSMAX>(f.gp->KS, f);
}

template <int KSMAX, int W>
static int launch(const ContractArgs& a, hipStream_t s)
{
    if (a.n_items == 0) return GD_OK;
    hipLaunchKernelGGL((k_contract_fp64<KSMAX, W>), dim3(a.n_items), dim3(64 * W), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_contract_fp64(const ContractArgs& a, int ksmax, int waves, hipStream_t s)
{
    if (waves != 4 && waves != 8) return fail(GD_EINVAL, "contraction workgroups have 4 or 8 waves");
    const bool w4 = waves == 4;
    if (ksmax <= 4) return w4 ? launch<4, 4>(a, s) : launch<4, 8>(a, s);
    if (ksmax <= 6) return w4 ? launch<6, 4>(a, s) : launch<6, 8>(a, s);
    if (ksmax <= 8) return w4 ? launch<8, 4>(a, s) : launch<8, 8>(a, s);
    if (ksmax <= 12) return w4 ? launch<12, 4>(a, s) : launch<12, 8>(a, s);
    if (ksmax <= kMaxKS) return w4 ? launch<kMaxKS, 4>(a, s) : launch<kMaxKS, 8>(a, s);
    return fail(GD_EUNSUPPORTED, "P too large for the FP64 contraction");
}

} // namespace gd
