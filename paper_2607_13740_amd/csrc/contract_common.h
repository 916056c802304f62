// Pieces shared by the two contraction kernels (split FP16 and FP64).
//
// Both compute, for every cell c of a work item and every row o of one row block,
//
//     Z_p(c)[o] = sum_{q>=p} Tf[o][p][q] g_q(c)     MFMA: A = T rows, B = cells
//     Y_o(c)   += w_p(c) Z_p(c)[o]                  VALU, FP64 accumulation
//
// i.e. the raw flux vector Y_o(c) = sum_{p<=q} Tf[o][p][q] g_p(c) g_q(c), the
// quadratic form of Sec. 3.3 in the Legendre coefficients.  A workgroup of W waves
// walks the iteration lists of its item.  The T fragments of the next iteration
// (2 KB each) are copied global -> LDS with the LDS-DMA path one iteration ahead,
// into the other of two static LDS buffers, while the waves run the current one; the
// buffers are distinct LDS objects, so reads of one are not ordered after the DMA
// into the other.  Each wave keeps the B operands of its tile of cells in registers
// for the whole item.  Every chain start lo has its own straight-line MFMA chain,
// chosen by a uniform branch, so that accumulators never cross a branch.
#pragma once

#include "gd_internal.h"

namespace gd {

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// copy nfrag 2 KB fragments into LDS as 1 KB chunks shared out over the waves
template <int W>
__device__ __forceinline__ void dma_frags(const GD_GLOBAL uint4* src, uint4* dst, int nfrag, int wave, int lane)
{
    for (int c = wave; c < 2 * nfrag; c += W)
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

// Calls F::template item<KS>() for the runtime KS of a group, KS <= KSMAX.
template <int KSMAX, int K = 1, class F>
__device__ __forceinline__ void dispatch_ks(int ks, F& f)
{
    if constexpr (K <= KSMAX) {
        if (ks == K) f.template item<K>();
        else dispatch_ks<KSMAX, K + 1>(ks, f);
    }
}

} // namespace gd
