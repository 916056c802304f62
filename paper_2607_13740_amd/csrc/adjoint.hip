// Reverse mode of the SSP-RK3 collision step (the adjoint): the vector-Jacobian
// product of the raw flux vector, the scaling limiter and the stage combinations,
// all in FP64.
//
// With Y_o(g) = sum_{p<=q} Tf[o][p][q] g_p g_q (Sec. 3.3) and a cotangent nu on Y,
//     G_p = d(nu . Y)/dg_p = sum_{q>=p} M_p[q] g_q + sum_{q<=p} M_q[p] g_q,
//     M_p[q] = sum_o nu_o Tf[o][p][q]                       (q >= p).
// The contraction computes the tiles M_p[q-block] (rows q, K = o, cells as columns)
// on the FP64 MFMA and reduces each tile twice: over its rows against g_q (the
// first sum, a partial per q block) and into per-row accumulators weighted by g_p
// (the second sum).  By Euler's theorem for the quadratic form,
// nu . Y = (1/2) g . G, which gives the derivative with respect to the per-cell
// kernel scale without another contraction; the level-difference part of a
// blended operator gives the derivative with respect to the blend weight,
// sum_p g_p sum_q M^diff_p[q] g_q.
#include <algorithm>

#include "bin_poly.h"
#include "contract_common.h"

namespace gd {

typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------- VJP contraction
template <int KS>
struct AdjSeg {
    const double* A;         // first fragment of the segment in LDS, + lane
    const double* b;         // [4 KS] nu of the lane's cell
    doublex4* Z;
    template <int LO>
    __device__ __forceinline__ void run()
    {
        doublex4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = LO; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                z = __builtin_amdgcn_mfma_f64_16x16x4f64(A[((ks - LO) * 4 + j) * 64], b[ks * 4 + j], z, 0, 0, 0);
        *Z = z;
    }
};

template <int W>
struct AdjItem {
    const GD_CONST GroupDev* gp;
    const double* gplan;
    int r, ob0, ob1, tile0, ntile;   // ntile: tiles of the item inside its bracket
    uint4* buf0;
    uint4* buf1;

    template <int KS>
    __device__ __forceinline__ void item()
    {
        constexpr int SEG = kSegMax;
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const GD_GLOBAL uint4* frag = gptr(gp->afrag);
        const GD_CONST IterDesc* iters = cptr(gp->aiters);
        const GD_GLOBAL int* perm = gptr(gp->perm);
        const GD_GLOBAL double* theta = gptr(gp->theta);
        const int P = gp->P, n_slots = gp->n_slots, NQB = gp->NQB, NPS = gp->NPS;
        const int tile = tile0 + wave;
        const int col = lane & 15, rsub = lane >> 4;
        const int slot = tile * 16 + col;
        int cell = -1;
        if (wave < ntile && tile < gp->tiles16 && slot < n_slots) cell = perm ? perm[slot] : slot;
        const int ccl = cell >= 0 ? cell : 0;
        const double th = (cell >= 0 && theta) ? theta[slot] : 0.0;
        const GD_GLOBAL double* gcell = gptr(gplan) + gp->val0 + (size_t)ccl * P;
        // B operand: the cotangent nu of the lane's cell, K = output row o
        double b[4 * KS];
        {
            const GD_GLOBAL double* nu = gptr(gp->nu) + (size_t)(cell >= 0 ? slot : 0) * (KS * 16);
#pragma unroll
            for (int k4 = 0; k4 < 4 * KS; ++k4) b[k4] = (cell >= 0) ? nu[k4 * 4 + rsub] : 0.0;
        }
        GD_GLOBAL double* G1p = gptr(gp->G1p);
        doublex4 G2;
        double yq[4];
        double dth;

        auto prefetch_w = [&](const IterDesc& d, double (&gw)[SEG]) {
#pragma unroll
            for (int s = 0; s < SEG; ++s) gw[s] = gcell[(s < d.nseg) ? d.p[s] : 0];
        };

        auto body = [&](const IterDesc& d, const IterDesc& dn, const double (&gw)[SEG], double (&gwn)[SEG],
                        const uint4* rd, uint4* wr, int qb) {
            dma_frags<W>(frag + (size_t)dn.frag * 128, wr, dn.nfrag, wave, lane);
            prefetch_w(dn, gwn);
            const double* rdd = reinterpret_cast<const double*>(rd);
            const double pw = d.delta ? th : 1.0;
            int f = 0;
#pragma unroll
            for (int s = 0; s < SEG; ++s) {
                if (s >= d.nseg) break;
                doublex4 z = {0.0, 0.0, 0.0, 0.0};
                AdjSeg<KS> seg{rdd + f * 256 + lane, b, &z};
                pick_lo<KS, 0>(d.lo[s], seg);
                f += KS - d.lo[s];
                const double w = (cell >= 0) ? gw[s] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) G2[q] = fma(pw * w, z[q], G2[q]);
                double t = yq[0] * z[0] + yq[1] * z[1] + yq[2] * z[2] + yq[3] * z[3];
                t += __shfl_xor(t, 16);
                t += __shfl_xor(t, 32);
                if (rsub == 0 && cell >= 0)
                    G1p[(((size_t)d.delta * NQB + qb) * n_slots + slot) * P + d.p[s]] = pw * t;
                if (d.delta) dth = fma(w, t, dth);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        };

        for (int ob = ob0; ob < ob1; ++ob) {
            const int qb = ob / NPS, ps = ob - qb * NPS;
            const int list = r * NQB * NPS + ob;
            const GD_CONST IterDesc* its = iters + cptr(gp->alist_off)[list];
            const int n_it = cptr(gp->alist_cnt)[list];
            G2 = doublex4{0.0, 0.0, 0.0, 0.0};
            dth = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int qq = qb * 16 + 4 * q + rsub;
                yq[q] = (cell >= 0 && qq < P) ? gcell[qq] : 0.0;
            }
            IterDesc dA = its[0], dB = its[1];
            double gw0[SEG], gw1[SEG];
            dma_frags<W>(frag + (size_t)dA.frag * 128, buf0, dA.nfrag, wave, lane);
            prefetch_w(dA, gw0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            for (int i = 0; i < n_it; i += 2) {
                const IterDesc dC = its[i + 2];
                body(dA, dB, gw0, gw1, buf0, buf1, qb);
                if (i + 1 >= n_it) break;
                const IterDesc dD = its[i + 3];
                body(dB, dC, gw1, gw0, buf1, buf0, qb);
                dA = dC;
                dB = dD;
            }
            if (cell >= 0) {
                GD_GLOBAL double* g2 = gptr(gp->G2) + ((size_t)ps * n_slots + slot) * P;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int qq = qb * 16 + 4 * q + rsub;
                    if (qq < P) g2[qq] = G2[q];
                }
                if (rsub == 0) gptr(gp->Dth)[((size_t)ps * NQB + qb) * n_slots + slot] = dth;
            }
        }
    }
};

template <int KSMAX, int W>
__global__ __launch_bounds__(64 * W) void k_adjoint_fp64(ContractArgs a)
{
    __shared__ uint4 buf0[frag_budget(KSMAX) * 128];
    __shared__ uint4 buf1[frag_budget(KSMAX) * 128];
    const int4 it = cptr(a.items)[blockIdx.x];
    if (it.x < 0) return;
    AdjItem<W> f{cptr(a.groups) + it.x, a.g, it.y, it.z & 0x3ff, (it.z >> 10) & 0x3ff, it.w, it.z >> 20, buf0, buf1};
    dispatch_ks<KSMAX>(f.gp->KSO, f);
}

template <int KSMAX, int W>
static int launch_adj(const ContractArgs& a, hipStream_t s)
{
    if (a.n_items == 0) return GD_OK;
    hipLaunchKernelGGL((k_adjoint_fp64<KSMAX, W>), dim3(a.n_items), dim3(64 * W), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_adjoint_fp64(const ContractArgs& a, int ksomax, hipStream_t s)
{
    if (ksomax <= 6) return launch_adj<6, kAdjWaves>(a, s);
    if (ksomax <= 12) return launch_adj<12, kAdjWaves>(a, s);
    if (ksomax <= kMaxKS) return launch_adj<kMaxKS, kAdjWaves>(a, s);
    return fail(GD_EUNSUPPORTED, "too many output rows for the adjoint contraction");
}

// ---------------------------------------------------------------------------- per-bin pieces
__device__ __forceinline__ int cdiv_dev(int a, int b) { return (a + b - 1) / b; }

// Cotangent through the limiter of one bin (1 <= k <= 4), from the limited state y and the
// factor gamma the forward limiter applied (y_i = gamma z_i for i >= 1, y_0 = z_0):
//   gamma = 1: identity;  gamma = 0 (flattened bin): the higher coefficients get 0;
//   else, with q = sum_{i>=1} z_i P_i(x*) at the minimiser x* (so gamma = -z_0/q and,
//   by the envelope theorem, dq/dz_i = P_i(x*)) and S = sum_{i>=1} lam_i z_i:
//   mu_0 = lam_0 - S/q,   mu_j = gamma lam_j + S z_0 P_j(x*) / q^2.
// Both are evaluated on u = z / z_0 (scale free: q/z_0 = sum u_i P_i(x*) <= -1), so
// that bins holding 1e-250 of the mass do not underflow q^2.  lam is updated in place.
__device__ __forceinline__ void limiter_vjp(int k, double gam, const GD_GLOBAL double* y, double* lam)
{
    if (gam == 1.0) return;
    if (gam == 0.0) {
        for (int i = 1; i <= k; ++i) lam[i] = 0.0;
        return;
    }
    double u[kMaxOrder + 1] = {1.0};
    for (int i = 1; i <= k; ++i) u[i] = (y[i] / gam) / y[0];
    double xs;
    bin_min(k, u, &xs);
    double qt = 0.0, St = 0.0;
    for (int i = 1; i <= k; ++i) {
        qt += u[i] * leg(i, xs);
        St += lam[i] * u[i];
    }
    if (!(qt < 0.0)) return;   // cannot happen for 0 < gamma < 1
    const double l0 = lam[0] - St / qt;
    for (int i = 1; i <= k; ++i) lam[i] = gam * lam[i] + St * leg(i, xs) / (qt * qt);
    lam[0] = l0;
}

// The per-slot work between two vector-Jacobian contractions of the reverse step, in
// one kernel per RK stage boundary (see AdjStageArgs):
//  C. (combine) lam = mu + s G, G_p = G2_p + the first-sum partials of every q block
//     (both parts) of the previous contraction, linearised at ylin; dkscale +=
//     (1/2) ylin . G; dvfrag += s (sum of the blend partials) dtheta/dv.  Without
//     combine, lam = mu.
//  1. lam <- J_limiter^T lam per bin (when the limiter factors are given); with out,
//     lam is the result and goes there; else acc (=|+=) a lam, prev (=|+=) b lam and
//  2. nu = A^T (b dt lam) in slot order, where A is the assembly of Eq. evo:
//     L_{j,i} = (2i+1)/h_j (V_{j,i} - F_{j+1} + (-1)^i F_j).
// One workgroup per kAdjSlots slots (a quarter of a 32-slot tile); lam of these slots
// is staged in LDS between the phases.
template <int PMAX>
__global__ __launch_bounds__(kAdjThreads) void k_adj_boundary(AdjStageArgs a)
{
    constexpr int SUB = 32 / kAdjSlots;
    constexpr int MAXNQB = (PMAX + 15) / 16, MAXNPS = (PMAX + kAdjPs - 1) / kAdjPs;   // q blocks, p ranges
    __shared__ double sl_lam[kAdjSlots * PMAX];
    __shared__ double red[kAdjSlots * PMAX];   // per-coefficient terms of the kernel-scale gradient
    const GD_CONST GroupDev* groups = cptr(a.groups);
    const int tile_all = (int)blockIdx.x / SUB, s0 = ((int)blockIdx.x % SUB) * kAdjSlots;
    int gi = 0;
    while (gi + 1 < a.n_groups && tile_all >= groups[gi + 1].tile_off) ++gi;
    const GD_CONST GroupDev* G = groups + gi;
    const int tile = tile_all - G->tile_off;
    const int N = G->N, k = G->k, K1 = k + 1, P = G->P, n_out = G->n_out, nus = G->KSO * 16;
    const int NQB = G->NQB, n_slots = G->n_slots;
    const bool conservative = G->conservative != 0, blend = G->R > 1;
    const GD_CONST double* h = cptr(G->h);
    const GD_GLOBAL int* perm = gptr(G->perm);
    const GD_GLOBAL double* mu = gptr(a.mu) + G->val0;
    const GD_GLOBAL double* gamma = a.gamma ? gptr(a.gamma) + G->gam0 : nullptr;
    const GD_GLOBAL double* ylim = a.ylim ? gptr(a.ylim) + G->val0 : nullptr;
    const GD_GLOBAL double* ylin = a.ylin ? gptr(a.ylin) + G->val0 : nullptr;
    const GD_GLOBAL double* kscale = a.kscale ? gptr(a.kscale) + G->cell0 : nullptr;
    GD_GLOBAL double* out = a.out ? gptr(a.out) + G->val0 : nullptr;
    GD_GLOBAL double* acc = a.acc ? gptr(a.acc) + G->val0 : nullptr;
    GD_GLOBAL double* prev = a.prev ? gptr(a.prev) + G->val0 : nullptr;

    // ---- phase C: one thread per (slot, coefficient)
    const GD_GLOBAL double* G2 = gptr(G->G2);
    const GD_GLOBAL double* G1p = gptr(G->G1p);
    for (int t = threadIdx.x; t < kAdjSlots * P; t += blockDim.x) {
        const int sl = t / P, p = t - sl * P;
        const int s = tile * 32 + s0 + sl;
        if (s >= n_slots) continue;
        const int c = perm ? perm[s] : s;
        if (c < 0) continue;
        double v = mu[(size_t)c * P + p];
        if (a.combine) {
            // second-sum partials: the p ranges present in the block of q = p
            // (fixed trip counts, so that all partial loads are in flight together)
            const int qbp = p / 16, npr = cdiv_dev(min(P, qbp * 16 + 16), kAdjPs);
            double g2[MAXNPS], g1[MAXNQB], g1d[MAXNQB];
#pragma unroll
            for (int ps = 0; ps < MAXNPS; ++ps)
                g2[ps] = (ps < npr) ? G2[((size_t)ps * n_slots + s) * P + p] : 0.0;
#pragma unroll
            for (int qb = 0; qb < MAXNQB; ++qb) {
                const bool in = qb >= qbp && qb < NQB;
                g1[qb] = in ? G1p[((size_t)qb * n_slots + s) * P + p] : 0.0;
                g1d[qb] = (in && blend) ? G1p[(((size_t)NQB + qb) * n_slots + s) * P + p] : 0.0;
            }
            double g = 0.0;
#pragma unroll
            for (int ps = 0; ps < MAXNPS; ++ps) g += g2[ps];
#pragma unroll
            for (int qb = 0; qb < MAXNQB; ++qb) g += g1[qb] + g1d[qb];
            const double sc = kscale ? kscale[c] : 1.0;
            v += sc * g;
            red[sl * P + p] = 0.5 * ylin[(size_t)c * P + p] * g;
        }
        sl_lam[sl * P + p] = v;
    }
    __syncthreads();
    if (a.combine && threadIdx.x < kAdjSlots) {
        const int s = tile * 32 + s0 + threadIdx.x;
        if (s < n_slots) {
            const int c = perm ? perm[s] : s;
            if (c >= 0) {
                // summed in coefficient order, so that the result does not depend on
                // the order in which the waves ran
                double rsum = 0.0;
                for (int p = 0; p < P; ++p) rsum += red[threadIdx.x * P + p];
                if (a.dkscale) a.dkscale[G->cell0 + c] += rsum;
                if (a.dvfrag && blend) {
                    double d = 0.0;
#pragma unroll
                    for (int qb = 0; qb < MAXNQB; ++qb) {
                        const int npr = cdiv_dev(min(P, qb * 16 + 16), kAdjPs);
                        double dq[MAXNPS];
#pragma unroll
                        for (int ps = 0; ps < MAXNPS; ++ps)
                            dq[ps] = (qb < NQB && ps < npr) ? G->Dth[((size_t)ps * NQB + qb) * n_slots + s] : 0.0;
#pragma unroll
                        for (int ps = 0; ps < MAXNPS; ++ps) d += dq[ps];
                    }
                    const double sc = kscale ? kscale[c] : 1.0;
                    a.dvfrag[G->cell0 + c] += sc * d * G->dthdv[s];
                }
            }
        }
    }

    // ---- phase 1: one thread per (slot, bin)
    for (int t = threadIdx.x; t < kAdjSlots * N; t += blockDim.x) {
        const int sl = t / N, j = t - sl * N;
        const int s = tile * 32 + s0 + sl;
        if (s >= n_slots) continue;
        const int c = perm ? perm[s] : s;
        if (c < 0) continue;
        const size_t base = (size_t)c * P + j * K1;
        double* m = sl_lam + sl * P + j * K1;
        if (gamma && k > 0) {
            double l[kMaxOrder + 1];
            for (int i = 0; i < K1; ++i) l[i] = m[i];
            limiter_vjp(k, gamma[(size_t)c * N + j], ylim + base, l);
            for (int i = 0; i < K1; ++i) m[i] = l[i];
        }
        for (int i = 0; i < K1; ++i) {
            if (out) {
                out[base + i] = m[i];
                continue;
            }
            if (acc) acc[base + i] = a.acc_add ? acc[base + i] + a.a * m[i] : a.a * m[i];
            if (prev) prev[base + i] = a.prev_add ? prev[base + i] + a.b * m[i] : a.b * m[i];
        }
    }
    if (out) return;
    __syncthreads();

    // ---- phase 2: nu, one thread per (slot, bin)
    GD_GLOBAL double* nu = gptr(G->nu);
    const int vbase = (N - 1) + (conservative ? 0 : 1);
    for (int t = threadIdx.x; t < kAdjSlots * N; t += blockDim.x) {
        const int sl = t / N, j = t - sl * N;
        const int s = tile * 32 + s0 + sl;
        if (s >= n_slots) continue;
        const int c = perm ? perm[s] : s;
        GD_GLOBAL double* nrow = nu + (size_t)s * nus;
        if (c < 0) {
            for (int o = j; o < nus; o += N) nrow[o] = 0.0;
            continue;
        }
        const double* m = sl_lam + sl * P + j * K1;
        double rho[kMaxOrder + 1];
        for (int i = 0; i < K1; ++i) rho[i] = a.bdt * m[i];
        const double hj = h[j];
        // V_{j,i}
        for (int i = 1; i < K1; ++i) nrow[vbase + j * k + i - 1] = rho[i] * (2.0 * i + 1.0) / hj;
        // F_j (interior interface j >= 1): from bin j (as F_j) and bin j-1 (as F_{j+1})
        if (j >= 1) {
            const double hl = h[j - 1];
            const double* ml = m - K1;
            double v = 0.0;
            for (int i = 0; i < K1; ++i)
                v += ((i & 1) ? -1.0 : 1.0) * rho[i] * (2.0 * i + 1.0) / hj - a.bdt * ml[i] * (2.0 * i + 1.0) / hl;
            nrow[j - 1] = v;
        }
        if (j == N - 1 && !conservative) {
            double v = 0.0;
            for (int i = 0; i < K1; ++i) v -= rho[i] * (2.0 * i + 1.0) / hj;
            nrow[N - 1] = v;
        }
        if (j == 0)
            for (int o = n_out; o < nus; ++o) nrow[o] = 0.0;
    }
}

int launch_adj_boundary(const AdjStageArgs& a, hipStream_t s)
{
    if (a.n_tiles == 0) return GD_OK;
    const dim3 grid((unsigned)a.n_tiles * (32 / kAdjSlots));
    if (a.max_p <= 96)
        hipLaunchKernelGGL(k_adj_boundary<96>, grid, dim3(kAdjThreads), 0, s, a);
    else if (a.max_p <= 192)
        hipLaunchKernelGGL(k_adj_boundary<192>, grid, dim3(kAdjThreads), 0, s, a);
    else if (a.max_p <= kMaxP)
        hipLaunchKernelGGL(k_adj_boundary<kMaxP>, grid, dim3(kAdjThreads), 0, s, a);
    else
        return fail(GD_EUNSUPPORTED, "P too large for the reverse stage kernel");
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

} // namespace gd
