// MI355X (gfx950) evaluation of the GRACE-DG collision operator.
//
// Per hydro cell c the raw flux vector is the quadratic form
//     Y_o(c) = sum_{p<=q} Tf[o][p][q] g_p(c) g_q(c)       (Tf: T folded over p<->q)
// (fluxes at the bin edges and volume moments of Sec. 3.3), from which the DG
// right-hand side L follows bin by bin (Sec. 3.1, Eq. evo).  The contraction is
// evaluated as
//     Z_p(c)[o] = sum_{q>=p} Tf[o][p][q] g_q(c)           (MFMA, K = q)
//     Y_o(c)   += g_p(c) Z_p(c)[o]                         (VALU, per lane)
// with T as the MFMA A operand (rows o), the cell states as the B operand
// (columns = cells) and the accumulators Z in registers.  The p loop walks p and
// P-1-p together so that every iteration carries the same number of K steps.
//
// Two precisions share the layout:
//  * FP64: v_mfma_f64_16x16x4, T and g in double;
//  * split FP16: the state is scaled per cell by a power of two, m = h_j g / 2^e,
//    T is divided by h_l h_m and scaled by powers of two per row and per
//    (row block, p); both operands are split into hi + lo FP16 halves and the
//    three products hi*hi + hi*lo + lo*hi are accumulated in FP32 by
//    v_mfma_f32_32x32x16_f16.  The bin-mass bookkeeping, the limiter and the
//    RK combination stay FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/gracedg.h"
#include "kernels.h"
#include "tensor_build.h"

using namespace gd;

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ============================================================================ errors
static thread_local std::string g_err;

static int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(GD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

extern "C" const char* gd_last_error(void) { return g_err.c_str(); }

// ============================================================================ kernels

// Minimum over xi in [-1,1] of sum_i c_i P_i(xi) for degree k <= 3: the end points
// and the real roots of the derivative g1 + 3 g2 xi + g3 (15 xi^2 - 3)/2 (Eq. gamma
// asks for the analytic minimum).
__device__ __forceinline__ double poly_val(int k, const double* c, double x)
{
    double v = c[0];
    if (k >= 1) v += c[1] * x;
    if (k >= 2) v += c[2] * (1.5 * x * x - 0.5);
    if (k >= 3) v += c[3] * (2.5 * x * x * x - 1.5 * x);
    return v;
}

__device__ double poly_min(int k, const double* c)
{
    double m = fmin(poly_val(k, c, -1.0), poly_val(k, c, 1.0));
    if (k < 2) return m;
    const double A = (k >= 3) ? 7.5 * c[3] : 0.0;
    const double B = 3.0 * c[2];
    const double C = c[1] - ((k >= 3) ? 1.5 * c[3] : 0.0);
    double r[2];
    int nr = 0;
    if (A != 0.0) {
        const double d = B * B - 4.0 * A * C;
        if (d >= 0.0) {
            const double sq = sqrt(d);
            const double qq = -0.5 * (B + copysign(sq, B));
            if (qq != 0.0) { r[nr++] = qq / A; r[nr++] = C / qq; }
            else r[nr++] = 0.0;
        }
    } else if (B != 0.0) {
        r[nr++] = -C / B;
    }
    for (int t = 0; t < nr; ++t)
        if (r[t] > -1.0 && r[t] < 1.0) m = fmin(m, poly_val(k, c, r[t]));
    return m;
}

// Scaling limiter (Eqs. recon, gamma) of one bin in registers; returns 1 for a
// negative cell average (the bin is flattened and counted).
__device__ __forceinline__ int limit_bin(int k, double* c)
{
    const double avg = c[0];
    double gamma;
    int viol = 0;
    if (avg <= 0.0) {
        gamma = 0.0;
        viol = avg < 0.0;
    } else {
        const double m = poly_min(k, c);
        gamma = (m < 0.0) ? fmin(1.0, avg / (avg - m)) : 1.0;
    }
    for (int i = 1; i <= k; ++i) c[i] *= gamma;
    return viol;
}

// ---------------------------------------------------------------------------
// Prologue, one thread per cell: optional limiter in place, then (mixed path)
// the per-cell power-of-two scale and the split hi/lo FP16 B-operand fragments.
//   mfrag[((tile*KS + ks)*2 + {0 hi,1 lo})*64 + lane] : 8 halves, lane = 32*hh + cell%32,
//        K index q = 16 ks + 8 hh + j
//   mt[(tile*P + p)*32 + cell%32]                        : m_p in FP32
struct PrologueArgs {
    double* g;                 // group state [C][P]
    int C, N, k, P, KS;
    int n_tiles;               // 32-cell tiles (mixed) ; unused for fp64
    int limit;                 // apply limiter in place
    int mixed;                 // write split fragments
    const double* h;           // [N]
    uint4* mfrag;
    float* mt;
    int* ecell;                // [C] exponent e
    unsigned long long* viol;  // violation counter
};

__global__ __launch_bounds__(256) void k_prologue(PrologueArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell_pad = a.mixed ? a.n_tiles * 32 : a.C;
    if (c >= ncell_pad) return;
    const int K1 = a.k + 1;
    double* gc = a.g + (size_t)c * a.P;
    const bool live = c < a.C;
    if (live && a.limit) {
        int v = 0;
        for (int j = 0; j < a.N; ++j) {
            double cc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i < K1; ++i) cc[i] = gc[j * K1 + i];
            v += limit_bin(a.k, cc);
            for (int i = 1; i < K1; ++i) gc[j * K1 + i] = cc[i];
        }
        if (v) atomicAdd(a.viol, (unsigned long long)v);
    }
    if (!a.mixed) return;
    // per-cell scale: max_p |h_j g_p| * 2^-e in [64, 128)
    double mx = 0.0;
    if (live)
        for (int p = 0; p < a.P; ++p) mx = fmax(mx, fabs(a.h[p / K1] * gc[p]));
    int e = 0;
    if (mx > 0.0) {
        int E;
        frexp(mx, &E);
        e = E - 7;
    }
    if (live) a.ecell[c] = e;
    const int tile = c >> 5, cl = c & 31;
    for (int ks = 0; ks < a.KS; ++ks)
        for (int hh = 0; hh < 2; ++hh) {
            half8_t hi, lo;
            for (int j = 0; j < 8; ++j) {
                const int q = ks * 16 + hh * 8 + j;
                float m = 0.0f;
                if (live && q < a.P) m = (float)ldexp(a.h[q / K1] * gc[q], -e);
                const _Float16 mh = (_Float16)m;
                hi[j] = mh;
                lo[j] = (_Float16)(m - (float)mh);
            }
            const size_t base = ((size_t)(tile * a.KS + ks) * 2) * 64 + hh * 32 + cl;
            a.mfrag[base] = *reinterpret_cast<uint4*>(&hi);
            a.mfrag[base + 64] = *reinterpret_cast<uint4*>(&lo);
        }
    for (int p = 0; p < a.P; ++p) {
        float m = 0.0f;
        if (live) m = (float)ldexp(a.h[p / K1] * gc[p], -e);
        a.mt[((size_t)tile * a.P + p) * 32 + cl] = m;
    }
}

// ---------------------------------------------------------------------------
// Split-FP16 contraction.  Workgroup = 4 waves; wave w owns NT tiles of 32 cells.
// Per iteration (row block ob, p pair) the workgroup stages the T fragments of
// both p values into LDS (double buffered) and every wave runs, per p,
//   Z = sum_{ks >= p/16} (Thi*mhi + Thi*mlo + Tlo*mhi)[ks]   (MFMA, FP32 acc)
//   Y += (m_p * scale[ob][p]) * Z                            (VALU)
// Output: Yraw[cell][ob*32 + row] in FP32, in units of rowscale * 2^(2e).
struct MixedArgs {
    MixedLevel lv;
    const int4* sched;
    const uint4* mfrag;
    const float* mt;
    float* Y;
    int C, P, KS, NOB, n_pairs, n_tiles, ystride;
};

template <int KSMAX, int NT>
__global__ __launch_bounds__(256) void k_contract_mixed(MixedArgs a)
{
    extern __shared__ uint4 lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile0 = (blockIdx.x * 4 + wave) * NT;
    constexpr int BUF = 2 * KSMAX * 128;   // uint4 per buffer

    half8_t bh[NT][KSMAX], bl[NT][KSMAX];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            uint4 vh = {0, 0, 0, 0}, vl = {0, 0, 0, 0};
            if (tile0 + t < a.n_tiles && ks < a.KS) {
                const size_t base = ((size_t)((tile0 + t) * a.KS + ks) * 2) * 64 + lane;
                vh = a.mfrag[base];
                vl = a.mfrag[base + 64];
            }
            bh[t][ks] = *reinterpret_cast<half8_t*>(&vh);
            bl[t][ks] = *reinterpret_cast<half8_t*>(&vl);
        }

    const int n_it = a.NOB * a.n_pairs;
    uint4 pre[KSMAX];
    auto fetch = [&](int it) {
        const int ob = it / a.n_pairs, pr = it - ob * a.n_pairs;
        const int f0 = ob * a.lv.frags_per_ob + a.lv.pair_off[pr];
        const int nf = a.lv.pair_off[pr + 1] - a.lv.pair_off[pr];
        const uint4* src = a.lv.frag + (size_t)f0 * 128;
#pragma unroll
        for (int i = 0; i < KSMAX; ++i) {
            const int idx = tid + 256 * i;
            if (idx < nf * 128) pre[i] = src[idx];
        }
        return nf;
    };
    auto store = [&](int buf, int nf) {
#pragma unroll
        for (int i = 0; i < KSMAX; ++i) {
            const int idx = tid + 256 * i;
            if (idx < nf * 128) lds[buf * BUF + idx] = pre[i];
        }
    };

    int nf = fetch(0);
    store(0, nf);
    __syncthreads();

    const bool tv0 = tile0 < a.n_tiles;
    int it = 0;
    for (int ob = 0; ob < a.NOB; ++ob) {
        floatx16 Y[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) Y[t][r] = 0.0f;

        for (int pr = 0; pr < a.n_pairs; ++pr, ++it) {
            const int buf = it & 1;
            int nf_next = 0;
            if (it + 1 < n_it) nf_next = fetch(it + 1);
            const int4 s = a.sched[pr];
            const uint4* B = lds + buf * BUF;
            int f = 0;
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                const int p = seg ? s.z : s.x;
                const int ks0 = seg ? s.w : s.y;
                if (p < 0) continue;
                float mp[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    mp[t] = (tile0 + t < a.n_tiles) ? a.mt[((size_t)(tile0 + t) * a.P + p) * 32 + (lane & 31)] : 0.0f;
                floatx16 Z[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 16; ++r) Z[t][r] = 0.0f;
#pragma unroll
                for (int ks = 0; ks < KSMAX; ++ks) {
                    if (ks >= ks0 && ks < a.KS) {
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
                const float sc = a.lv.scale[ob * a.P + p];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const float w = mp[t] * sc;
#pragma unroll
                    for (int r = 0; r < 16; ++r) Y[t][r] = fmaf(w, Z[t][r], Y[t][r]);
                }
            }
            if (it + 1 < n_it) store(buf ^ 1, nf_next);
            __syncthreads();
        }
        // D layout of 32x32 MFMA: lane holds column lane%32, rows 8*(r/4) + 4*(lane/32) + r%4
        (void)tv0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int cell = (tile0 + t) * 32 + (lane & 31);
            if (cell < a.C) {
                float* dst = a.Y + (size_t)cell * a.ystride + ob * 32 + 4 * (lane >> 5);
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    float4 v = make_float4(Y[t][4 * r4], Y[t][4 * r4 + 1], Y[t][4 * r4 + 2], Y[t][4 * r4 + 3]);
                    *reinterpret_cast<float4*>(dst + 8 * r4) = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 contraction with v_mfma_f64_16x16x4: tiles of 16 cells, row blocks of 16,
// K steps of 4.  Operand layouts: A lane l holds T[o = l%16][q = 4ks + l/16];
// B lane l holds g[cell = l%16][q = 4ks + l/16]; D lane l holds rows 4*(l/16)+i.
struct F64Args {
    F64Level lv;
    const int4* sched;
    const double* g;
    double* Y;
    int C, P, KS, NOB, n_pairs, n_tiles, ystride;
};

template <int KSMAX, int NT>
__global__ __launch_bounds__(256) void k_contract_fp64(F64Args a)
{
    extern __shared__ uint4 lds4[];
    double* lds = reinterpret_cast<double*>(lds4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile0 = (blockIdx.x * 4 + wave) * NT;
    constexpr int BUF = 2 * KSMAX * 64;        // doubles per buffer
    constexpr int PRE = (2 * KSMAX * 64 + 2 * 256 - 1) / (2 * 256);   // double2 per thread

    double b[NT][KSMAX];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int cell = (tile0 + t) * 16 + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            const int q = ks * 4 + (lane >> 4);
            b[t][ks] = (cell < a.C && q < a.P) ? a.g[(size_t)cell * a.P + q] : 0.0;
        }
    }

    const int n_it = a.NOB * a.n_pairs;
    double2 pre[PRE];
    auto fetch = [&](int it) {
        const int ob = it / a.n_pairs, pr = it - ob * a.n_pairs;
        const int f0 = ob * a.lv.frags_per_ob + a.lv.pair_off[pr];
        const int nf = a.lv.pair_off[pr + 1] - a.lv.pair_off[pr];
        const double2* src = reinterpret_cast<const double2*>(a.lv.frag + (size_t)f0 * 64);
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int idx = tid + 256 * i;
            if (idx < nf * 32) pre[i] = src[idx];
        }
        return nf;
    };
    auto store = [&](int buf, int nf) {
        double2* dst = reinterpret_cast<double2*>(lds + buf * BUF);
#pragma unroll
        for (int i = 0; i < PRE; ++i) {
            const int idx = tid + 256 * i;
            if (idx < nf * 32) dst[idx] = pre[i];
        }
    };

    int nf = fetch(0);
    store(0, nf);
    __syncthreads();

    int it = 0;
    for (int ob = 0; ob < a.NOB; ++ob) {
        doublex4 Y[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) Y[t] = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int pr = 0; pr < a.n_pairs; ++pr, ++it) {
            const int buf = it & 1;
            int nf_next = 0;
            if (it + 1 < n_it) nf_next = fetch(it + 1);
            const int4 s = a.sched[pr];
            const double* B = lds + buf * BUF;
            int f = 0;
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                const int p = seg ? s.z : s.x;
                const int ks0 = seg ? s.w : s.y;
                if (p < 0) continue;
                double gp[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int cell = (tile0 + t) * 16 + (lane & 15);
                    gp[t] = (cell < a.C) ? a.g[(size_t)cell * a.P + p] : 0.0;
                }
                doublex4 Z[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) Z[t] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < KSMAX; ++ks) {
                    if (ks >= ks0 && ks < a.KS) {
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
            if (it + 1 < n_it) store(buf ^ 1, nf_next);
            __syncthreads();
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int cell = (tile0 + t) * 16 + (lane & 15);
            if (cell < a.C) {
                double* dst = a.Y + (size_t)cell * a.ystride + ob * 16 + 4 * (lane >> 4);
#pragma unroll
                for (int r = 0; r < 4; ++r) dst[r] = Y[t][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Epilogue, one thread per (cell, bin): fluxes in FP64, L (Eq. evo) and the
// SSP-RK3 stage combination (Eq. RK3).
//   F_j = row j-1 of Y (F_0 = 0; F_N = 0 conservative, else row N-1)
//   L_{j,i} = (2i+1)/h_j (V_{j,i} - F_{j+1} + (-1)^i F_j)
//   mode 0: out = L;  mode 1: out = gs + dt L;  mode 2: out = 0.75 gn + 0.25 (gs + dt L)
//   mode 3: out = gn/3 + 2/3 (gs + dt L)
struct EpilogueArgs {
    const float* Yf;            // mixed raw (scaled)  or NULL
    const double* Yd;           // fp64 raw            or NULL
    const double* rowscale;     // mixed: [n_out_pad]
    const int* ecell;           // mixed: [C]
    const double* kscale;       // [C] or NULL
    const double* gn;           // RK base state
    const double* gs;           // stage input state
    double* out;
    double* raw;                // optional FP64 raw output [C][n_out]
    const double* h;
    double dt;
    int C, N, k, P, n_out, ystride, conservative, mode;
};

__global__ __launch_bounds__(256) void k_epilogue(EpilogueArgs a)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)a.C * a.N) return;
    const int c = (int)(t / a.N), j = (int)(t - (long long)c * a.N);
    const int K1 = a.k + 1;
    double fac = a.kscale ? a.kscale[c] : 1.0;
    if (a.Yf) fac = ldexp(fac, 2 * a.ecell[c]);
    auto row = [&](int o) -> double {
        if (a.Yf) return (double)a.Yf[(size_t)c * a.ystride + o] * a.rowscale[o] * fac;
        return a.Yd[(size_t)c * a.ystride + o] * fac;
    };
    const double Fl = (j == 0) ? 0.0 : row(j - 1);
    double Fr;
    if (j + 1 < a.N) Fr = row(j);
    else Fr = a.conservative ? 0.0 : row(a.N - 1);
    const int vbase = (a.N - 1) + (a.conservative ? 0 : 1);
    const double hj = a.h[j];
    const size_t base = (size_t)c * a.P + j * K1;
    if (a.raw) {
        double* rw = a.raw + (size_t)c * a.n_out;
        if (j >= 1) rw[j - 1] = Fl;
        if (j == a.N - 1 && !a.conservative) rw[a.N - 1] = Fr;
    }
    for (int i = 0; i <= a.k; ++i) {
        const double V = (i == 0) ? 0.0 : row(vbase + j * a.k + i - 1);
        if (a.raw && i > 0) a.raw[(size_t)c * a.n_out + vbase + j * a.k + i - 1] = V;
        const double sgn = (i & 1) ? -1.0 : 1.0;
        const double L = (2.0 * i + 1.0) / hj * (V - Fr + sgn * Fl);
        double o;
        switch (a.mode) {
        case 0: o = L; break;
        case 1: o = a.gs[base + i] + a.dt * L; break;
        case 2: o = 0.75 * a.gn[base + i] + 0.25 * (a.gs[base + i] + a.dt * L); break;
        default: o = a.gn[base + i] / 3.0 + 2.0 / 3.0 * (a.gs[base + i] + a.dt * L); break;
        }
        a.out[base + i] = o;
    }
}

// ============================================================================ host side
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

template <class T>
static int upload(std::vector<std::unique_ptr<DevBuf>>& owner, const std::vector<T>& v, const T** out, size_t* bytes)
{
    auto b = std::make_unique<DevBuf>();
    const size_t n = std::max<size_t>(1, v.size()) * sizeof(T);
    HIP_TRY(hipMalloc(&b->p, n));
    if (!v.empty()) HIP_TRY(hipMemcpy(b->p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<const T*>(b->p);
    *bytes += n;
    owner.push_back(std::move(b));
    return GD_OK;
}

struct gd_tensor {
    TensorSpec spec;
    HostTensor host;
    int N = 0, k = 0, P = 0, n_out = 0, R = 0;
    int n_pairs = 0;
    int KS = 0, NOB = 0;       // mixed: K steps of 16, row blocks of 32
    int KS4 = 0, NOB16 = 0;    // fp64: K steps of 4, row blocks of 16
    long long nnz = 0;
    size_t bytes = 0;
    bool packed = false;      // device layouts uploaded (done by the first plan)
    std::vector<std::unique_ptr<DevBuf>> bufs;
    const int4* sched = nullptr;
    const double* h = nullptr;
    std::vector<MixedLevel> mixed;
    std::vector<F64Level> f64;
};

static int cdiv(int a, int b) { return (a + b - 1) / b; }

// p schedule: pairs (p, P-1-p) so that every iteration holds about the same K work
static void make_pairs(int P, std::vector<std::pair<int, int>>& pairs)
{
    pairs.clear();
    for (int i = 0; i < P / 2; ++i) pairs.push_back({i, P - 1 - i});
    if (P & 1) pairs.push_back({P / 2, -1});
}

// structurally nonzero entries of the folded level-0 tensor (p <= q)
static void count_nnz(gd_tensor* t)
{
    const int P = t->P, NO = t->n_out;
    const double* T = t->host.T.data();
    long long n = 0;
    for (int o = 0; o < NO; ++o) {
        const double* To = T + size_t(o) * P * P;
        for (int p = 0; p < P; ++p)
            for (int q = p; q < P; ++q) {
                const double v = (q == p) ? To[size_t(p) * P + p] : To[size_t(p) * P + q] + To[size_t(q) * P + p];
                if (v != 0.0) ++n;
            }
    }
    t->nnz = n;
}

static int pack_tensor(gd_tensor* t)
{
    if (t->packed) return GD_OK;
    const int P = t->P, NO = t->n_out, R = t->R;
    std::vector<std::pair<int, int>> pairs;
    make_pairs(P, pairs);
    t->n_pairs = int(pairs.size());
    t->KS = cdiv(P, 16);
    t->NOB = cdiv(NO, 32);
    t->KS4 = cdiv(P, 4);
    t->NOB16 = cdiv(NO, 16);

    std::vector<int4> sched;
    for (auto& pr : pairs)
        sched.push_back(make_int4(pr.first, pr.first / 16, pr.second, pr.second >= 0 ? pr.second / 16 : 0));
    // the fp64 path uses its own K step; store a second schedule after the first
    for (auto& pr : pairs)
        sched.push_back(make_int4(pr.first, pr.first / 4, pr.second, pr.second >= 0 ? pr.second / 4 : 0));
    int rc = upload(t->bufs, sched, &t->sched, &t->bytes);
    if (rc) return rc;

    std::vector<double> h(t->N);
    for (int j = 0; j < t->N; ++j) h[j] = t->host.edges[j + 1] - t->host.edges[j];
    rc = upload(t->bufs, h, &t->h, &t->bytes);
    if (rc) return rc;

    const int K1 = t->k + 1;
    for (int r = 0; r < R; ++r) {
        const double* T = &t->host.T[size_t(r) * NO * P * P];
        // folded tensor Tf[o][p][q] for q >= p
        auto Tf = [&](int o, int p, int q) -> double {
            const double* To = T + size_t(o) * P * P;
            return (q == p) ? To[size_t(p) * P + p] : To[size_t(p) * P + q] + To[size_t(q) * P + p];
        };

        // ---------------- FP64 fragments: 16 rows x 4 K per fragment
        {
            std::vector<int> off(1, 0);
            for (auto& pr : pairs) {
                int n = t->KS4 - pr.first / 4;
                if (pr.second >= 0) n += t->KS4 - pr.second / 4;
                off.push_back(off.back() + n);
            }
            const int per_ob = off.back();
            std::vector<double> fr(size_t(t->NOB16) * per_ob * 64, 0.0);
            for (int ob = 0; ob < t->NOB16; ++ob)
                for (size_t ip = 0; ip < pairs.size(); ++ip) {
                    size_t f = size_t(ob) * per_ob + off[ip];
                    for (int seg = 0; seg < 2; ++seg) {
                        const int p = seg ? pairs[ip].second : pairs[ip].first;
                        if (p < 0) continue;
                        for (int ks = p / 4; ks < t->KS4; ++ks, ++f)
                            for (int l = 0; l < 64; ++l) {
                                const int o = ob * 16 + (l & 15), q = ks * 4 + (l >> 4);
                                if (o < NO && q < P && q >= p) fr[f * 64 + l] = Tf(o, p, q);
                            }
                    }
                }
            F64Level L{};
            rc = upload(t->bufs, fr, &L.frag, &t->bytes);
            if (rc) return rc;
            rc = upload(t->bufs, off, &L.pair_off, &t->bytes);
            if (rc) return rc;
            L.frags_per_ob = per_ob;
            t->f64.push_back(L);
        }

        // ---------------- split-FP16 fragments: 32 rows x 16 K per fragment
        {
            const int NOBp = t->NOB * 32;
            // U = Tf / (h_l h_m), row scale r_o, block scale s[ob][p]
            auto U = [&](int o, int p, int q) -> double { return Tf(o, p, q) / (h[p / K1] * h[q / K1]); };
            std::vector<double> rs(NOBp, 1.0);
            for (int o = 0; o < NO; ++o) {
                double mx = 0.0;
                for (int p = 0; p < P; ++p)
                    for (int q = p; q < P; ++q) mx = std::max(mx, std::fabs(U(o, p, q)));
                if (mx > 0.0) {
                    int E;
                    std::frexp(mx, &E);
                    rs[o] = std::ldexp(1.0, E);
                }
            }
            std::vector<float> sc(size_t(t->NOB) * P, 1.0f);
            for (int ob = 0; ob < t->NOB; ++ob)
                for (int p = 0; p < P; ++p) {
                    double mx = 0.0;
                    for (int o = ob * 32; o < std::min(NO, ob * 32 + 32); ++o)
                        for (int q = p; q < P; ++q) mx = std::max(mx, std::fabs(U(o, p, q)) / rs[o]);
                    if (mx > 0.0) {
                        int E;
                        std::frexp(mx, &E);
                        // block maximum lands in [2^14, 2^15)
                        const int ex = std::max(-126, E - 15);
                        sc[size_t(ob) * P + p] = std::ldexp(1.0f, ex);
                    }
                }
            std::vector<int> off(1, 0);
            for (auto& pr : pairs) {
                int n = t->KS - pr.first / 16;
                if (pr.second >= 0) n += t->KS - pr.second / 16;
                off.push_back(off.back() + n);
            }
            const int per_ob = off.back();
            std::vector<uint16_t> fr(size_t(t->NOB) * per_ob * 1024, 0);
            for (int ob = 0; ob < t->NOB; ++ob)
                for (size_t ip = 0; ip < pairs.size(); ++ip) {
                    size_t f = size_t(ob) * per_ob + off[ip];
                    for (int seg = 0; seg < 2; ++seg) {
                        const int p = seg ? pairs[ip].second : pairs[ip].first;
                        if (p < 0) continue;
                        const double s = sc[size_t(ob) * P + p];
                        for (int ks = p / 16; ks < t->KS; ++ks, ++f)
                            for (int l = 0; l < 64; ++l)
                                for (int j = 0; j < 8; ++j) {
                                    const int o = ob * 32 + (l & 31), q = ks * 16 + 8 * (l >> 5) + j;
                                    double v = 0.0;
                                    if (o < NO && q < P && q >= p) v = U(o, p, q) / (rs[o] * s);
                                    const _Float16 hi = (_Float16)v;
                                    const _Float16 lo = (_Float16)(v - (double)hi);
                                    uint16_t bh, bl;
                                    std::memcpy(&bh, &hi, 2);
                                    std::memcpy(&bl, &lo, 2);
                                    fr[f * 1024 + l * 8 + j] = bh;
                                    fr[f * 1024 + 512 + l * 8 + j] = bl;
                                }
                    }
                }
            MixedLevel L{};
            const uint16_t* dfr = nullptr;
            rc = upload(t->bufs, fr, &dfr, &t->bytes);
            if (rc) return rc;
            L.frag = reinterpret_cast<const uint4*>(dfr);
            rc = upload(t->bufs, off, &L.pair_off, &t->bytes);
            if (rc) return rc;
            L.frags_per_ob = per_ob;
            rc = upload(t->bufs, sc, &L.scale, &t->bytes);
            if (rc) return rc;
            rc = upload(t->bufs, rs, &L.rowscale, &t->bytes);
            if (rc) return rc;
            t->mixed.push_back(L);
        }
    }
    t->packed = true;
    return GD_OK;
}

extern "C" int gd_init_tensor(const gd_kernel* kernel, const gd_frag_law* frag, int bins, int order,
                              const gd_grid* grid, gd_tensor** out)
{
    if (!kernel || !frag || !grid || !out) return fail(GD_EINVAL, "null argument");
    if (bins < 2 || bins > 256 || order < 0 || order > 3) return fail(GD_EINVAL, "bins must be 2..256, order 0..3");
    if (kernel->kind < 0 || kernel->kind > 3) return fail(GD_EINVAL, "unknown kernel");
    if (frag->kind < 0 || frag->kind > 3) return fail(GD_EINVAL, "unknown fragmentation law");
    if (!(grid->x_min > 0.0) || !(grid->x_max > grid->x_min)) return fail(GD_EINVAL, "need 0 < x_min < x_max");
    if (grid->quad_points < 0 || grid->quad_points > 32) return fail(GD_EINVAL, "quad_points must be 0..32");
    if (frag->kind != GD_FRAG_NONE && (frag->n_levels < 1 || !frag->levels))
        return fail(GD_EINVAL, "fragmentation needs at least one threshold level");
    const int P = bins * (order + 1);
    if (P > 192) return fail(GD_EINVAL, "P = bins*(order+1) must be <= 192");
    auto t = std::unique_ptr<gd_tensor>(new (std::nothrow) gd_tensor());
    if (!t) return fail(GD_ENOMEM, "host allocation");
    TensorSpec& sp = t->spec;
    sp.kernel = kernel->kind;
    sp.v0 = kernel->v0;
    sp.frag = frag->kind;
    sp.alpha = frag->alpha;
    if (frag->kind != GD_FRAG_NONE) sp.levels.assign(frag->levels, frag->levels + frag->n_levels);
    for (size_t i = 1; i < sp.levels.size(); ++i)
        if (!(sp.levels[i] > sp.levels[i - 1])) return fail(GD_EINVAL, "levels must be ascending");
    sp.bins = bins;
    sp.order = order;
    sp.quad_points = grid->quad_points;
    sp.x_min = grid->x_min;
    sp.x_max = grid->x_max;
    sp.conservative = grid->conservative ? 1 : 0;
    try {
        build_tensor(sp, t->host);
    } catch (const std::exception& e) {
        return fail(GD_EINVAL, e.what());
    }
    t->N = bins;
    t->k = order;
    t->P = P;
    t->n_out = t->host.n_out;
    t->R = t->host.n_levels;
    count_nnz(t.get());
    *out = t.release();
    return GD_OK;
}

extern "C" int gd_tensor_info(const gd_tensor* t, gd_tensor_info_t* info)
{
    if (!t || !info) return fail(GD_EINVAL, "null argument");
    info->bins = t->N;
    info->order = t->k;
    info->P = t->P;
    info->n_out = t->n_out;
    info->n_levels = t->R;
    info->nnz_folded = t->nnz;
    info->flops_per_eval = 2.0 * double(t->nnz);
    info->device_bytes = t->bytes;
    return GD_OK;
}

extern "C" int gd_tensor_export(const gd_tensor* t, int level, double* host_out)
{
    if (!t || !host_out || level < 0 || level >= t->R) return fail(GD_EINVAL, "bad tensor export");
    const size_t n = size_t(t->n_out) * t->P * t->P;
    std::memcpy(host_out, &t->host.T[size_t(level) * n], n * sizeof(double));
    return GD_OK;
}

extern "C" int gd_tensor_edges(const gd_tensor* t, double* host_out)
{
    if (!t || !host_out) return fail(GD_EINVAL, "null argument");
    std::memcpy(host_out, t->host.edges.data(), sizeof(double) * (t->N + 1));
    return GD_OK;
}

extern "C" void gd_free_tensor(gd_tensor* t) { delete t; }

// ---------------------------------------------------------------- plans
struct Group {
    const gd_tensor* t;
    int C;
    long long cell0, val0;
    int tiles32, tiles16;
    uint4* mfrag = nullptr;
    float* mt = nullptr;
    int* ecell = nullptr;
    float* Yf = nullptr;
    double* Yd = nullptr;
    int ystride = 0;
};

struct gd_plan {
    std::vector<Group> groups;
    int prec = GD_PREC_FP64;
    hipStream_t stream = nullptr;
    long long n_cells = 0, n_values = 0;
    double* y1 = nullptr;
    double* y2 = nullptr;
    double* L = nullptr;
    unsigned long long* viol = nullptr;
    std::vector<void*> allocs;
    ~gd_plan()
    {
        for (void* p : allocs) (void)hipFree(p);
    }
};

template <class T>
static int dalloc(gd_plan* pl, T** p, size_t n)
{
    void* q = nullptr;
    HIP_TRY(hipMalloc(&q, std::max<size_t>(1, n) * sizeof(T)));
    pl->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return GD_OK;
}

extern "C" int gd_plan_create(const gd_tensor* const* tensors, const int* cells_per_group, int n_groups,
                              int precision, void* stream, gd_plan** out)
{
    if (!tensors || !cells_per_group || n_groups < 1 || !out) return fail(GD_EINVAL, "null argument");
    if (precision != GD_PREC_FP64 && precision != GD_PREC_MIXED_F16X3) return fail(GD_EINVAL, "unknown precision");
    auto pl = std::unique_ptr<gd_plan>(new (std::nothrow) gd_plan());
    if (!pl) return fail(GD_ENOMEM, "host allocation");
    pl->prec = precision;
    pl->stream = (hipStream_t)stream;
    for (int g = 0; g < n_groups; ++g) {
        if (!tensors[g] || cells_per_group[g] < 0) return fail(GD_EINVAL, "bad group");
        int prc = pack_tensor(const_cast<gd_tensor*>(tensors[g]));
        if (prc) return prc;
        Group G{};
        G.t = tensors[g];
        G.C = cells_per_group[g];
        G.cell0 = pl->n_cells;
        G.val0 = pl->n_values;
        G.tiles32 = cdiv(G.C, 32);
        G.tiles16 = cdiv(G.C, 16);
        pl->n_cells += G.C;
        pl->n_values += (long long)G.C * G.t->P;
        pl->groups.push_back(G);
    }
    int rc;
    if ((rc = dalloc(pl.get(), &pl->y1, pl->n_values))) return rc;
    if ((rc = dalloc(pl.get(), &pl->y2, pl->n_values))) return rc;
    if ((rc = dalloc(pl.get(), &pl->L, pl->n_values))) return rc;
    if ((rc = dalloc(pl.get(), &pl->viol, 1))) return rc;
    HIP_TRY(hipMemset(pl->viol, 0, sizeof(unsigned long long)));
    for (Group& G : pl->groups) {
        const gd_tensor* t = G.t;
        if (precision == GD_PREC_MIXED_F16X3) {
            G.ystride = t->NOB * 32;
            if ((rc = dalloc(pl.get(), &G.mfrag, size_t(G.tiles32) * t->KS * 128))) return rc;
            if ((rc = dalloc(pl.get(), &G.mt, size_t(G.tiles32) * 32 * t->P))) return rc;
            if ((rc = dalloc(pl.get(), &G.ecell, size_t(G.C)))) return rc;
            if ((rc = dalloc(pl.get(), &G.Yf, size_t(G.C) * G.ystride))) return rc;
        } else {
            G.ystride = t->NOB16 * 16;
            if ((rc = dalloc(pl.get(), &G.Yd, size_t(G.C) * G.ystride))) return rc;
        }
    }
    *out = pl.release();
    return GD_OK;
}

extern "C" int gd_plan_sizes(const gd_plan* pl, long long* n_cells, long long* n_values)
{
    if (!pl) return fail(GD_EINVAL, "null plan");
    if (n_cells) *n_cells = pl->n_cells;
    if (n_values) *n_values = pl->n_values;
    return GD_OK;
}

extern "C" void gd_plan_destroy(gd_plan* pl) { delete pl; }

// launch helpers --------------------------------------------------------------
template <int KSMAX, int NT>
static int launch_mixed_t(const MixedArgs& a, hipStream_t s)
{
    const int waves = cdiv(a.n_tiles, NT);
    const int blocks = cdiv(waves, 4);
    const size_t lds = size_t(2) * 2 * KSMAX * 128 * sizeof(uint4);
    static bool attr = false;
    if (!attr && lds > 65536) {
        HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_contract_mixed<KSMAX, NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        attr = true;
    }
    hipLaunchKernelGGL((k_contract_mixed<KSMAX, NT>), dim3(blocks), dim3(256), lds, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

static int launch_mixed(const MixedArgs& a, hipStream_t s)
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
    const int waves = cdiv(a.n_tiles, NT);
    const int blocks = cdiv(waves, 4);
    const size_t lds = size_t(2) * 2 * KSMAX * 64 * sizeof(double);
    static bool attr = false;
    if (!attr && lds > 65536) {
        HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_contract_fp64<KSMAX, NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        attr = true;
    }
    hipLaunchKernelGGL((k_contract_fp64<KSMAX, NT>), dim3(blocks), dim3(256), lds, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

static int launch_f64(const F64Args& a, hipStream_t s)
{
    if (a.KS <= 8) return launch_f64_t<8, 2>(a, s);
    if (a.KS <= 16) return launch_f64_t<16, 2>(a, s);
    if (a.KS <= 24) return launch_f64_t<24, 2>(a, s);
    if (a.KS <= 32) return launch_f64_t<32, 1>(a, s);
    if (a.KS <= 48) return launch_f64_t<48, 1>(a, s);
    return fail(GD_EUNSUPPORTED, "P too large for the FP64 contraction");
}

// one right-hand-side evaluation of group G on stage state gs
static int eval_group(gd_plan* pl, Group& G, double* gs, int limit, const double* kscale,
                      int mode, const double* gn, double* out, double dt, double* raw)
{
    const gd_tensor* t = G.t;
    if (G.C == 0) return GD_OK;
    hipStream_t s = pl->stream;
    const bool mixed = pl->prec == GD_PREC_MIXED_F16X3;
    PrologueArgs pa{};
    pa.g = gs;
    pa.C = G.C;
    pa.N = t->N;
    pa.k = t->k;
    pa.P = t->P;
    pa.KS = t->KS;
    pa.n_tiles = G.tiles32;
    pa.limit = limit;
    pa.mixed = mixed ? 1 : 0;
    pa.h = t->h;
    pa.mfrag = G.mfrag;
    pa.mt = G.mt;
    pa.ecell = G.ecell;
    pa.viol = pl->viol;
    if (limit || mixed) {
        const int n = mixed ? G.tiles32 * 32 : G.C;
        hipLaunchKernelGGL(k_prologue, dim3(cdiv(n, 256)), dim3(256), 0, s, pa);
        HIP_TRY(hipGetLastError());
    }
    int rc;
    if (mixed) {
        MixedArgs ma{};
        ma.lv = t->mixed[0];
        ma.sched = t->sched;
        ma.mfrag = G.mfrag;
        ma.mt = G.mt;
        ma.Y = G.Yf;
        ma.C = G.C;
        ma.P = t->P;
        ma.KS = t->KS;
        ma.NOB = t->NOB;
        ma.n_pairs = t->n_pairs;
        ma.n_tiles = G.tiles32;
        ma.ystride = G.ystride;
        if ((rc = launch_mixed(ma, s))) return rc;
    } else {
        F64Args fa{};
        fa.lv = t->f64[0];
        fa.sched = t->sched + t->n_pairs;
        fa.g = gs;
        fa.Y = G.Yd;
        fa.C = G.C;
        fa.P = t->P;
        fa.KS = t->KS4;
        fa.NOB = t->NOB16;
        fa.n_pairs = t->n_pairs;
        fa.n_tiles = G.tiles16;
        fa.ystride = G.ystride;
        if ((rc = launch_f64(fa, s))) return rc;
    }
    EpilogueArgs ea{};
    ea.Yf = mixed ? G.Yf : nullptr;
    ea.Yd = mixed ? nullptr : G.Yd;
    ea.rowscale = mixed ? t->mixed[0].rowscale : nullptr;
    ea.ecell = G.ecell;
    ea.kscale = kscale ? kscale + G.cell0 : nullptr;
    ea.gn = gn;
    ea.gs = gs;
    ea.out = out;
    ea.raw = raw;
    ea.h = t->h;
    ea.dt = dt;
    ea.C = G.C;
    ea.N = t->N;
    ea.k = t->k;
    ea.P = t->P;
    ea.n_out = t->n_out;
    ea.ystride = G.ystride;
    ea.conservative = t->spec.conservative;
    ea.mode = mode;
    const long long nthr = (long long)G.C * t->N;
    hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, ea);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

static int check_levels(const gd_plan* pl, const double* vfrag)
{
    for (const Group& G : pl->groups)
        if (G.t->R > 1 || vfrag) return fail(GD_EUNSUPPORTED, "per-cell thresholds are not built yet");
    return GD_OK;
}

extern "C" int gd_collision_rhs(gd_plan* pl, const double* g, const double* kscale, const double* vfrag,
                                double* rhs, double* raw)
{
    if (!pl || !g || !rhs) return fail(GD_EINVAL, "null argument");
    int rc = check_levels(pl, vfrag);
    if (rc) return rc;
    long long rawoff = 0;
    for (Group& G : pl->groups) {
        // the prologue never writes g when it does not limit
        double* gs = const_cast<double*>(g) + G.val0;
        rc = eval_group(pl, G, gs, 0, kscale, 0, nullptr, rhs + G.val0, 0.0, raw ? raw + rawoff : nullptr);
        if (rc) return rc;
        rawoff += (long long)G.C * G.t->n_out;
    }
    return GD_OK;
}

__global__ void k_limit_only(double* g, int C, int N, int k, int P, unsigned long long* viol)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double* gc = g + (size_t)c * P;
    int v = 0;
    for (int j = 0; j < N; ++j) {
        double cc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i <= k; ++i) cc[i] = gc[j * (k + 1) + i];
        v += limit_bin(k, cc);
        for (int i = 1; i <= k; ++i) gc[j * (k + 1) + i] = cc[i];
    }
    if (v) atomicAdd(viol, (unsigned long long)v);
}

extern "C" int gd_rk_step(gd_plan* pl, double* g, const double* kscale, const double* vfrag, double dt,
                          int n_steps, long long* violations)
{
    if (!pl || !g || n_steps < 0) return fail(GD_EINVAL, "bad argument");
    int rc = check_levels(pl, vfrag);
    if (rc) return rc;
    HIP_TRY(hipMemsetAsync(pl->viol, 0, sizeof(unsigned long long), pl->stream));
    for (int n = 0; n < n_steps; ++n) {
        for (Group& G : pl->groups) {
            double* gn = g + G.val0;
            double* y1 = pl->y1 + G.val0;
            double* y2 = pl->y2 + G.val0;
            if ((rc = eval_group(pl, G, gn, 1, kscale, 1, gn, y1, dt, nullptr))) return rc;
            if ((rc = eval_group(pl, G, y1, 1, kscale, 2, gn, y2, dt, nullptr))) return rc;
            if ((rc = eval_group(pl, G, y2, 1, kscale, 3, gn, gn, dt, nullptr))) return rc;
        }
    }
    for (Group& G : pl->groups) {
        if (G.C == 0) continue;
        hipLaunchKernelGGL(k_limit_only, dim3(cdiv(G.C, 256)), dim3(256), 0, pl->stream, g + G.val0, G.C,
                           G.t->N, G.t->k, G.t->P, pl->viol);
        HIP_TRY(hipGetLastError());
    }
    if (violations) {
        unsigned long long v = 0;
        HIP_TRY(hipMemcpyAsync(&v, pl->viol, sizeof(v), hipMemcpyDeviceToHost, pl->stream));
        HIP_TRY(hipStreamSynchronize(pl->stream));
        *violations = (long long)v;
    }
    return GD_OK;
}

// ---------------------------------------------------------------- projection (Eq. init)
// g_j^i = (2i+1)/2 sum_a w_a g0(c_j + h_j s_a/2) P_i(s_a) with a 16-point rule per
// bin; the caller samples g0 at the points given by gd_projection_points.
static constexpr int kProjPts = 16;

__global__ __launch_bounds__(256) void k_project(const double* samples, const double* wP, double* coef,
                                                 int C, int N, int k)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)C * N) return;
    const double* sm = samples + t * kProjPts;
    double* out = coef + t * (k + 1);
    for (int i = 0; i <= k; ++i) {
        double acc = 0.0;
        for (int a = 0; a < kProjPts; ++a) acc += wP[i * kProjPts + a] * sm[a];
        out[i] = acc;
    }
}

extern "C" int gd_projection_points(const gd_tensor* t, double* host_x)
{
    if (!t || !host_x) return fail(GD_EINVAL, "null argument");
    std::vector<double> s, w;
    gauss_legendre(kProjPts, s, w);
    for (int j = 0; j < t->N; ++j) {
        const double a = t->host.edges[j], b = t->host.edges[j + 1];
        for (int q = 0; q < kProjPts; ++q) host_x[j * kProjPts + q] = 0.5 * (a + b) + 0.5 * (b - a) * s[q];
    }
    return GD_OK;
}

extern "C" int gd_project(const gd_tensor* t, int n_cells, const double* samples, double* coef, void* stream)
{
    if (!t || !samples || !coef || n_cells < 0) return fail(GD_EINVAL, "bad argument");
    if (n_cells == 0) return GD_OK;
    std::vector<double> s, w;
    gauss_legendre(kProjPts, s, w);
    const int K1 = t->k + 1;
    std::vector<double> wP(size_t(K1) * kProjPts);
    for (int a = 0; a < kProjPts; ++a) {
        double P0 = 1.0, P1 = s[a];
        for (int i = 0; i < K1; ++i) {
            double Pi;
            if (i == 0) Pi = 1.0;
            else if (i == 1) Pi = s[a];
            else {
                Pi = ((2 * i - 1) * s[a] * P1 - (i - 1) * P0) / i;
                P0 = P1;
                P1 = Pi;
            }
            wP[size_t(i) * kProjPts + a] = 0.5 * (2 * i + 1) * w[a] * Pi;
        }
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, wP.size() * sizeof(double)));
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d, wP.data(), wP.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const long long n = (long long)n_cells * t->N;
        hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, samples, d, coef,
                           n_cells, t->N, t->k);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GD_EHIP, std::string("gd_project: ") + hipGetErrorString(e));
    return GD_OK;
}
