// Per-cell and per-bin kernels around the contraction: the assembly of the DG
// right-hand side (Sec. 3.1, Eq. evo), the SSP-RK3 stage combination (Eq. RK3), the
// scaling limiter (Sec. 3.2, Eqs. recon/gamma), the split of the scaled state into
// FP16 halves for the next contraction, and the projection of initial profiles
// (Eq. init).
#include <algorithm>

#include "bin_poly.h"
#include "gd_internal.h"

namespace gd {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// Limiter of one bin in registers: g^i <- gamma g^i (i >= 1) with
// gamma = min(1, avg / (avg - min)); a non-positive average flattens the bin and a
// negative one is reported.  K is the order, fixed at compile time: the minimum's
// root finding then runs without loops or branches on the order.
template <int K>
__device__ __forceinline__ int limit_bin(double* c, double& gamma)
{
    const double avg = c[0];
    int viol = 0;
    if (!(avg > 0.0) || avg == INFINITY) {
        // a negative (or non-finite) average cannot be repaired by scaling: reported
        gamma = 0.0;
        viol = !(avg == 0.0);
    } else {
        // |P_i| <= 1 on [-1,1]: avg - sum |c_i| >= 0 proves the minimum nonnegative
        double lb = avg;
#pragma unroll
        for (int i = 1; i <= K; ++i) lb -= fabs(c[i]);
        if (lb >= 0.0) {
            gamma = 1.0;
        } else {
            const double m = bin_min<K>(c);
            viol = !(m > -INFINITY);   // a non-finite higher coefficient
            gamma = (m < 0.0) ? fmin(1.0, avg / (avg - m)) : 1.0;
        }
    }
#pragma unroll
    for (int i = 1; i <= K; ++i) c[i] *= gamma;
    return viol;
}

// the order of a group is the same for the whole workgroup: no divergence
__device__ __forceinline__ int limit_bin(int k, double* c, double& gamma)
{
    switch (k) {
    case 0: return limit_bin<0>(c, gamma);
    case 1: return limit_bin<1>(c, gamma);
    case 2: return limit_bin<2>(c, gamma);
    case 3: return limit_bin<3>(c, gamma);
    default: return limit_bin<4>(c, gamma);
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_fill_f64(double* p, long long n, double v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// g_j^i = (2i+1)/2 sum_a w_a g0(x_a) P_i(s_a); wP holds (2i+1)/2 w_a P_i(s_a).
__global__ __launch_bounds__(256) void k_project(const double* samples, const double* wP, double* coef,
                                                 int C, int N, int k)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)C * N) return;
    const double* sm = samples + t * 16;
    double* out = coef + t * (k + 1);
    for (int i = 0; i <= k; ++i) {
        double acc = 0.0;
        for (int a2 = 0; a2 < 16; ++a2) acc += wP[i * 16 + a2] * sm[a2];
        out[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// Fused stage kernel (see StageArgs), one workgroup per tile of 32 slots of one group,
// with one thread per (slot, bin) task where the workgroup size allows.  The per-slot
// values (cell, exponent, kernel scale) are fetched once into LDS, and the
// coefficients of a bin move as 16-byte vectors when order + 1 is even.
// With the split on, phase 1 stages the scaled new state h_j g_q colscale_q of the
// tile in LDS (FP64: its range exceeds FP32 before the per-slot power of two is
// known; rows padded to P+1 against bank conflicts) and collects the largest binary
// exponent of every slot, so that the FP16 fragments and FP32 weights are written
// coalesced in phase 2.  Small workgroups with LDS sized to the plan's largest P keep
// most tiles of a launch resident at once.
// With ADAPT the stage also takes each cell's own step under the CFL bound of Eq. dt:
// before the RK combination of the first stage, the workgroup forms per slot the
// minimum of h_j g_j^0 / (F(e_{j+1}) - F(e_j)) over the bins that lose mass and hold
// a positive average (only those can be driven negative by a forward-Euler stage,
// and none can be helped by a step when the average is zero), then
// dt = min(dt_max, t_end - t, cfl * bound).  With a positive flux floor, a first
// pass takes the slot's largest edge flux and bins whose net outflow is at most
// floor times it are left out (with split-FP16 fluxes such outflows can be rounding
// noise).  A cell with dt = 0 (done, or stuck at a zero bound) keeps its state bit
// for bit: no combination, no limiter.
constexpr int kStageMidP = 192;
constexpr int kStageThreads = 256;

template <int PMAX, bool ADAPT>
__global__ __launch_bounds__(kStageThreads) void k_stage(StageArgs a)
{
    __shared__ double st[32 * (PMAX + 1)];
    __shared__ int smax[32];
    const GD_CONST GroupDev* groups = cptr(a.groups);
    int gi = 0;
    const int gtile = (int)blockIdx.x + a.tile0;
    while (gi + 1 < a.n_groups && gtile >= groups[gi + 1].tile_off) ++gi;
    const GD_CONST GroupDev* G = groups + gi;
    const int tile = gtile - G->tile_off, tid = threadIdx.x;
    const int N = G->N, k = G->k, K1 = k + 1, P = G->P, LD = P + 1, n_out = G->n_out;
    const int n_slots = G->n_slots, ystride = G->ystride;
    const bool conservative = G->conservative != 0;
    const GD_CONST double* h = cptr(G->h);
    const GD_GLOBAL double* cs = gptr(G->colscale);
    const GD_CONST double* rowscale = cptr(G->rowscale);
    const GD_GLOBAL int* perm = gptr(G->perm);
    const GD_GLOBAL float* Yf = gptr(G->Yf);
    const GD_GLOBAL double* Yd = gptr(G->Yd);
    GD_GLOBAL int* eslot = gptr(G->eslot);
    const GD_GLOBAL double* kscale = a.kscale ? gptr(a.kscale) + G->cell0 : nullptr;
    const GD_GLOBAL double* gn = a.gn ? gptr(a.gn) + G->val0 : nullptr;
    const GD_GLOBAL double* gs = gptr(a.gs) + G->val0;
    GD_GLOBAL double* out = a.out ? gptr(a.out) + G->val0 : nullptr;
    GD_GLOBAL double* raw = a.raw ? gptr(a.raw) + G->raw0 : nullptr;
    __shared__ int scell[32];
    __shared__ double sfac[32];
    if (tid < 32) {
        const int s = tile * 32 + tid;
        int c = (s < n_slots) ? (perm ? perm[s] : s) : -1;
        if constexpr (kChecks) {
            if (c >= G->n_cells || (tile < 0 || tile >= G->tiles32)) {
                check_fail(G->checks, kCheckSlot);
                c = -1;
            }
        }
        scell[tid] = c;
        double fac = (c >= 0 && kscale) ? kscale[c] : 1.0;
        if (c >= 0 && a.mode >= 0 && Yf) fac = ldexp(fac, 2 * eslot[s]);
        sfac[tid] = fac;
        if (a.split) smax[tid] = INT_MIN;
    }
    __syncthreads();

    // per-slot step of this sub-step (ADAPT), or the common dt
    __shared__ double sdt[32];
    if constexpr (ADAPT) {
        const int nthr = blockDim.x;
        if (a.mode == 1) {
            // nonnegative doubles order as their bit patterns
            __shared__ unsigned long long sbnd[32], sfmax[32];
            if (tid < 32) {
                sbnd[tid] = 0x7ff0000000000000ull;   // +infinity
                sfmax[tid] = 0ull;
            }
            __syncthreads();
            // flux at raw position q of slot sl (edge fluxes sit at j(k+1)-1)
            auto flux = [&](int sl, int q) -> double {
                const size_t at = (size_t)(tile * 32 + sl) * ystride + q;
                if (Yf) return (double)Yf[at] * rowscale[q] * sfac[sl];
                return Yd[at] * sfac[sl];
            };
            if (a.floor > 0.0) {
                for (int t = tid; t < 32 * N; t += nthr) {
                    const int sl = t / N, j = t - sl * N;
                    if (scell[sl] < 0) continue;
                    const double Fl = (j == 0) ? 0.0 : flux(sl, j * K1 - 1);
                    const double Fr = (j + 1 < N || !conservative) ? flux(sl, (j + 1) * K1 - 1) : 0.0;
                    const double m = fmax(fabs(Fl), fabs(Fr));
                    if (m > 0.0) atomicMax(&sfmax[sl], (unsigned long long)__double_as_longlong(m));
                }
                __syncthreads();
            }
            for (int t = tid; t < 32 * N; t += nthr) {
                const int sl = t / N, j = t - sl * N, c = scell[sl];
                if (c < 0) continue;
                const double Fl = (j == 0) ? 0.0 : flux(sl, j * K1 - 1);
                const double Fr = (j + 1 < N || !conservative) ? flux(sl, (j + 1) * K1 - 1) : 0.0;
                const double d = Fr - Fl, gj = gs[(size_t)c * P + j * K1];
                const double fl = a.floor * __longlong_as_double((long long)sfmax[sl]);
                if (d > 0.0 && d > fl && gj > 0.0) {
                    const double b = h[j] * gj / d;
                    if (b == b) atomicMin(&sbnd[sl], (unsigned long long)__double_as_longlong(b));
                }
            }
            __syncthreads();
            if (tid < 32) {
                const int c = scell[tid];
                double dt = 0.0;
                if (c >= 0) {
                    const double rem = a.t_end - a.tcell[G->cell0 + c];
                    if (rem > 0.0) {
                        dt = a.dt < rem ? a.dt : rem;
                        const double cb = a.cfl * __longlong_as_double((long long)sbnd[tid]);
                        if (cb < dt) dt = cb;
                        if (!(dt > 0.0)) dt = 0.0;
                    }
                    a.dtc[G->cell0 + c] = dt;
                }
                sdt[tid] = dt;
            }
        } else if (tid < 32) {
            const int c = scell[tid];
            sdt[tid] = (c >= 0) ? a.dtc[G->cell0 + c] : 0.0;
        }
        __syncthreads();
        if (a.mode == 3 && tid < 32) {
            const int c = scell[tid];
            const double dt = sdt[tid];
            if (c >= 0 && dt > 0.0) {
                const double tc = a.tcell[G->cell0 + c], rem = a.t_end - tc;
                a.tcell[G->cell0 + c] = (dt == rem) ? a.t_end : tc + dt;
            }
        }
    }

    // 16-byte moves need an even order + 1 and 16-byte aligned bin starts
    auto al16 = [](const void* p) { return p == nullptr || ((uintptr_t)p & 15) == 0; };
    const bool vec = (K1 & 1) == 0 && al16(gs) && al16(gn) && al16(out);

    // ---- phase 1: one task per (slot, bin)
    int viol = 0;
    const int nthr = blockDim.x;
    for (int t = tid; t < 32 * N; t += nthr) {
        const int sl = t / N, j = t - sl * N;
        const int s = tile * 32 + sl;
        const int c = scell[sl];
        double v[kMaxOrder + 1] = {};
        if (c >= 0) {
            const size_t base = (size_t)c * P + j * K1;
            // bin coefficients, as 16-byte vectors when K1 is even (base is then even)
            auto load = [&](const GD_GLOBAL double* src, double (&x)[kMaxOrder + 1]) {
                if (vec) {
                    const GD_GLOBAL double2* s2 = reinterpret_cast<const GD_GLOBAL double2*>(src + base);
                    for (int i2 = 0; i2 < K1 / 2; ++i2) {
                        const double2 d2 = s2[i2];
                        x[2 * i2] = d2.x;
                        x[2 * i2 + 1] = d2.y;
                    }
                } else {
                    for (int i = 0; i < K1; ++i) x[i] = src[base + i];
                }
            };
            if (a.mode < 0) {
                load(gs, v);
            } else {
                const double fac = sfac[sl];
                // raw rows are stored bin by bin: F_j at position j(k+1)-1, V_{j,i} at
                // j(k+1)+i-1, F_{j+1} (and F_N of the non-conservative flux) at (j+1)(k+1)-1
                auto pos = [&](int q) -> double {
                    if (Yf) return (double)Yf[(size_t)s * ystride + q] * rowscale[q] * fac;
                    return Yd[(size_t)s * ystride + q] * fac;
                };
                const double Fl = (j == 0) ? 0.0 : pos(j * K1 - 1);
                const double Fr = (j + 1 < N || !conservative) ? pos((j + 1) * K1 - 1) : 0.0;
                const int vbase = (N - 1) + (conservative ? 0 : 1);
                const double ihj = 1.0 / h[j];
                if (raw) {
                    GD_GLOBAL double* rw = raw + (size_t)c * n_out;
                    if (j >= 1) rw[j - 1] = Fl;
                    if (j == N - 1 && !conservative) rw[N - 1] = Fr;
                }
                double xs[kMaxOrder + 1] = {}, xn[kMaxOrder + 1] = {};
                if (a.mode >= 1) load(gs, xs);
                if (a.mode >= 2) load(gn, xn);
                const double dt = ADAPT ? sdt[sl] : a.dt;
                const bool hold = ADAPT && !(dt > 0.0);   // this cell takes no step
                for (int i = 0; i < K1; ++i) {
                    const double V = (i == 0) ? 0.0 : pos(j * K1 + i - 1);
                    if (raw && i > 0) raw[(size_t)c * n_out + vbase + j * k + i - 1] = V;
                    const double sgn = (i & 1) ? -1.0 : 1.0;
                    const double L = (2.0 * i + 1.0) * ihj * (V - Fr + sgn * Fl);
                    switch (a.mode) {
                    case 0: v[i] = L; break;
                    case 1: v[i] = hold ? xs[i] : xs[i] + dt * L; break;
                    case 2: v[i] = hold ? xn[i] : 0.75 * xn[i] + 0.25 * (xs[i] + dt * L); break;
                    default: v[i] = hold ? xn[i] : (1.0 / 3.0) * xn[i] + (2.0 / 3.0) * (xs[i] + dt * L); break;
                    }
                }
            }
            if constexpr (kChecks) {
                bool fin = true;
                for (int i = 0; i < K1; ++i) fin = fin && isfinite(v[i]);
                if (!fin) check_fail(G->checks, kCheckNonFinite);
            }
            if (a.limit && !(ADAPT && a.mode >= 1 && !(sdt[sl] > 0.0))) {
                double gam;
                viol += limit_bin(k, v, gam);
                if (a.gamma) a.gamma[G->gam0 + (size_t)c * N + j] = gam;
            }
            if (a.mode >= 0 || a.limit) {
                GD_GLOBAL double* o = (a.mode >= 0 || out) ? out : const_cast<GD_GLOBAL double*>(gs);
                if (vec) {
                    GD_GLOBAL double2* o2 = reinterpret_cast<GD_GLOBAL double2*>(o + base);
                    for (int i2 = 0; i2 < K1 / 2; ++i2) o2[i2] = make_double2(v[2 * i2], v[2 * i2 + 1]);
                } else {
                    for (int i = 0; i < K1; ++i) o[base + i] = v[i];
                }
            }
        }
        if (a.split) {
            int emax = INT_MIN;
            for (int i = 0; i < K1; ++i) {
                const int q = j * K1 + i;
                const double u = h[j] * v[i] * cs[q];
                st[sl * LD + q] = u;
                if (u != 0.0) {
                    int E;
                    frexp(u, &E);
                    emax = max(emax, E);
                }
            }
            if (emax != INT_MIN) atomicMax(&smax[sl], emax);
        }
    }
    if (viol) atomicAdd(a.viol, (unsigned long long)viol);
    if (!a.split) return;
    __syncthreads();
    // ---- phase 2: per-slot exponent e with max_q |h_j g_q c_q| 2^-e in [64, 128),
    // then the fragments and weights, coalesced
    if (tid < 32) {
        const int e = (smax[tid] == INT_MIN) ? 0 : smax[tid] - 7;
        smax[tid] = e;
        const int s = tile * 32 + tid;
        if (s < n_slots) eslot[s] = e;
    }
    __syncthreads();
    // each lane splits 8 consecutive coefficients of one slot: hi/lo halves into the
    // B-operand fragment, the FP32 value into the weights [tile][q][32 slots]
    const int KS = G->KS;
    GD_GLOBAL uint4* mfrag = gptr(G->mfrag);
    GD_GLOBAL float* mt = gptr(G->mt) + (size_t)tile * P * 32;
    for (int t = tid; t < KS * 64; t += nthr) {
        const int ks = t >> 6, lane = t & 63, sl = lane & 31, hh = lane >> 5;
        half8_t hi, lo;
        for (int jj = 0; jj < 8; ++jj) {
            const int q = ks * 16 + hh * 8 + jj;
            float m = 0.0f;
            if (q < P) {
                m = (float)ldexp(st[sl * LD + q], -smax[sl]);
                mt[(size_t)q * 32 + sl] = m;
            }
            const _Float16 mh = (_Float16)m;
            hi[jj] = mh;
            lo[jj] = (_Float16)(m - (float)mh);
        }
        const size_t base = ((size_t)(tile * KS + ks) * 2) * 64 + lane;
        mfrag[base] = __builtin_bit_cast(uint4, hi);
        mfrag[base + 64] = __builtin_bit_cast(uint4, lo);
    }
}

int launch_stage(const StageArgs& a, hipStream_t s)
{
    if (a.n_tiles == 0) return GD_OK;
    if (a.max_p > kMaxP) return fail(GD_EUNSUPPORTED, "P too large for the stage kernel");
    // LDS sized to the plan's largest P (more resident workgroups for small P)
    const dim3 grid(a.n_tiles), block(kStageThreads);
    if (a.adapt) {
        if (a.mode < 1 || !a.tcell || !a.dtc) return fail(GD_EINVAL, "adaptive stage needs an RK mode and time arrays");
        if (a.max_p <= 96) hipLaunchKernelGGL((k_stage<96, true>), grid, block, 0, s, a);
        else if (a.max_p <= kStageMidP) hipLaunchKernelGGL((k_stage<kStageMidP, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stage<kMaxP, true>), grid, block, 0, s, a);
    } else {
        if (a.max_p <= 96) hipLaunchKernelGGL((k_stage<96, false>), grid, block, 0, s, a);
        else if (a.max_p <= kStageMidP) hipLaunchKernelGGL((k_stage<kStageMidP, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_stage<kMaxP, false>), grid, block, 0, s, a);
    }
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

// number of entries below t_end (the cells an adaptive call has not brought there)
__global__ void k_count_below(const double* t, long long n, double t_end, unsigned long long* count)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool below = i < n && !(t[i] >= t_end);
    const unsigned long long m = __ballot(below);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

int launch_count_below(const double* t, long long n, double t_end, unsigned long long* count, hipStream_t s)
{
    if (n <= 0) return GD_OK;
    hipLaunchKernelGGL(k_count_below, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, n, t_end, count);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

// ---------------------------------------------------------------------------
int launch_fill_u64(unsigned long long* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(cdiv(n, 64)), dim3(64), 0, s, p, n);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_fill_f64(double* p, long long n, double v, hipStream_t s)
{
    if (n <= 0) return GD_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_project(const double* samples, const double* wP, double* coef, int C, int N, int k, hipStream_t s)
{
    const long long n = (long long)C * N;
    if (n == 0) return GD_OK;
    hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, samples, wP, coef, C, N, k);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

} // namespace gd
