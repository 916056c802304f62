// Per-cell and per-bin kernels around the contraction: the assembly of the DG
// right-hand side (Sec. 3.1, Eq. evo), the SSP-RK3 stage combination (Eq. RK3), the
// scaling limiter (Sec. 3.2, Eqs. recon/gamma), the split of the scaled state into
// FP16 halves for the next contraction, and the projection of initial profiles
// (Eq. init).
#include "gd_internal.h"

namespace gd {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// Value of sum_i c_i P_i(x), degree k <= 3.
__device__ __forceinline__ double poly_val(int k, const double* c, double x)
{
    double v = c[0];
    if (k >= 1) v += c[1] * x;
    if (k >= 2) v += c[2] * (1.5 * x * x - 0.5);
    if (k >= 3) v += c[3] * (2.5 * x * x * x - 1.5 * x);
    return v;
}

// Minimum over [-1,1]: end points and the real roots of the derivative
// c1 + 3 c2 x + c3 (15 x^2 - 3)/2 inside (-1,1) (the analytic minimum of Eq. gamma).
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

// Limiter of one bin in registers: g^i <- gamma g^i (i >= 1) with
// gamma = min(1, avg / (avg - min)); a non-positive average flattens the bin and a
// negative one is reported.
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

__global__ void k_fill_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
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
// Fused stage kernel (see StageArgs), 256 threads per tile of 32 slots.  The new
// state of the tile is staged in LDS (rows padded to P+1 doubles against bank
// conflicts) so that the split fragments and weights are written coalesced.
constexpr int kStageMaxP = 192;

__global__ __launch_bounds__(256) void k_stage(StageArgs a)
{
    __shared__ double st[32 * (kStageMaxP + 1)];
    __shared__ int sexp[32];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int K1 = a.k + 1, P = a.P, LD = P + 1;

    // ---- phase 1: one task per (slot, bin)
    int viol = 0;
    for (int t = tid; t < 32 * a.N; t += 256) {
        const int sl = t / a.N, j = t - sl * a.N;
        const int s = tile * 32 + sl;
        const int c = (s < a.n_slots) ? (a.perm ? a.perm[s] : s) : -1;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (c >= 0) {
            const size_t base = (size_t)c * P + j * K1;
            if (a.mode < 0) {
                for (int i = 0; i < K1; ++i) v[i] = a.gs[base + i];
            } else {
                double fac = a.kscale ? a.kscale[c] : 1.0;
                if (a.Yf) fac = ldexp(fac, 2 * a.eslot[s]);
                auto row = [&](int o) -> double {
                    if (a.Yf) return (double)a.Yf[(size_t)s * a.ystride + o] * a.rowscale[o] * fac;
                    return a.Yd[(size_t)s * a.ystride + o] * fac;
                };
                const double Fl = (j == 0) ? 0.0 : row(j - 1);
                const double Fr = (j + 1 < a.N) ? row(j) : (a.conservative ? 0.0 : row(a.N - 1));
                const int vbase = (a.N - 1) + (a.conservative ? 0 : 1);
                const double hj = a.h[j];
                if (a.raw) {
                    double* rw = a.raw + (size_t)c * a.n_out;
                    if (j >= 1) rw[j - 1] = Fl;
                    if (j == a.N - 1 && !a.conservative) rw[a.N - 1] = Fr;
                }
                for (int i = 0; i < K1; ++i) {
                    const double V = (i == 0) ? 0.0 : row(vbase + j * a.k + i - 1);
                    if (a.raw && i > 0) a.raw[(size_t)c * a.n_out + vbase + j * a.k + i - 1] = V;
                    const double sgn = (i & 1) ? -1.0 : 1.0;
                    const double L = (2.0 * i + 1.0) / hj * (V - Fr + sgn * Fl);
                    switch (a.mode) {
                    case 0: v[i] = L; break;
                    case 1: v[i] = a.gs[base + i] + a.dt * L; break;
                    case 2: v[i] = 0.75 * a.gn[base + i] + 0.25 * (a.gs[base + i] + a.dt * L); break;
                    default: v[i] = a.gn[base + i] / 3.0 + 2.0 / 3.0 * (a.gs[base + i] + a.dt * L); break;
                    }
                }
            }
            if (a.limit) viol += limit_bin(a.k, v);
            if (a.mode >= 0 || a.limit) {
                double* o = (a.mode >= 0) ? a.out : const_cast<double*>(a.gs);
                for (int i = 0; i < K1; ++i) o[base + i] = v[i];
            }
        }
        if (a.split)
            for (int i = 0; i < K1; ++i) st[sl * LD + j * K1 + i] = v[i];
    }
    if (viol) atomicAdd(a.viol, (unsigned long long)viol);
    if (!a.split) return;
    __syncthreads();
    // ---- phase 2: per-slot exponent, then coalesced fragments and weights
    if (tid < 32) {
        // per-slot scale: max_q |h_j g_q c_q| 2^-e in [64, 128)
        double mx = 0.0;
        for (int q = 0; q < P; ++q) mx = fmax(mx, fabs(a.h[q / K1] * st[tid * LD + q] * a.colscale[q]));
        int e = 0;
        if (mx > 0.0) {
            int E;
            frexp(mx, &E);
            e = E - 7;
        }
        sexp[tid] = e;
        const int s = tile * 32 + tid;
        if (s < a.n_slots) a.eslot[s] = e;
    }
    __syncthreads();
    for (int t = tid; t < a.KS * 64; t += 256) {
        const int ks = t >> 6, lane = t & 63, sl = lane & 31, hh = lane >> 5;
        half8_t hi, lo;
        for (int jj = 0; jj < 8; ++jj) {
            const int q = ks * 16 + hh * 8 + jj;
            float m = 0.0f;
            if (q < P) m = (float)ldexp(a.h[q / K1] * st[sl * LD + q] * a.colscale[q], -sexp[sl]);
            const _Float16 mh = (_Float16)m;
            hi[jj] = mh;
            lo[jj] = (_Float16)(m - (float)mh);
        }
        const size_t base = ((size_t)(tile * a.KS + ks) * 2) * 64 + lane;
        a.mfrag[base] = __builtin_bit_cast(uint4, hi);
        a.mfrag[base + 64] = __builtin_bit_cast(uint4, lo);
    }
    for (int t = tid; t < P * 32; t += 256) {
        const int q = t >> 5, sl = t & 31;
        a.mt[((size_t)tile * P + q) * 32 + sl] = (float)ldexp(a.h[q / K1] * st[sl * LD + q] * a.colscale[q], -sexp[sl]);
    }
}

int launch_stage(const StageArgs& a, hipStream_t s)
{
    if (a.n_tiles == 0) return GD_OK;
    if (a.P > kStageMaxP) return fail(GD_EUNSUPPORTED, "P too large for the stage kernel");
    hipLaunchKernelGGL(k_stage, dim3(a.n_tiles), dim3(256), 0, s, a);
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

int launch_project(const double* samples, const double* wP, double* coef, int C, int N, int k, hipStream_t s)
{
    const long long n = (long long)C * N;
    if (n == 0) return GD_OK;
    hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, samples, wP, coef, C, N, k);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

} // namespace gd
