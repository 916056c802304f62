// Per-cell and per-bin kernels around the contraction: the scaling limiter
// (Sec. 3.2, Eqs. recon/gamma), the split of the scaled state into FP16 halves,
// the assembly of the DG right-hand side (Sec. 3.1, Eq. evo), the SSP-RK3 stage
// combination (Eq. RK3) and the projection of initial profiles (Eq. init).
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

// ---------------------------------------------------------------------------
// One thread per slot: limiter in place (optional) and, for the split path, the
// per-slot power-of-two scale e with max_q |h_j g_q c_q| 2^-e in [64, 128), the
// hi/lo FP16 B-operand fragments and the FP32 stage-2 weights.
//   mfrag[((tile*KS + ks)*2 + {0 hi, 1 lo})*64 + 32 hh + slot%32] : q = 16 ks + 8 hh + j
//   mt[(tile*P + p)*32 + slot%32]
__global__ __launch_bounds__(256) void k_prologue(PrologueArgs a)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int nslot_pad = a.mixed ? a.n_tiles * 32 : a.n_slots;
    if (s >= nslot_pad) return;
    const int K1 = a.k + 1;
    int cell = -1;
    if (s < a.n_slots) cell = a.perm ? a.perm[s] : s;
    const bool live = cell >= 0;
    double* gc = a.g + (size_t)(live ? cell : 0) * a.P;
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
    double mx = 0.0;
    if (live)
        for (int p = 0; p < a.P; ++p) mx = fmax(mx, fabs(a.h[p / K1] * gc[p] * a.colscale[p]));
    int e = 0;
    if (mx > 0.0) {
        int E;
        frexp(mx, &E);
        e = E - 7;
    }
    if (s < a.n_slots) a.eslot[s] = e;
    const int tile = s >> 5, sl = s & 31;
    for (int ks = 0; ks < a.KS; ++ks)
        for (int hh = 0; hh < 2; ++hh) {
            half8_t hi, lo;
            for (int j = 0; j < 8; ++j) {
                const int q = ks * 16 + hh * 8 + j;
                float m = 0.0f;
                if (live && q < a.P) m = (float)ldexp(a.h[q / K1] * gc[q] * a.colscale[q], -e);
                const _Float16 mh = (_Float16)m;
                hi[j] = mh;
                lo[j] = (_Float16)(m - (float)mh);
            }
            const size_t base = ((size_t)(tile * a.KS + ks) * 2) * 64 + hh * 32 + sl;
            a.mfrag[base] = *reinterpret_cast<uint4*>(&hi);
            a.mfrag[base + 64] = *reinterpret_cast<uint4*>(&lo);
        }
    for (int p = 0; p < a.P; ++p) {
        float m = 0.0f;
        if (live) m = (float)ldexp(a.h[p / K1] * gc[p] * a.colscale[p], -e);
        a.mt[((size_t)tile * a.P + p) * 32 + sl] = m;
    }
}

// ---------------------------------------------------------------------------
// One thread per (slot, bin): fluxes in FP64 and the right-hand side
//   L_{j,i} = (2i+1)/h_j (V_{j,i} - F_{j+1} + (-1)^i F_j)         (Eq. evo, P_i(+-1) = (+-1)^i)
// with F_0 = 0, F_N = 0 (conservative) or row N-1, F_j = row j-1 otherwise.
//   mode 0: out = L                     mode 1: out = gs + dt L
//   mode 2: out = 0.75 gn + 0.25 (gs + dt L)      mode 3: out = gn/3 + 2/3 (gs + dt L)
__global__ __launch_bounds__(256) void k_epilogue(EpilogueArgs a)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)a.n_slots * a.N) return;
    const int s = (int)(t / a.N), j = (int)(t - (long long)s * a.N);
    const int c = a.perm ? a.perm[s] : s;
    if (c < 0) return;
    const int K1 = a.k + 1;
    double fac = a.kscale ? a.kscale[c] : 1.0;
    if (a.Yf) fac = ldexp(fac, 2 * a.eslot[s]);
    auto row = [&](int o) -> double {
        if (a.Yf) return (double)a.Yf[(size_t)s * a.ystride + o] * a.rowscale[o] * fac;
        return a.Yd[(size_t)s * a.ystride + o] * fac;
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

__global__ __launch_bounds__(256) void k_limit(double* g, int C, int N, int k, int P, unsigned long long* viol)
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
int launch_prologue(const PrologueArgs& a, hipStream_t s)
{
    const int n = a.mixed ? a.n_tiles * 32 : a.n_slots;
    if (n == 0) return GD_OK;
    hipLaunchKernelGGL(k_prologue, dim3(cdiv(n, 256)), dim3(256), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_epilogue(const EpilogueArgs& a, hipStream_t s)
{
    const long long n = (long long)a.n_slots * a.N;
    if (n == 0) return GD_OK;
    hipLaunchKernelGGL(k_epilogue, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

int launch_limit(double* g, int C, int N, int k, int P, unsigned long long* viol, hipStream_t s)
{
    if (C == 0) return GD_OK;
    hipLaunchKernelGGL(k_limit, dim3(cdiv(C, 256)), dim3(256), 0, s, g, C, N, k, P, viol);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

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
