// The hydro half of operator splitting: transport of the dust between the hydro
// cells of a plan's group, which form one row in the plan's cell order.  The paper
// splits the collision step from the evolution of the hydrodynamics (Sec. 5.2); this
// is the transport such a split alternates with: first-order upwind finite volumes in
// space for every Legendre coefficient of every mass bin, bin j moving with its own
// velocity.  With Courant number c_j = vel_j dt / dx, |c_j| <= 1,
//     g_c <- (1 - |c_j|) g_c + |c_j| g_{c-1}   (vel_j >= 0; g_{c+1} for vel_j < 0),
// a convex combination of bin polynomials: positivity of every bin polynomial is
// kept and, on a periodic row, the total mass of every bin is kept to round-off.
#include "gd_internal.h"

namespace gd {

// one thread per (cell, coefficient) of a group; out must not alias g
__global__ __launch_bounds__(256) void k_advect(const double* g, double* out, const double* courant, long long C,
                                                int N, int K1, int periodic)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int P = N * K1;
    if (i >= C * P) return;
    const long long c = i / P;
    const int p = int(i - c * P), j = p / K1;
    const double cj = courant[j];
    const double a = fabs(cj);
    long long up = cj >= 0.0 ? c - 1 : c + 1;      // upwind neighbour
    double gu = 0.0;                                 // nothing flows in through an open end
    if (up >= 0 && up < C) gu = g[up * P + p];
    else if (periodic) gu = g[((up + C) % C) * P + p];
    out[i] = (1.0 - a) * g[i] + a * gu;
}

int launch_advect(const double* g, double* out, const double* courant, long long C, int N, int K1, int periodic,
                  hipStream_t s)
{
    const long long n = C * N * K1;
    if (n == 0) return GD_OK;
    hipLaunchKernelGGL(k_advect, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, out, courant, C, N, K1,
                       periodic);
    HIP_TRY(hipGetLastError());
    return GD_OK;
}

} // namespace gd
