// The polynomial of one bin, p(x) = sum_i c_i P_i(x) on the reference interval
// [-1,1] (degree k <= 4), and its minimum there (Sec. 3.2, Eq. gamma): the end
// points and the zeros of p' inside.
//   p'(x) = c1 + 3 c2 x + c3 (15 x^2 - 3)/2 + c4 (35 x^3 - 15 x)/2.
// Up to k = 3 the zeros come from the stable quadratic formula.  For k = 4 the
// zeros of p'' split [-1,1] into intervals on which p' is monotone; a sign change
// of p' on such an interval is bracketed and bisected to the last bit.
#pragma once

#include <hip/hip_runtime.h>

namespace gd {

constexpr int kMaxOrder = 4;

__device__ __forceinline__ double leg(int i, double x)
{
    switch (i) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return 1.5 * x * x - 0.5;
    case 3: return (2.5 * x * x - 1.5) * x;
    default: return (4.375 * x * x - 3.75) * x * x + 0.375;
    }
}

// p at x (K compile-time: the loops unroll and the coefficients stay in registers)
template <int K>
__device__ __forceinline__ double bin_val(const double* c, double x)
{
    double v = c[0];
#pragma unroll
    for (int i = 1; i <= K; ++i) v += c[i] * leg(i, x);
    return v;
}

// zeros of a x^2 + b x + c (stable form); returns how many were written
__device__ __forceinline__ int quad_roots(double a, double b, double c, double* r)
{
    if (a != 0.0) {
        const double d = b * b - 4.0 * a * c;
        if (d < 0.0) return 0;
        const double q = -0.5 * (b + copysign(sqrt(d), b));
        if (q == 0.0) { r[0] = 0.0; return 1; }
        r[0] = q / a;
        r[1] = c / q;
        return 2;
    }
    if (b != 0.0) { r[0] = -c / b; return 1; }
    return 0;
}

// zeros of p' inside (-1,1); returns their number (at most 3)
template <int K>
__device__ __forceinline__ int bin_critical(const double* c, double* r)
{
    if constexpr (K < 2) {
        return 0;
    } else {
        const double c3 = K >= 3 ? c[3] : 0.0;
        int n = 0;
        if constexpr (K <= 3) {
            // p'(x) = a2 x^2 + a1 x + a0
            double q[2];
            const int m = quad_roots(7.5 * c3, 3.0 * c[2], c[1] - 1.5 * c3, q);
            for (int t = 0; t < m; ++t)
                if (q[t] > -1.0 && q[t] < 1.0) r[n++] = q[t];
            return n;
        } else {
            const double c4 = c[4];
            // p'(x) = a3 x^3 + a2 x^2 + a1 x + a0
            const double a3 = 17.5 * c4, a2 = 7.5 * c3, a1 = 3.0 * c[2] - 7.5 * c4, a0 = c[1] - 1.5 * c3;
            if (a3 == 0.0) {
                double q[2];
                const int m = quad_roots(a2, a1, a0, q);
                for (int t = 0; t < m; ++t)
                    if (q[t] > -1.0 && q[t] < 1.0) r[n++] = q[t];
                return n;
            }
            auto dp = [&](double x) { return ((a3 * x + a2) * x + a1) * x + a0; };
            // interval ends: -1, the zeros of p'' inside, 1 (ascending)
            double e[4], q[2];
            int ne = 0;
            e[ne++] = -1.0;
            const int m = quad_roots(3.0 * a3, 2.0 * a2, a1, q);
            if (m == 2 && q[0] > q[1]) { const double t = q[0]; q[0] = q[1]; q[1] = t; }
            for (int t = 0; t < m; ++t)
                if (q[t] > -1.0 && q[t] < 1.0) e[ne++] = q[t];
            e[ne++] = 1.0;
            for (int s = 0; s + 1 < ne; ++s) {
                double lo = e[s], hi = e[s + 1];
                double flo = dp(lo), fhi = dp(hi);
                if (flo == 0.0) { if (lo > -1.0 && n < 3) r[n++] = lo; continue; }
                if ((flo < 0.0) == (fhi < 0.0)) continue;
                for (int it = 0; it < 64; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (!(mid > lo && mid < hi)) break;
                    const double fm = dp(mid);
                    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
                }
                const double x = 0.5 * (lo + hi);
                if (x > -1.0 && x < 1.0 && n < 3) r[n++] = x;
            }
            return n;
        }
    }
}

// minimum of p over [-1,1] and where it is attained
template <int K>
__device__ __forceinline__ double bin_min(const double* c, double* argmin = nullptr)
{
    double xb = -1.0, mb = bin_val<K>(c, -1.0);
    const double v1 = bin_val<K>(c, 1.0);
    if (v1 < mb) { xb = 1.0; mb = v1; }
    double r[3];
    const int n = bin_critical<K>(c, r);
    for (int t = 0; t < n; ++t) {
        const double v = bin_val<K>(c, r[t]);
        if (v < mb) { xb = r[t]; mb = v; }
    }
    if (argmin) *argmin = xb;
    return mb;
}

// the same for an order known only at run time (uniform across the workgroup where
// it is called: one group's order)
__device__ inline double bin_min(int k, const double* c, double* argmin = nullptr)
{
    switch (k) {
    case 0: return bin_min<0>(c, argmin);
    case 1: return bin_min<1>(c, argmin);
    case 2: return bin_min<2>(c, argmin);
    case 3: return bin_min<3>(c, argmin);
    default: return bin_min<4>(c, argmin);
    }
}

} // namespace gd
