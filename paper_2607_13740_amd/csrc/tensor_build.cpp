// Host FP64 construction of the collision tensor T.
//
// With the quadrature rule fixed, the DG right-hand side (Sec. 3.1, Eq. evo)
// depends on the coefficients g only through the fluxes F(x) at the bin edges and
// at the interior Gauss nodes (Sec. 3.3), and each F(x) is a quadratic form in g:
// the nested Gauss-Legendre sums of the truncated coagulation and fragmentation
// fluxes (Eqs. Fcoagtrun, Ffragtrun; inner fragment-mass integrals of App. B,
// Eqs. inte1/inte2) multiply g(u) by g(v) node by node.  Collecting the
// contribution of every node pair to every pair of Legendre coefficients gives
//     Y_o = sum_{p,q} T[o][p][q] g_p g_q,
// with one row o per interior edge flux F(e_j) (plus F(e_N) for the
// non-conservative truncation) and one per volume moment
// V_{j,i} = sum_theta w_theta P_i'(s_theta) F(x_j^theta), i >= 1.
//
// This file walks the nodes once per tensor; the GPU evaluates the quadratic
// form for many cells at once.
#include "tensor_build.h"

#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <cstring>
#include <stdexcept>

namespace gd {

// Gauss-Legendre nodes/weights on [-1,1] by Newton's method on P_n, starting from
// the Chebyshev-like guess cos(pi (i + 3/4) / (n + 1/2)); weights 2/((1-x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // one more derivative evaluation at the converged node
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = z;   // ascending order
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Legendre values P_0..P_k and derivatives at xi (three-term recurrence).
static void legendre_all(int k, double xi, double* P, double* dP)
{
    P[0] = 1.0;
    if (dP) dP[0] = 0.0;
    if (k >= 1) { P[1] = xi; if (dP) dP[1] = 1.0; }
    for (int n = 1; n < k; ++n) {
        P[n + 1] = ((2 * n + 1) * xi * P[n] - n * P[n - 1]) / (n + 1);
        if (dP) dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n];
    }
}

namespace {

struct Node { double x, w; int bin; };

struct Ctx {
    const TensorSpec* sp;
    std::vector<double> e;   // edges
    std::vector<double> s, w;
    double beta;              // 2 + alpha
    double xmin_beta;
    // Maxwellian kernel: outcome probabilities (coagulation; fragmentation per level)
    double p_coag = 1.0;
    std::vector<double> p_frag;
};

// composite rule over [a,b], split at edges (Sec. 3.3, the partial bins A..B)
void pieces(const Ctx& c, double a, double b, std::vector<Node>& out)
{
    out.clear();
    if (!(b > a)) return;
    const int N = c.sp->bins;
    // first bin whose right edge exceeds a
    int j0 = int(std::upper_bound(c.e.begin(), c.e.end(), a) - c.e.begin()) - 1;
    j0 = std::max(0, std::min(j0, N - 1));
    for (int j = j0; j < N; ++j) {
        double lo = std::max(a, c.e[j]);
        double hi = std::min(b, c.e[j + 1]);
        if (c.e[j] >= b) break;
        if (!(hi > lo)) continue;
        double m = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
        for (size_t q = 0; q < c.s.size(); ++q) out.push_back({m + hw * c.s[q], hw * c.w[q], j});
    }
}

double kernel_value(const TensorSpec& sp, double u, double v)
{
    switch (sp.kernel) {
    case GD_KERNEL_CONST: return 1.0;
    case GD_KERNEL_ADDITIVE: return u + v;
    case GD_KERNEL_MULTIPLICATIVE: return u * v;
    default: {
        double r = std::cbrt(u) + std::cbrt(v);
        return r * r * sp.v0 * (std::pow(u, -1.0 / 6.0) + std::pow(v, -1.0 / 6.0));
    }
    }
}

// relative velocity deciding the collision outcome at a node pair
double rel_speed(const TensorSpec& sp, double u, double v)
{
    return sp.v0 * (std::pow(u, -1.0 / 6.0) + std::pow(v, -1.0 / 6.0));
}

// Probability that a Maxwellian relative speed with rms s is below vb (sticking)
// or above vf (fragmentation), Sec. 4.5: with a = sqrt(3/2)/s the speed CDF is
// erf(a V) - (2/sqrt(pi)) a V exp(-a^2 V^2).
double maxwell_below(double vb, double s)
{
    const double z = std::sqrt(1.5) * vb / s;
    return std::erf(z) - 2.0 / std::sqrt(M_PI) * z * std::exp(-z * z);
}
double maxwell_above(double vf, double s) { return 1.0 - maxwell_below(vf, s); }

// Geometric cross section times the rms speed of the Maxwellian kernel.
double maxwell_rate(const TensorSpec& sp, double u, double v)
{
    const double r = std::cbrt(u) + std::cbrt(v);
    return M_PI * r * r * sp.v0;
}

// Mass of the power-law fragments of a (u,v) collision by the mass-ratio law of
// Eq. mfrag; the rest, u + v minus this, is the remnant.  (u+v)/(1+q) = min(u,v).
double general_frag_mass(double u, double v)
{
    const double lo = std::min(u, v), q = std::max(u, v) / lo;
    if (q <= 10.0) return u + v;                                                  // destructive
    if (q <= 12.0) return lo * (6.5 + 4.5 * std::cos(M_PI * (q - 10.0) / 2.0));  // transition I
    if (q <= 15.0) return 2.0 * lo;                                               // cratering
    if (q <= 50.0) return lo * (1.45 + 0.55 * std::cos(M_PI * (q - 15.0) / 35.0)); // transition II
    return 0.9 * lo;                                                              // mass transfer
}

// fragment mass above x produced by a (u,v) collision: int_x^{u+v} w b(w,u,v) dw
double mass_above(const Ctx& c, double x, double u, double v)
{
    const double S = u + v;
    switch (c.sp->frag) {
    case GD_FRAG_POWERLAW: {
        if (x >= S) return 0.0;
        double Sb = std::pow(S, c.beta);
        return S * (Sb - std::pow(x, c.beta)) / (Sb - c.xmin_beta);
    }
    case GD_FRAG_UNIFORM_BINARY: {
        double r = 0.0;
        if (x < u) r += u - x * x / u;
        if (x < v) r += v - x * x / v;
        return r;
    }
    case GD_FRAG_REMNANT_ONLY: return x < S ? S : 0.0;
    case GD_FRAG_GENERAL: {
        // power law A w^alpha on [x_min, m_frag], A/(2+alpha) = m_frag/(m_frag^b - x_min^b)
        // (Eq. inte1); a fragment mass at or below x_min lies below every x
        const double mf = general_frag_mass(u, v), rem = S - mf;
        double r = (x < rem) ? rem : 0.0;
        if (mf > c.sp->x_min && x < mf) {
            const double mb = std::pow(mf, c.beta);
            r += mf * (mb - std::pow(x, c.beta)) / (mb - c.xmin_beta);
        }
        return r;
    }
    default: return 0.0;
    }
}

// fragment mass in [x_min, x]: int_{x_min}^x w b(w,u,v) dw
double mass_below(const Ctx& c, double x, double u, double v)
{
    const double S = u + v, xm = c.sp->x_min;
    switch (c.sp->frag) {
    case GD_FRAG_POWERLAW: {
        double top = std::min(x, S);
        double Sb = std::pow(S, c.beta);
        return S * (std::pow(top, c.beta) - c.xmin_beta) / (Sb - c.xmin_beta);
    }
    case GD_FRAG_UNIFORM_BINARY: {
        double a = std::min(x, u), b = std::min(x, v);
        return (a * a - xm * xm) / u + (b * b - xm * xm) / v;
    }
    case GD_FRAG_REMNANT_ONLY: return (xm < S && S < x) ? S : 0.0;
    case GD_FRAG_GENERAL: {
        // Eq. inte2
        const double mf = general_frag_mass(u, v), rem = S - mf;
        double r = (xm < rem && rem < x) ? rem : 0.0;
        if (mf > xm) {
            const double mb = std::pow(mf, c.beta);
            r += mf * (std::pow(std::min(x, mf), c.beta) - c.xmin_beta) / (mb - c.xmin_beta);
        } else {
            r += mf;
        }
        return r;
    }
    default: return 0.0;
    }
}

// Quadratic form of F(x) for every threshold level: B[r][p][q] with F = sum B g_p g_q.
// with_frag = false keeps the coagulation part only (the general law's volume
// moments take their fragmentation part from the reordered integral below).
void flux_form(const Ctx& c, double x, bool with_frag, std::vector<double>& B, std::vector<Node>& un,
               std::vector<Node>& vn, std::vector<double>& acc)
{
    const TensorSpec& sp = *c.sp;
    const int N = sp.bins, K1 = sp.order + 1, P = N * K1;
    const int R = std::max(1, int(sp.levels.size()));
    const bool frag = sp.frag != GD_FRAG_NONE && with_frag;
    const bool maxwell = sp.kernel == GD_KERNEL_MAXWELL;
    std::fill(B.begin(), B.end(), 0.0);
    double Pu[16], Pv[16];
    acc.assign(size_t(R) * P, 0.0);

    auto close_u = [&](const Node& un_) {
        // B[r][(l,a)][q] += wu P_a(xi_l(u)) acc[r][q]
        double h = c.e[un_.bin + 1] - c.e[un_.bin];
        legendre_all(sp.order, 2.0 * (un_.x - 0.5 * (c.e[un_.bin] + c.e[un_.bin + 1])) / h, Pu, nullptr);
        for (int r = 0; r < R; ++r) {
            const double* ar = &acc[size_t(r) * P];
            for (int a = 0; a < K1; ++a) {
                double f = un_.w * Pu[a];
                if (f == 0.0) continue;
                double* row = &B[(size_t(r) * P + un_.bin * K1 + a) * P];
                for (int q = 0; q < P; ++q) row[q] += f * ar[q];
            }
        }
    };

    // positive part: u in [x_min, x], v in [x - u + x_min, Vmax(u)]
    pieces(c, sp.x_min, x, un);
    for (const Node& u : un) {
        std::fill(acc.begin(), acc.end(), 0.0);
        double vmax = sp.conservative ? sp.x_max - u.x + sp.x_min : sp.x_max;
        pieces(c, x - u.x + sp.x_min, vmax, vn);
        for (const Node& v : vn) {
            double h = c.e[v.bin + 1] - c.e[v.bin];
            legendre_all(sp.order, 2.0 * (v.x - 0.5 * (c.e[v.bin] + c.e[v.bin + 1])) / h, Pv, nullptr);
            const double above = frag ? mass_above(c, x, u.x, v.x) / (v.x * (u.x + v.x)) : 0.0;
            const bool split = sp.frag != GD_FRAG_NONE;   // sharp outcome decided per pair
            double coag, fr = 0.0, dv = 0.0;
            if (maxwell) {
                const double K = maxwell_rate(sp, u.x, v.x);
                coag = K * c.p_coag / v.x;
                fr = K * above;   // times the level's fragmentation probability
            } else {
                const double K = kernel_value(sp, u.x, v.x);
                coag = K / v.x;
                fr = K * above;
                if (split) dv = rel_speed(sp, u.x, v.x);
            }
            for (int r = 0; r < R; ++r) {
                double val;
                if (maxwell) val = coag + (frag ? fr * c.p_frag[r] : 0.0);
                else val = (!split || dv <= sp.levels[r]) ? coag : fr;
                if (val == 0.0) continue;
                double* ar = &acc[size_t(r) * P + v.bin * K1];
                for (int b = 0; b < K1; ++b) ar[b] += v.w * Pv[b] * val;
            }
        }
        close_u(u);
    }
    if (!frag) return;
    // negative part: u in [x, x_max], v in [x_min, Vmax(u)]
    pieces(c, x, sp.x_max, un);
    for (const Node& u : un) {
        std::fill(acc.begin(), acc.end(), 0.0);
        double vmax = sp.conservative ? sp.x_max - u.x + sp.x_min : sp.x_max;
        pieces(c, sp.x_min, vmax, vn);
        for (const Node& v : vn) {
            double h = c.e[v.bin + 1] - c.e[v.bin];
            legendre_all(sp.order, 2.0 * (v.x - 0.5 * (c.e[v.bin] + c.e[v.bin + 1])) / h, Pv, nullptr);
            const double K = maxwell ? maxwell_rate(sp, u.x, v.x) : kernel_value(sp, u.x, v.x);
            const double val = -K * mass_below(c, x, u.x, v.x) / (v.x * (u.x + v.x));
            const double dv = maxwell ? 0.0 : rel_speed(sp, u.x, v.x);
            for (int r = 0; r < R; ++r) {
                double vr;
                if (maxwell) vr = val * c.p_frag[r];
                else vr = (dv > sp.levels[r]) ? val : 0.0;
                if (vr == 0.0) continue;
                double* ar = &acc[size_t(r) * P + v.bin * K1];
                for (int b = 0; b < K1; ++b) ar[b] += v.w * Pv[b] * vr;
            }
        }
        close_u(u);
    }
}

// ---------------------------------------------------------------------------
// General law (Eq. break with Eq. mfrag): the fragmentation part of the volume
// moments int_{I_j} F dphi_i/dx dx with the order of integration exchanged (App. B).
// The remnant makes F jump in x, so instead of F at Gauss nodes in x, every node pair
// (u, v) of the outer sums -- u over the whole domain, v over [x_min, Vmax(u)] with the
// Delta x of the flux -- integrates the x-ranges on which each piece of the inner
// integrals is active (Eqs. inte1/inte2), with a Q-point rule per range:
//   u < x <= u + v - x_min (positive flux; the upper bound is the lower v-limit of
//   Eq. Ffragtrun read for x):  power law above x while x < m_frag, remnant while x < m_left;
//   x < u (negative flux): power law between x_min and min(x, m_frag), remnant once
//   m_left (> x_min) lies below x.
// A fragment mass at or below x_min leaves no power law inside the domain: the whole
// fragment mass counts below every x.
void general_x_integrals(const Ctx& c, double u, double v, std::vector<double>& X)
{
    const TensorSpec& sp = *c.sp;
    const int N = sp.bins, k = sp.order, Q = int(c.s.size());
    std::fill(X.begin(), X.end(), 0.0);
    const double xm = sp.x_min, S = u + v, mf = general_frag_mass(u, v), rem = S - mf;
    const double cap = S - xm;
    const bool inside = mf > xm;
    const double nrm = inside ? mf / (std::pow(mf, c.beta) - c.xmin_beta) : 0.0;   // A/(2+alpha)
    const double mfb = inside ? std::pow(mf, c.beta) : 0.0;
    double dP[16], Pv[16];
    // add int_{[lo,hi] ^ I_j} f(x) dphi_i/dx dx for every bin the range meets
    auto range = [&](double lo, double hi, auto f) {
        if (!(hi > lo)) return;
        int j = int(std::upper_bound(c.e.begin(), c.e.end(), lo) - c.e.begin()) - 1;
        j = std::max(0, j);
        for (; j < N && c.e[j] < hi; ++j) {
            const double a = std::max(lo, c.e[j]), b = std::min(hi, c.e[j + 1]);
            if (!(b > a)) continue;
            const double h = c.e[j + 1] - c.e[j], mid = 0.5 * (c.e[j] + c.e[j + 1]);
            const double cm = 0.5 * (a + b), hw = 0.5 * (b - a);
            for (int t = 0; t < Q; ++t) {
                const double x = cm + hw * c.s[t];
                legendre_all(k, 2.0 * (x - mid) / h, Pv, dP);
                const double wf = hw * c.w[t] * f(x) * (2.0 / h);
                for (int i = 1; i <= k; ++i) X[size_t(j) * k + i - 1] += wf * dP[i];
            }
        }
    };
    if (inside) {
        range(u, std::min(mf, cap), [&](double x) { return nrm * (mfb - std::pow(x, c.beta)); });
        range(xm, u, [&](double x) { return -nrm * (std::pow(x, c.beta) - c.xmin_beta); });
        range(mf, u, [&](double x) { return nrm * (std::pow(x, c.beta) - mfb); });
    } else {
        range(xm, u, [&](double) { return -mf; });
    }
    if (rem > xm) {
        range(u, std::min(rem, cap), [&](double) { return rem; });
        range(rem, u, [&](double) { return -rem; });
    }
}

// Adds the reordered fragmentation part to the volume rows (vbase + j*k + i - 1) of
// every level.  Threads own disjoint sets of u bins (the p = (l, a) index of T), so the
// summation order of every entry is fixed.
void general_volume(const Ctx& c, HostTensor& out, int vbase)
{
    const TensorSpec& sp = *c.sp;
    const int N = sp.bins, k = sp.order, K1 = k + 1, P = N * K1, NO = out.n_out;
    const int R = std::max(1, int(sp.levels.size()));
    const bool maxwell = sp.kernel == GD_KERNEL_MAXWELL;
    std::atomic<int> next{0};
    auto worker = [&]() {
        std::vector<Node> un, vn;
        std::vector<double> X(size_t(N) * k);
        double Pu[16], Pv[16];
        for (int l = next++; l < N; l = next++) {
            pieces(c, c.e[l], c.e[l + 1], un);
            for (const Node& u : un) {
                const double hu = c.e[u.bin + 1] - c.e[u.bin];
                legendre_all(k, 2.0 * (u.x - 0.5 * (c.e[u.bin] + c.e[u.bin + 1])) / hu, Pu, nullptr);
                const double vmax = sp.conservative ? sp.x_max - u.x + sp.x_min : sp.x_max;
                pieces(c, sp.x_min, vmax, vn);
                for (const Node& v : vn) {
                    const double hv = c.e[v.bin + 1] - c.e[v.bin];
                    legendre_all(k, 2.0 * (v.x - 0.5 * (c.e[v.bin] + c.e[v.bin + 1])) / hv, Pv, nullptr);
                    general_x_integrals(c, u.x, v.x, X);
                    const double K = maxwell ? maxwell_rate(sp, u.x, v.x) : kernel_value(sp, u.x, v.x);
                    const double dv = maxwell ? 0.0 : rel_speed(sp, u.x, v.x);
                    const double w = u.w * v.w * K / (v.x * (u.x + v.x));
                    for (int r = 0; r < R; ++r) {
                        const double pf = maxwell ? c.p_frag[r] : (dv > sp.levels[r] ? 1.0 : 0.0);
                        if (pf == 0.0) continue;
                        for (int o = 0; o < N * k; ++o) {
                            const double val = w * pf * X[o];
                            if (val == 0.0) continue;
                            double* rowT = &out.T[(size_t(r) * NO + vbase + o) * P * P];
                            for (int a = 0; a < K1; ++a) {
                                double* dst = rowT + size_t(u.bin * K1 + a) * P + v.bin * K1;
                                const double f = val * Pu[a];
                                for (int b = 0; b < K1; ++b) dst[b] += f * Pv[b];
                            }
                        }
                    }
                }
            }
        }
    };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, unsigned(N));
    std::vector<std::thread> th;
    for (unsigned i = 1; i < nth; ++i) th.emplace_back(worker);
    worker();
    for (auto& x : th) x.join();
}

} // namespace

int n_out_rows(const TensorSpec& sp)
{
    return (sp.bins - 1) + (sp.conservative ? 0 : 1) + sp.bins * sp.order;
}

std::vector<double> make_edges(int N, double x_min, double x_max)
{
    std::vector<double> e(N + 1);
    const double ratio = x_max / x_min;
    for (int j = 0; j <= N; ++j) e[j] = x_min * std::pow(ratio, double(j) / double(N));
    e[0] = x_min;
    e[N] = x_max;
    return e;
}

void build_tensor(const TensorSpec& sp, HostTensor& out)
{
    if (sp.bins < 1 || sp.order < 0 || sp.order > 15 || !(sp.x_min > 0) || !(sp.x_max > sp.x_min))
        throw std::invalid_argument("bad grid");
    const int N = sp.bins, k = sp.order, K1 = k + 1, P = N * K1;
    const int Q = sp.quad_points > 0 ? sp.quad_points : K1;
    const int R = std::max(1, int(sp.levels.size()));
    const int NO = n_out_rows(sp);

    Ctx c;
    c.sp = &sp;
    c.e = make_edges(N, sp.x_min, sp.x_max);
    gauss_legendre(Q, c.s, c.w);
    c.beta = 2.0 + sp.alpha;
    c.xmin_beta = std::pow(sp.x_min, c.beta);
    if (sp.kernel == GD_KERNEL_MAXWELL) {
        c.p_coag = maxwell_below(sp.v_bounce, sp.v0);
        for (double vf : sp.levels) c.p_frag.push_back(maxwell_above(vf, sp.v0));
    }

    out.P = P;
    out.n_out = NO;
    out.n_levels = R;
    out.edges = c.e;
    out.T.assign(size_t(R) * NO * P * P, 0.0);

    // flux evaluation points and the rows they feed (edge fluxes with the whole flux;
    // volume nodes without the general law's fragmentation part, which follows App. B)
    const bool reorder = sp.frag == GD_FRAG_GENERAL && k > 0;
    struct Pt { double x; int row0; int nrow; double coef[16]; };
    std::vector<Pt> pts;
    int o = 0;
    for (int j = 1; j < N; ++j) { Pt p{c.e[j], o++, 1, {1.0}}; pts.push_back(p); }
    if (!sp.conservative) { Pt p{c.e[N], o++, 1, {1.0}}; pts.push_back(p); }
    const int vbase = o;
    double Pl[16], dPl[16];
    if (k > 0) {
        for (int j = 0; j < N; ++j) {
            double h = c.e[j + 1] - c.e[j], mid = 0.5 * (c.e[j] + c.e[j + 1]);
            for (int t = 0; t < Q; ++t) {
                Pt p{};
                p.x = mid + 0.5 * h * c.s[t];
                p.row0 = vbase + j * k;
                p.nrow = k;
                legendre_all(k, c.s[t], Pl, dPl);
                for (int i = 1; i <= k; ++i) p.coef[i - 1] = c.w[t] * dPl[i];
                pts.push_back(p);
            }
        }
    }

    // points feeding the same rows (the Q points of one bin) form a group that one
    // thread sums in a fixed order, so that the tensor is the same on every run
    std::vector<int> grp{0};
    for (int t = 1; t < int(pts.size()); ++t)
        if (pts[t].row0 != pts[t - 1].row0) grp.push_back(t);
    const int ngrp = int(grp.size());
    grp.push_back(int(pts.size()));
    std::atomic<int> next{0};
    auto worker = [&]() {
        std::vector<double> B(size_t(R) * P * P), acc;
        std::vector<Node> un, vn;
        un.reserve((N + 2) * Q);
        vn.reserve((N + 2) * Q);
        for (int gi = next++; gi < ngrp; gi = next++)
            for (int t = grp[gi]; t < grp[gi + 1]; ++t) {
                flux_form(c, pts[t].x, !(reorder && pts[t].row0 >= vbase), B, un, vn, acc);
                for (int r = 0; r < R; ++r)
                    for (int i = 0; i < pts[t].nrow; ++i) {
                        const double cf = pts[t].coef[i];
                        double* dst = &out.T[(size_t(r) * NO + pts[t].row0 + i) * P * P];
                        const double* src = &B[size_t(r) * P * P];
                        for (int q = 0; q < P * P; ++q) dst[q] += cf * src[q];
                    }
            }
    };
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, unsigned(ngrp));
    std::vector<std::thread> th;
    for (unsigned i = 1; i < nth; ++i) th.emplace_back(worker);
    worker();
    for (auto& x : th) x.join();
    if (reorder) general_volume(c, out, vbase);
}

} // namespace gd
