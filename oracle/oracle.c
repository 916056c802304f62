/*
 * FP64 CPU oracle for the GRACE-DG collision operator (Yang, Chen & Bai,
 * "GRACE-DG: A Discontinuous Galerkin Method-Based Code for General Nonlinear
 * Coagulation-Fragmentation Equations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * It evaluates the paper's discrete operator directly: the nested
 * Gauss-Legendre sums of the truncated coagulation and fragmentation fluxes
 * (Sec. 3.3, Eqs. Fcoagtrun and Ffragtrun, with the inner fragment-mass
 * integrals of App. B, Eqs. inte1/inte2), assembled into the DG right-hand
 * side (Sec. 3.1, Eq. evo), the scaling limiter (Sec. 3.2, Eqs. recon/gamma)
 * and the SSP-RK3 step (Eq. RK3).  No tensor is precomputed; every call walks
 * the quadrature nodes again.  Plain loops, FP64, OpenMP across hydro cells only.
 *
 * The Gauss-Legendre rule (nodes/weights on [-1,1]) is passed in by the
 * caller, which takes it from a library routine.
 *
 * Readings of points the paper leaves open (each one is listed with its reason
 * in the design notes):
 *  - grid: e_j = x_min exp(j ln(x_max/x_min)/N), bin centre = arithmetic
 *    midpoint (Sec. 3.1 says "logarithmic grid" and defines the centre as
 *    the midpoint);
 *  - the u-integral for a flux at an interior node x_j^theta includes the
 *    partial bin [e_j, x_j^theta] with its own Q-point rule (Sec. 3.3 only says
 *    "x_{j+1/2} simply replaced by x_j^theta");
 *  - every integration range is split at every bin edge inside it and pieces
 *    of zero length are skipped (Sec. 3.3, the A..B partial-bin sums);
 *  - the sharp collision outcome: a node pair (u,v) fragments iff
 *    dv(u,v) = v0 (u^-1/6 + v^-1/6) > v_frag, else it coagulates;
 *  - the Maxwellian kernel of Sec. 4.5 keeps the paper's pi in the cross
 *    section and takes the rms speed constant (the paper's toy model), so both
 *    outcome probabilities are constants; every node pair coagulates and
 *    fragments with these weights (no sharp split);
 *  - the general breakage law (Eq. break with Eq. mfrag): a remnant at or below
 *    x_min is outside the domain and contributes to neither inner integral; the
 *    fragmentation part of its volume moments takes the reordered x-integral of
 *    App. B with one Delta x in both parts of the flux and the positive part's
 *    lower v-limit carried over to x (x <= u + v - x_min); the coagulation part
 *    and every other law use F at the Gauss nodes of the bin;
 *  - per-cell v_frag between tabulated levels: the raw flux vector is the
 *    linear blend of the two neighbouring level evaluations (clamped at the
 *    ends);
 *  - the limiter with a non-positive cell average flattens the bin (gamma=0);
 *    a negative average is counted as a positivity violation.  The limiter is
 *    applied to the initial state and after every RK stage;
 *  - the CFL bound of Eq. dt runs over the bins that lose mass (only those can
 *    turn negative in a forward-Euler stage) and hold a positive average; the
 *    per-cell steps take it at the start state of every sub-step.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ---- enums mirrored by value in oracle.py (not shared with the library) ---- */
enum { OK_CONST = 0, OK_ADDITIVE = 1, OK_MULTIPLICATIVE = 2, OK_BALLISTIC = 3, OK_MAXWELL = 4 };
enum { OF_NONE = 0, OF_POWERLAW = 1, OF_UNIFORM_BINARY = 2, OF_REMNANT_ONLY = 3, OF_GENERAL = 4 };

typedef struct {
    int N, k, Q;            /* mass bins, Legendre degree, GL points per piece */
    const double *s, *w;    /* GL nodes / weights on [-1,1], length Q           */
    double xmin, xmax;
    int conservative;       /* 1: dx = -u + x_min ; 0: dx = 0                    */
    int kern;               /* OK_*                                              */
    double v0;              /* relative-velocity scale of the threshold          */
    int frag;               /* OF_*                                              */
    double alpha;           /* power-law index of the fragment distribution      */
    double vb;              /* bouncing threshold of the Maxwellian kernel        */
} ocfg;

/* per-evaluation parameters that vary by cell */
typedef struct {
    double vfrag;           /* sharp fragmentation threshold                     */
    double kscale;          /* multiplies both kernels                           */
} ocell;

/* ---------------------------------------------------------------- grid (Sec 3.1) */
static void make_edges(const ocfg* c, double* e)
{
    double lr = log(c->xmax / c->xmin);
    for (int j = 0; j <= c->N; ++j) e[j] = c->xmin * exp(lr * (double)j / (double)c->N);
    e[0] = c->xmin;
    e[c->N] = c->xmax;
}

/* ---------------------------------------------------- Legendre basis (Eq. 2.4) */
static double legendre(int n, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = x;
    for (int m = 1; m < n; ++m) {
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        p0 = p1; p1 = p2;
    }
    return p1;
}

/* P_n'(x) from P'_{m+1} = P'_{m-1} + (2m+1) P_m */
static double legendre_d(int n, double x)
{
    if (n == 0) return 0.0;
    double dm1 = 0.0, d = 1.0;     /* P'_0, P'_1 */
    for (int m = 1; m < n; ++m) {
        double dn = dm1 + (2.0 * m + 1.0) * legendre(m, x);
        dm1 = d; d = dn;
    }
    return d;
}

/* value of the DG polynomial of bin j at mass x (Eq. 2.3) */
static double g_at(const ocfg* c, const double* e, const double* g, int j, double x)
{
    double h = e[j + 1] - e[j], mid = 0.5 * (e[j] + e[j + 1]);
    double xi = 2.0 * (x - mid) / h;
    double acc = 0.0;
    for (int i = 0; i <= c->k; ++i) acc += g[j * (c->k + 1) + i] * legendre(i, xi);
    return acc;
}

/* ------------------------------------------------------------- kernels */
static double kernel_K(const ocfg* c, double u, double v)
{
    switch (c->kern) {
    case OK_CONST: return 1.0;
    case OK_ADDITIVE: return u + v;
    case OK_MULTIPLICATIVE: return u * v;
    default: {
        double a = cbrt(u) + cbrt(v);
        return a * a * c->v0 * (pow(u, -1.0 / 6.0) + pow(v, -1.0 / 6.0));
    }
    }
}

static double rel_velocity(const ocfg* c, double u, double v)
{
    return c->v0 * (pow(u, -1.0 / 6.0) + pow(v, -1.0 / 6.0));
}

/* Probability that the relative speed is at most V when speeds follow the
 * Maxwellian of Sec. 4.5 with rms s (the paper's closed form of beta_coag). */
static double maxwell_cdf(double V, double s)
{
    double a = sqrt(3.0 / (2.0 * s * s));
    return erf(a * V) - V * sqrt(6.0 / (M_PI * s * s)) * exp(-3.0 * V * V / (2.0 * s * s));
}

/* split into coagulating and fragmenting parts at one node pair */
static void kernel_split(const ocfg* c, const ocell* p, double u, double v, double* kc, double* kf)
{
    if (c->kern == OK_MAXWELL) {
        /* K_coag = sigma dv_rms beta_coag, K_frag = sigma dv_rms beta_frag (Sec. 4.5) */
        double r = cbrt(u) + cbrt(v);
        double sv = p->kscale * M_PI * r * r * c->v0;
        *kc = sv * maxwell_cdf(c->vb, c->v0);
        *kf = (c->frag == OF_NONE) ? 0.0 : sv * (1.0 - maxwell_cdf(p->vfrag, c->v0));
        return;
    }
    double K = p->kscale * kernel_K(c, u, v);
    if (c->frag == OF_NONE) { *kc = K; *kf = 0.0; return; }
    if (rel_velocity(c, u, v) > p->vfrag) { *kc = 0.0; *kf = K; }
    else { *kc = K; *kf = 0.0; }
}

/* ------------------------------------------- inner w-integrals (App. B, inte1/2)
 * Pw = int_x^{u+v} w b(w,u,v) dw ,  Nw = int_{x_min}^x w b(w,u,v) dw              */

/* mass of the power-law fragments of a (u,v) collision, Eq. mfrag (after Li 2022),
 * with the mass ratio q = max(u,v)/min(u,v) */
static double mfrag_general(double u, double v)
{
    double S = u + v, q = (u > v) ? u / v : v / u;
    if (q <= 10.0) return S;                                                        /* destructive   */
    if (q <= 12.0) return S / (1.0 + q) * (6.5 + 4.5 * cos((q - 10.0) / (12.0 - 10.0) * M_PI));
    if (q <= 15.0) return S * 2.0 / (1.0 + q);                                      /* cratering     */
    if (q <= 50.0) return S / (1.0 + q) * (1.45 + 0.55 * cos((q - 15.0) / (50.0 - 15.0) * M_PI));
    return S * 0.9 / (1.0 + q);                                                     /* mass transfer */
}

/* A/(2+alpha) of the power-law part, A = (2+alpha) m_frag/(m_frag^(2+alpha) - x_min^(2+alpha)) */
static double general_norm(const ocfg* c, double mf)
{
    double be = 2.0 + c->alpha;
    return mf / (pow(mf, be) - pow(c->xmin, be));
}
static double Pw(const ocfg* c, double x, double u, double v)
{
    double S = u + v;
    switch (c->frag) {
    case OF_POWERLAW: {
        /* destructive: m_frag = u+v, no remnant; A/(2+alpha) = S/D */
        if (x >= S) return 0.0;
        double be = 2.0 + c->alpha;
        double D = pow(S, be) - pow(c->xmin, be);
        return S * (pow(S, be) - pow(x, be)) / D;
    }
    case OF_UNIFORM_BINARY: {
        double r = 0.0;
        if (x < u) r += (u * u - x * x) / u;
        if (x < v) r += (v * v - x * x) / v;
        return r;
    }
    case OF_REMNANT_ONLY:
        return (x < S) ? S : 0.0;
    case OF_GENERAL: {
        /* Eq. inte1: power law above x (x < m_frag) plus the remnant (x < m_left) */
        double mf = mfrag_general(u, v), ml = S - mf, be = 2.0 + c->alpha, r = 0.0;
        if (x < mf && mf > c->xmin) r += general_norm(c, mf) * (pow(mf, be) - pow(x, be));
        if (x < ml) r += ml;
        return r;
    }
    default:
        return 0.0;
    }
}

static double Nw(const ocfg* c, double x, double u, double v)
{
    double S = u + v;
    switch (c->frag) {
    case OF_POWERLAW: {
        double be = 2.0 + c->alpha;
        double D = pow(S, be) - pow(c->xmin, be);
        double top = (x < S) ? x : S;
        return S * (pow(top, be) - pow(c->xmin, be)) / D;
    }
    case OF_UNIFORM_BINARY: {
        double mu = (x < u) ? x : u, mv = (x < v) ? x : v;
        return (mu * mu - c->xmin * c->xmin) / u + (mv * mv - c->xmin * c->xmin) / v;
    }
    case OF_REMNANT_ONLY:
        return (c->xmin < S && S < x) ? S : 0.0;
    case OF_GENERAL: {
        /* Eq. inte2: power law from x_min up to min(x, m_frag) plus the remnant
         * when it lies inside (x_min, x); with m_frag <= x_min the whole fragment
         * mass is below every x (the ratio of the formula is 1) */
        double mf = mfrag_general(u, v), ml = S - mf, be = 2.0 + c->alpha, r;
        if (mf > c->xmin) {
            double top = (x < mf) ? x : mf;
            r = general_norm(c, mf) * (pow(top, be) - pow(c->xmin, be));
        } else {
            r = mf;
        }
        if (c->xmin < ml && ml < x) r += ml;
        return r;
    }
    default:
        return 0.0;
    }
}

/* ---------------------------------------- composite GL rule G[a,b] (Sec. 3.3)
 * Split [a,b] at every bin edge inside it, skip pieces of length <= 0, map the Q
 * nodes to every piece.  Returns the node count; bin[] says which polynomial
 * evaluates g at the node.                                                        */
static int composite(const ocfg* c, const double* e, double a, double b,
                     double* x, double* wt, int* bin)
{
    int n = 0;
    if (!(b > a)) return 0;
    for (int j = 0; j < c->N; ++j) {
        double lo = (a > e[j]) ? a : e[j];
        double hi = (b < e[j + 1]) ? b : e[j + 1];
        if (!(hi > lo)) continue;
        double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        for (int q = 0; q < c->Q; ++q) {
            x[n] = mid + half * c->s[q];
            wt[n] = half * c->w[q];
            bin[n] = j;
            ++n;
        }
    }
    return n;
}

/* ---------------------------------------------- flux at one mass point (O6)
 * F(x) = sum_{u in G[xmin,x]} wu g(u) sum_{v in G[x-u+xmin, Vmax(u)]} wv g(v)
 *            [Kc/v + Kf Pw/(v(u+v))]
 *      - sum_{u in G[x,xmax]} wu g(u) sum_{v in G[xmin, Vmax(u)]} wv g(v) Kf Nw/(v(u+v))
 * with Vmax(u) = xmax - u + xmin (conservative) or xmax.                          */
static double flux_at(const ocfg* c, const ocell* p, const double* e, const double* g, double x, int with_frag,
                      double* ux, double* uw, int* ub, double* vx, double* vw, int* vb)
{
    double F = 0.0;
    /* positive part: u < x */
    int nu = composite(c, e, c->xmin, x, ux, uw, ub);
    for (int a = 0; a < nu; ++a) {
        double u = ux[a];
        double gu = g_at(c, e, g, ub[a], u);
        double vmax = c->conservative ? (c->xmax - u + c->xmin) : c->xmax;
        int nv = composite(c, e, x - u + c->xmin, vmax, vx, vw, vb);
        double inner = 0.0;
        for (int b = 0; b < nv; ++b) {
            double v = vx[b];
            double kc, kf;
            kernel_split(c, p, u, v, &kc, &kf);
            if (!with_frag) kf = 0.0;
            double integrand = kc / v;
            if (kf != 0.0) integrand += kf * Pw(c, x, u, v) / (v * (u + v));
            inner += vw[b] * g_at(c, e, g, vb[b], v) * integrand;
        }
        F += uw[a] * gu * inner;
    }
    if (c->frag == OF_NONE || !with_frag) return F;
    /* negative part: u > x */
    nu = composite(c, e, x, c->xmax, ux, uw, ub);
    for (int a = 0; a < nu; ++a) {
        double u = ux[a];
        double gu = g_at(c, e, g, ub[a], u);
        double vmax = c->conservative ? (c->xmax - u + c->xmin) : c->xmax;
        int nv = composite(c, e, c->xmin, vmax, vx, vw, vb);
        double inner = 0.0;
        for (int b = 0; b < nv; ++b) {
            double v = vx[b];
            double kc, kf;
            kernel_split(c, p, u, v, &kc, &kf);
            if (kf == 0.0) continue;
            inner += vw[b] * g_at(c, e, g, vb[b], v) * kf * Nw(c, x, u, v) / (v * (u + v));
        }
        F -= uw[a] * gu * inner;
    }
    return F;
}

/* ------------------------------- reordered volume integral of App. B (general law)
 * With the remnant delta(w - m_left) of Eq. break the fragmentation flux jumps in x
 * wherever x crosses a remnant mass, so the volume moment int_{I_j} F dphi_i/dx dx is
 * not taken at Gauss nodes in x.  Exchanging the order (App. B) puts x innermost:
 * for every node pair (u,v) of the outer sums -- u over the whole domain, v over
 * [x_min, Vmax(u)] -- the x-integrals over I_j cut to the ranges where each term of
 * the inner integrals (Eqs. inte1/inte2) is active run with their own Q-point rule:
 *   positive flux (u < x, and x - u + x_min <= v, i.e. x <= u + v - x_min):
 *     T1  + int_{I_j ^ [u, min(m_frag, u+v-x_min)]}  A/(2+a) (m_frag^(2+a) - x^(2+a))
 *     T4  + int_{I_j ^ [u, min(m_left, u+v-x_min)]}  m_left
 *   negative flux (x < u):
 *     T2  - int_{I_j ^ [x_min, u]}                  A/(2+a) (x^(2+a) - x_min^(2+a))
 *     T3  + int_{I_j ^ [m_frag, u]}                 A/(2+a) (x^(2+a) - m_frag^(2+a))
 *     T5  - int_{I_j ^ [m_left, u]}                 m_left   (a remnant above x_min)
 * each times dphi_i/dx and K_frag g(u) g(v) / (v (u+v)).  The v-limits are those of
 * Eq. Ffragtrun with the same Delta x in both parts (the printed reordered formula
 * mixes x_max and x_max - u + x_min), and the cap x <= u + v - x_min carries the
 * lower v-limit of the positive part over to x.  A fragment mass at or below x_min
 * puts the whole fragment mass below every x: T1 and T3 vanish and T2 becomes
 * - int_{I_j ^ [x_min, u]} m_frag.  Only the fragmentation part is reordered; the
 * coagulation part of the volume moments keeps the node rule of Sec. 3.3.          */
enum { APPB_T1, APPB_T2, APPB_T2_ALL, APPB_T3, APPB_T4, APPB_T5 };

static void appb_piece(const ocfg* c, const double* e, int j, double a, double b, int term, double mf,
                       double ml, double coef, double* V)
{
    double lo = (a > e[j]) ? a : e[j];
    double hi = (b < e[j + 1]) ? b : e[j + 1];
    if (!(hi > lo)) return;
    double h = e[j + 1] - e[j], mid = 0.5 * (e[j] + e[j + 1]);
    double cen = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
    double be = 2.0 + c->alpha, An = (mf > c->xmin) ? general_norm(c, mf) : 0.0;
    for (int q = 0; q < c->Q; ++q) {
        double x = cen + half * c->s[q], f;
        switch (term) {
        case APPB_T1: f = An * (pow(mf, be) - pow(x, be)); break;
        case APPB_T2: f = -An * (pow(x, be) - pow(c->xmin, be)); break;
        case APPB_T2_ALL: f = -mf; break;
        case APPB_T3: f = An * (pow(x, be) - pow(mf, be)); break;
        case APPB_T4: f = ml; break;
        default: f = -ml; break;
        }
        double xi = 2.0 * (x - mid) / h, wf = coef * half * c->w[q] * f * 2.0 / h;
        for (int i = 1; i <= c->k; ++i) V[j * c->k + (i - 1)] += wf * legendre_d(i, xi);
    }
}

/* adds the fragmentation part of V_{j,i} (j < N, 1 <= i <= k) to V [N*k] */
static void vol_frag_reordered(const ocfg* c, const ocell* p, const double* e, const double* g, double* V,
                               double* ux, double* uw, int* ub, double* vx, double* vw, int* vb)
{
    int nu = composite(c, e, c->xmin, c->xmax, ux, uw, ub);
    for (int a = 0; a < nu; ++a) {
        double u = ux[a];
        double gu = g_at(c, e, g, ub[a], u);
        double vmax = c->conservative ? (c->xmax - u + c->xmin) : c->xmax;
        int nv = composite(c, e, c->xmin, vmax, vx, vw, vb);
        for (int b = 0; b < nv; ++b) {
            double v = vx[b];
            double kc, kf;
            kernel_split(c, p, u, v, &kc, &kf);
            if (kf == 0.0) continue;
            double coef = uw[a] * vw[b] * gu * g_at(c, e, g, vb[b], v) * kf / (v * (u + v));
            double mf = mfrag_general(u, v), ml = (u + v) - mf, top = u + v - c->xmin;
            for (int j = 0; j < c->N; ++j) {
                if (mf > c->xmin) {
                    appb_piece(c, e, j, u, (mf < top) ? mf : top, APPB_T1, mf, ml, coef, V);
                    appb_piece(c, e, j, c->xmin, u, APPB_T2, mf, ml, coef, V);
                    appb_piece(c, e, j, mf, u, APPB_T3, mf, ml, coef, V);
                } else {
                    appb_piece(c, e, j, c->xmin, u, APPB_T2_ALL, mf, ml, coef, V);
                }
                if (ml > c->xmin) {
                    appb_piece(c, e, j, u, (ml < top) ? ml : top, APPB_T4, mf, ml, coef, V);
                    appb_piece(c, e, j, ml, u, APPB_T5, mf, ml, coef, V);
                }
            }
        }
    }
}

/* -------------------------------------------- raw flux vector of one cell (O7)
 * Y = [F(e_1) .. F(e_{N-1}), (F(e_N) if non-conservative),
 *      V_{0,1..k}, V_{1,1..k}, ..., V_{N-1,1..k}]
 * with V_{j,i} = sum_theta w_theta P_i'(s_theta) F(c_j + h_j s_theta/2) (Sec. 3.3).
 * Fe gets all N+1 edge fluxes (F(e_0) and, if conservative, F(e_N) evaluate to 0). */
static int n_out(const ocfg* c) { return (c->N - 1) + (c->conservative ? 0 : 1) + c->N * c->k; }

static void raw_flux(const ocfg* c, const ocell* p, const double* e, const double* g, double* Y, double* Fe)
{
    int maxn = (c->N + 2) * c->Q;
    double* ux = malloc(sizeof(double) * maxn);
    double* uw = malloc(sizeof(double) * maxn);
    double* vx = malloc(sizeof(double) * maxn);
    double* vw = malloc(sizeof(double) * maxn);
    int* ub = malloc(sizeof(int) * maxn);
    int* vb = malloc(sizeof(int) * maxn);

    for (int j = 0; j <= c->N; ++j) Fe[j] = flux_at(c, p, e, g, e[j], 1, ux, uw, ub, vx, vw, vb);
    int o = 0;
    for (int j = 1; j < c->N; ++j) Y[o++] = Fe[j];
    if (!c->conservative) Y[o++] = Fe[c->N];
    /* the general law's fragmentation part of the volume moments follows App. B */
    const int reorder = (c->frag == OF_GENERAL);
    double* Vr = calloc((size_t)c->N * (c->k > 0 ? c->k : 1), sizeof(double));
    if (reorder && c->k > 0) vol_frag_reordered(c, p, e, g, Vr, ux, uw, ub, vx, vw, vb);
    for (int j = 0; j < c->N; ++j) {
        double h = e[j + 1] - e[j], mid = 0.5 * (e[j] + e[j + 1]);
        double Fn[64];
        for (int t = 0; t < c->Q; ++t)
            Fn[t] = flux_at(c, p, e, g, mid + 0.5 * h * c->s[t], !reorder, ux, uw, ub, vx, vw, vb);
        for (int i = 1; i <= c->k; ++i) {
            double V = 0.0;
            for (int t = 0; t < c->Q; ++t) V += c->w[t] * legendre_d(i, c->s[t]) * Fn[t];
            Y[o++] = V + Vr[j * c->k + (i - 1)];
        }
    }
    free(Vr);
    free(ux); free(uw); free(vx); free(vw); free(ub); free(vb);
}

/* DG right-hand side from the raw vector (Eq. evo with Eq. 2.5):
 * L_{j,i} = (2i+1)/h_j (V_{j,i} - F_{j+1} P_i(1) + F_j P_i(-1)),  V_{j,0} = 0.     */
static void assemble_L(const ocfg* c, const double* e, const double* Y, double* L)
{
    int N = c->N, k = c->k;
    double* F = malloc(sizeof(double) * (N + 1));
    F[0] = 0.0;
    for (int j = 1; j < N; ++j) F[j] = Y[j - 1];
    F[N] = c->conservative ? 0.0 : Y[N - 1];
    int vbase = (N - 1) + (c->conservative ? 0 : 1);
    for (int j = 0; j < N; ++j) {
        double h = e[j + 1] - e[j];
        for (int i = 0; i <= k; ++i) {
            double V = (i == 0) ? 0.0 : Y[vbase + j * k + (i - 1)];
            double sgn = (i % 2 == 0) ? 1.0 : -1.0;   /* P_i(-1) */
            L[j * (k + 1) + i] = (2.0 * i + 1.0) / h * (V - F[j + 1] + sgn * F[j]);
        }
    }
    free(F);
}

/* raw vector with the per-cell threshold read through the level table */
static void raw_flux_cell(const ocfg* c, const double* e, const double* g, double kscale,
                          double vfrag, int nlev, const double* lev, double* Y, double* Fe)
{
    ocell p = { vfrag, kscale };
    if (nlev < 2 || c->frag == OF_NONE) { raw_flux(c, &p, e, g, Y, Fe); return; }
    int r = 0;
    while (r < nlev - 2 && vfrag >= lev[r + 1]) ++r;
    double th = (vfrag - lev[r]) / (lev[r + 1] - lev[r]);
    if (th < 0.0) th = 0.0;
    if (th > 1.0) th = 1.0;
    int no = n_out(c);
    double* Y1 = malloc(sizeof(double) * no);
    double* F1 = malloc(sizeof(double) * (c->N + 1));
    p.vfrag = lev[r];
    raw_flux(c, &p, e, g, Y, Fe);
    p.vfrag = lev[r + 1];
    raw_flux(c, &p, e, g, Y1, F1);
    for (int o = 0; o < no; ++o) Y[o] = (1.0 - th) * Y[o] + th * Y1[o];
    for (int j = 0; j <= c->N; ++j) Fe[j] = (1.0 - th) * Fe[j] + th * F1[j];
    free(Y1); free(F1);
}

/* ------------------------------------------------------- limiter (Eqs. recon, gamma)
 * Minimum of sum_i g^i P_i on [-1,1]: the end points and the real roots of the
 * derivative inside (-1,1).  For k <= 3 the derivative is at most quadratic:
 *   p'(xi) = g1 + 3 g2 xi + g3 (15 xi^2 - 3)/2.                                    */

/* value of sum_i gi[i] P_i(x) */
static double bin_poly(int k, const double* gi, double x)
{
    double v = 0.0;
    for (int i = 0; i <= k; ++i) v += gi[i] * legendre(i, x);
    return v;
}

static double bin_dpoly(int k, const double* gi, double x)
{
    double v = 0.0;
    for (int i = 1; i <= k; ++i) v += gi[i] * legendre_d(i, x);
    return v;
}

/* minimum of the bin polynomial over [-1,1] (Eq. gamma): the end points and the
 * zeros of its derivative inside.  k <= 3: the derivative is at most quadratic and
 * its roots come from the stable quadratic formula.  k >= 4: the derivative is
 * scanned on a uniform grid of 4096 cells; every sign change is bisected to the
 * last bit (a pair of zeros closer than a cell bounds a local minimum whose depth
 * below the grid values is second order in the cell width). */
static double bin_min(int k, const double* gi)
{
    double m = bin_poly(k, gi, -1.0), v1 = bin_poly(k, gi, 1.0);
    if (v1 < m) m = v1;
    if (k >= 4) {
        const int n = 4096;
        double xa = -1.0, da = bin_dpoly(k, gi, xa);
        for (int t = 1; t <= n; ++t) {
            double xb = -1.0 + 2.0 * (double)t / (double)n, db = bin_dpoly(k, gi, xb);
            if (da < 0.0 && db >= 0.0) {
                double lo = xa, hi = xb;
                for (int it = 0; it < 200 && hi > lo; ++it) {
                    double mid = 0.5 * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    if (bin_dpoly(k, gi, mid) < 0.0) lo = mid; else hi = mid;
                }
                double v = bin_poly(k, gi, 0.5 * (lo + hi));
                if (v < m) m = v;
            }
            xa = xb;
            da = db;
        }
        return m;
    }
    double g1 = k >= 1 ? gi[1] : 0.0, g2 = k >= 2 ? gi[2] : 0.0, g3 = k >= 3 ? gi[3] : 0.0;
    double A = 7.5 * g3, B = 3.0 * g2, Cc = g1 - 1.5 * g3;
    double cand[2];
    int nc = 0;
    if (A != 0.0) {
        double disc = B * B - 4.0 * A * Cc;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double qq = -0.5 * (B + (B >= 0.0 ? sq : -sq));
            if (qq != 0.0) { cand[nc++] = qq / A; cand[nc++] = Cc / qq; }
            else { cand[nc++] = 0.0; }
        }
    } else if (B != 0.0) {
        cand[nc++] = -Cc / B;
    }
    for (int t = 0; t < nc; ++t) {
        double x = cand[t];
        if (x < -1.0 || x > 1.0) continue;
        double val = bin_poly(k, gi, x);
        if (val < m) m = val;
    }
    return m;
}

/* trace: NULL, or a running FNV-1a hash of the bins the limiter changes (gamma < 1),
 * so that two runs can tell whether the limiter's active set differed */
static void trace_mix(unsigned long long* h, unsigned long long v)
{
    *h = (*h ^ v) * 1099511628211ull;
}

static long limit_cell(int N, int k, double* g, unsigned long long* trace)
{
    long viol = 0;
    if (trace) trace_mix(trace, 0xFFFFFFFFull);   /* one mark per limiter call */
    for (int j = 0; j < N; ++j) {
        double* gi = g + j * (k + 1);
        double avg = gi[0];
        double gamma;
        if (avg <= 0.0) {
            /* an empty bin is flattened; a negative average cannot be repaired
             * by scaling and is counted as a positivity violation            */
            gamma = 0.0;
            if (avg < 0.0) ++viol;
        } else {
            double m = bin_min(k, gi);
            gamma = (m < 0.0) ? avg / (avg - m) : 1.0;
            if (gamma > 1.0) gamma = 1.0;
        }
        if (trace && gamma < 1.0) trace_mix(trace, (unsigned long long)j + 1ull);
        for (int i = 1; i <= k; ++i) gi[i] *= gamma;
    }
    return viol;
}

/* ================================================================ public entry points */
static int check(const ocfg* c)
{
    if (c->N < 1 || c->k < 0 || c->k > 16 || c->Q < 1 || c->Q > 64) return -1;
    if (!(c->xmin > 0.0) || !(c->xmax > c->xmin)) return -1;
    return 0;
}

int oracle_n_out(const ocfg* c) { return n_out(c); }

/* inner fragment-mass integrals at one (x,u,v), for unit tests */
int oracle_inner(const ocfg* c, double x, double u, double v, double* pw, double* nw)
{
    *pw = Pw(c, x, u, v);
    *nw = Nw(c, x, u, v);
    return 0;
}

/* the two rates of a node pair and the fragment mass of the general law, for unit tests */
int oracle_rates(const ocfg* c, double u, double v, double kscale, double vfrag, double* kc, double* kf, double* mf)
{
    ocell p = { vfrag, kscale };
    kernel_split(c, &p, u, v, kc, kf);
    *mf = mfrag_general(u, v);
    return 0;
}

int oracle_edges(const ocfg* c, double* e)
{
    if (check(c)) return -1;
    make_edges(c, e);
    return 0;
}

/* flux at arbitrary mass points for one cell (used by the continuous-flux pins) */
int oracle_flux_points(const ocfg* c, const double* g, double kscale, double vfrag,
                       int npts, const double* xs, double* F)
{
    if (check(c)) return -1;
    double* e = malloc(sizeof(double) * (c->N + 1));
    make_edges(c, e);
    int maxn = (c->N + 2) * c->Q;
    double* ux = malloc(sizeof(double) * maxn);
    double* uw = malloc(sizeof(double) * maxn);
    double* vx = malloc(sizeof(double) * maxn);
    double* vw = malloc(sizeof(double) * maxn);
    int* ub = malloc(sizeof(int) * maxn);
    int* vb = malloc(sizeof(int) * maxn);
    ocell p = { vfrag, kscale };
    for (int t = 0; t < npts; ++t) F[t] = flux_at(c, &p, e, g, xs[t], 1, ux, uw, ub, vx, vw, vb);
    free(ux); free(uw); free(vx); free(vw); free(ub); free(vb); free(e);
    return 0;
}

/* raw flux vector Y [C][n_out] and right-hand side L [C][N(k+1)] for a batch */
int oracle_rhs(const ocfg* c, int C, const double* g, const double* kscale, const double* vfrag,
               double vfrag_default, int nlev, const double* lev, double* Y, double* L, double* Fe)
{
    if (check(c) || C < 0) return -1;
    int P = c->N * (c->k + 1), no = n_out(c);
    double* e = malloc(sizeof(double) * (c->N + 1));
    make_edges(c, e);
#pragma omp parallel for schedule(dynamic, 1)
    for (int cell = 0; cell < C; ++cell) {
        double* fe = malloc(sizeof(double) * (c->N + 1));
        double ks = kscale ? kscale[cell] : 1.0;
        double vf = vfrag ? vfrag[cell] : vfrag_default;
        raw_flux_cell(c, e, g + (size_t)cell * P, ks, vf, nlev, lev, Y + (size_t)cell * no, fe);
        if (L) assemble_L(c, e, Y + (size_t)cell * no, L + (size_t)cell * P);
        if (Fe) memcpy(Fe + (size_t)cell * (c->N + 1), fe, sizeof(double) * (c->N + 1));
        free(fe);
    }
    free(e);
    return 0;
}

/* limiter in place over a batch; returns the violation count */
long oracle_limit(const ocfg* c, int C, double* g)
{
    if (check(c) || c->k > 4) return -1;
    int P = c->N * (c->k + 1);
    long viol = 0;
    for (int cell = 0; cell < C; ++cell) viol += limit_cell(c->N, c->k, g + (size_t)cell * P, NULL);
    return viol;
}

/* One SSP-RK3 step (Eq. RK3) of one cell in place on gn, with the limiter after
 * every stage; returns the violations found.  Work arrays of P (y1, y2, L),
 * n_out (Y) and N+1 (fe) doubles. */
static long rk3_cell(const ocfg* c, const double* e, double* gn, double ks, double vf, int nlev,
                     const double* lev, double dt, double* y1, double* y2, double* L, double* Y, double* fe,
                     unsigned long long* trace)
{
    int P = c->N * (c->k + 1);
    long viol = 0;
    raw_flux_cell(c, e, gn, ks, vf, nlev, lev, Y, fe);
    assemble_L(c, e, Y, L);
    for (int t = 0; t < P; ++t) y1[t] = gn[t] + dt * L[t];
    viol += limit_cell(c->N, c->k, y1, trace);

    raw_flux_cell(c, e, y1, ks, vf, nlev, lev, Y, fe);
    assemble_L(c, e, Y, L);
    for (int t = 0; t < P; ++t) y2[t] = 0.75 * gn[t] + 0.25 * (y1[t] + dt * L[t]);
    viol += limit_cell(c->N, c->k, y2, trace);

    raw_flux_cell(c, e, y2, ks, vf, nlev, lev, Y, fe);
    assemble_L(c, e, Y, L);
    for (int t = 0; t < P; ++t) gn[t] = gn[t] / 3.0 + 2.0 / 3.0 * (y2[t] + dt * L[t]);
    viol += limit_cell(c->N, c->k, gn, trace);
    return viol;
}

/* n_steps of SSP-RK3 (Eq. RK3) with the limiter on the initial state and after
 * every stage.  g is [C][N(k+1)] in place. */
long oracle_rk_trace(const ocfg* c, int C, double* g, const double* kscale, const double* vfrag,
                     double vfrag_default, int nlev, const double* lev, double dt, int n_steps,
                     unsigned long long* trace);

long oracle_rk(const ocfg* c, int C, double* g, const double* kscale, const double* vfrag,
               double vfrag_default, int nlev, const double* lev, double dt, int n_steps)
{
    return oracle_rk_trace(c, C, g, kscale, vfrag, vfrag_default, nlev, lev, dt, n_steps, NULL);
}

/* oracle_rk that also hashes, per cell, every bin the limiter changes (trace [C], or NULL) */
long oracle_rk_trace(const ocfg* c, int C, double* g, const double* kscale, const double* vfrag,
                     double vfrag_default, int nlev, const double* lev, double dt, int n_steps,
                     unsigned long long* trace)
{
    if (check(c) || c->k > 4 || C < 0 || n_steps < 0) return -1;
    int P = c->N * (c->k + 1), no = n_out(c);
    double* e = malloc(sizeof(double) * (c->N + 1));
    make_edges(c, e);
    long viol = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : viol)
    for (int cell = 0; cell < C; ++cell) {
        double* gn = g + (size_t)cell * P;
        double* y1 = malloc(sizeof(double) * P);
        double* y2 = malloc(sizeof(double) * P);
        double* L = malloc(sizeof(double) * P);
        double* Y = malloc(sizeof(double) * no);
        double* fe = malloc(sizeof(double) * (c->N + 1));
        double ks = kscale ? kscale[cell] : 1.0;
        double vf = vfrag ? vfrag[cell] : vfrag_default;
        unsigned long long* tr = trace ? trace + cell : NULL;
        if (tr) *tr = 14695981039346656037ull;
        viol += limit_cell(c->N, c->k, gn, tr);
        for (int n = 0; n < n_steps; ++n) viol += rk3_cell(c, e, gn, ks, vf, nlev, lev, dt, y1, y2, L, Y, fe, tr);
        free(y1); free(y2); free(L); free(Y); free(fe);
    }
    free(e);
    return viol;
}

/* Per-cell time steps under the CFL bound (Eq. dt), n_sub sub-steps of SSP-RK3
 * toward the common end time t_end.  t is [C], the time each cell has reached
 * (in/out).  In every sub-step a cell with t < t_end takes
 *     dt = min(dt_max, t_end - t, cfl * B),
 *     B  = min over bins with F(e_{j+1}) - F(e_j) > floor * max_i |F(e_i)| and
 *          g_j^0 > 0 of h_j g_j^0 / (F(e_{j+1}) - F(e_j)),
 * B from the fluxes of its state at the start of the sub-step; t becomes t_end when
 * dt = t_end - t, else t + dt.  A cell with t >= t_end (or dt = 0) is left as it
 * is.  Only a bin that loses mass can turn negative in a forward-Euler stage, and
 * a bin with a zero average cannot be kept positive by any step, so both are left
 * out of B; floor = 0 is the bound as printed, floor > 0 also leaves out bins whose
 * net outflow is below that fraction of the cell's largest edge flux (their
 * positivity is left to the limiter).  The limiter acts on the start state and
 * after every stage, as in oracle_rk. */
long oracle_rk_adaptive(const ocfg* c, int C, double* g, const double* kscale, const double* vfrag,
                        double vfrag_default, int nlev, const double* lev, double cfl, double dt_max,
                        double floor, double t_end, int n_sub, double* t)
{
    if (check(c) || c->k > 4 || C < 0 || n_sub < 0 || !(cfl > 0.0) || !(dt_max > 0.0) || !(floor >= 0.0))
        return -1;
    int P = c->N * (c->k + 1), no = n_out(c);
    double* e = malloc(sizeof(double) * (c->N + 1));
    make_edges(c, e);
    long viol = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : viol)
    for (int cell = 0; cell < C; ++cell) {
        double* gn = g + (size_t)cell * P;
        double* y1 = malloc(sizeof(double) * P);
        double* y2 = malloc(sizeof(double) * P);
        double* L = malloc(sizeof(double) * P);
        double* Y = malloc(sizeof(double) * no);
        double* fe = malloc(sizeof(double) * (c->N + 1));
        double ks = kscale ? kscale[cell] : 1.0;
        double vf = vfrag ? vfrag[cell] : vfrag_default;
        viol += limit_cell(c->N, c->k, gn, NULL);
        for (int n = 0; n < n_sub; ++n) {
            double rem = t_end - t[cell];
            if (!(rem > 0.0)) break;
            raw_flux_cell(c, e, gn, ks, vf, nlev, lev, Y, fe);
            double fmax = 0.0;
            for (int j = 0; j <= c->N; ++j)
                if (fabs(fe[j]) > fmax) fmax = fabs(fe[j]);
            double B = INFINITY;
            for (int j = 0; j < c->N; ++j) {
                double d = fe[j + 1] - fe[j], gj = gn[j * (c->k + 1)];
                if (d > 0.0 && d > floor * fmax && gj > 0.0) {
                    double b = (e[j + 1] - e[j]) * gj / d;
                    if (b < B) B = b;
                }
            }
            double dt = dt_max < rem ? dt_max : rem;
            if (cfl * B < dt) dt = cfl * B;
            if (!(dt > 0.0)) break;
            viol += rk3_cell(c, e, gn, ks, vf, nlev, lev, dt, y1, y2, L, Y, fe, NULL);
            t[cell] = (dt == rem) ? t_end : t[cell] + dt;
        }
        free(y1); free(y2); free(L); free(Y); free(fe);
    }
    free(e);
    return viol;
}

/* Largest dt allowed by the CFL bound (Eq. dt) for the given states.  Only bins
 * that lose mass (F_{j+1} > F_j) can be driven negative by a forward-Euler stage,
 * so the bound is min over such bins of h_j g_j^0 / (F_{j+1} - F_j).              */
double oracle_cfl_dt(const ocfg* c, int C, const double* g, const double* kscale,
                     const double* vfrag, double vfrag_default, int nlev, const double* lev)
{
    if (check(c)) return -1.0;
    int P = c->N * (c->k + 1), no = n_out(c);
    double* e = malloc(sizeof(double) * (c->N + 1));
    make_edges(c, e);
    double best = INFINITY;
    for (int cell = 0; cell < C; ++cell) {
        double* Y = malloc(sizeof(double) * no);
        double* fe = malloc(sizeof(double) * (c->N + 1));
        raw_flux_cell(c, e, g + (size_t)cell * P, kscale ? kscale[cell] : 1.0,
                      vfrag ? vfrag[cell] : vfrag_default, nlev, lev, Y, fe);
        for (int j = 0; j < c->N; ++j) {
            double d = fe[j + 1] - fe[j];
            if (d > 0.0) {
                double t = (e[j + 1] - e[j]) * g[(size_t)cell * P + j * (c->k + 1)] / d;
                if (t < best) best = t;
            }
        }
        free(Y); free(fe);
    }
    free(e);
    return best;
}

/* threads of the batch loops (timing of the oracle itself); n <= 0 keeps the default */
int oracle_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
