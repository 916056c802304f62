// C ABI of libgracedg: tensors (host FP64 build + device schedules), plans
// (groups of hydro cells, workspaces, threshold brackets) and the calls that run
// the right-hand side and the SSP-RK3 step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "gd_internal.h"

namespace gd {

static thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
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

} // namespace gd

using namespace gd;

extern "C" const char* gd_last_error(void) { return g_err.c_str(); }

// ============================================================================ tensors
struct gd_tensor {
    TensorSpec spec;
    HostTensor host;
    int N = 0, k = 0, P = 0, n_out = 0, R = 0;
    int KS = 0, NOB = 0;       // split-FP16 path: K steps of 16, row blocks of 32
    int KS4 = 0, NOB16 = 0;    // FP64 path: K steps of 4, row blocks of 16
    long long nnz = 0;
    size_t bytes = 0;
    bool packed = false;       // device layouts uploaded (by the first plan)
    std::vector<std::unique_ptr<DevBuf>> bufs;
    const double* h = nullptr;
    const double* colscale = nullptr;   // [P]
    const double* rowscale = nullptr;   // [NOB*32]
    Schedule mixed, f64;
};

// folded tensor of level r: Tf[o][p][q] = T[o][p][q] + T[o][q][p] (p < q), T[o][p][p]
static inline double fold(const gd_tensor* t, int r, int o, int p, int q)
{
    const int P = t->P;
    const double* To = &t->host.T[(size_t(r) * t->n_out + o) * P * P];
    return (q == p) ? To[size_t(p) * P + p] : To[size_t(p) * P + q] + To[size_t(q) * P + p];
}

// part value: level r (delta = 0) or level difference r+1 - r (delta = 1)
static inline double part(const gd_tensor* t, int r, int delta, int o, int p, int q)
{
    return delta ? fold(t, r + 1, o, p, q) - fold(t, r, o, p, q) : fold(t, r, o, p, q);
}

static void count_nnz(gd_tensor* t)
{
    long long n = 0;
    for (int o = 0; o < t->n_out; ++o)
        for (int p = 0; p < t->P; ++p)
            for (int q = p; q < t->P; ++q)
                if (fold(t, 0, o, p, q) != 0.0) ++n;
    t->nnz = n;
}

static void make_pairs(int P, std::vector<std::pair<int, int>>& pairs)
{
    pairs.clear();
    for (int i = 0; i < P / 2; ++i) pairs.push_back({i, P - 1 - i});
    if (P & 1) pairs.push_back({P / 2, -1});
}

static inline int pow2_exp(double v)
{
    int E;
    std::frexp(v, &E);
    return E;
}

// Generic schedule builder: row blocks of RB rows, K steps of KW columns, up to SEG
// p segments per iteration.  emit(r, delta, ob, p, ks) appends one fragment;
// blockscale(r, delta, ob) returns the offset of the stage-2 scale table of that
// (part, ob) (or 0).  Every level ends with two empty sentinel descriptors (ob = -1).
template <class Emit, class BlockScale>
static void build_schedule(const gd_tensor* t, int RB, int KW, int SEG, std::vector<IterDesc>& iters,
                           std::vector<int>& off, std::vector<int>& cnt, Emit emit, BlockScale blockscale)
{
    const int P = t->P, NO = t->n_out, R = t->R;
    const int NOBx = cdiv(NO, RB), KSx = cdiv(P, KW);
    std::vector<std::pair<int, int>> pairs;
    make_pairs(P, pairs);
    int nfrag = 0;
    for (int r = 0; r < R; ++r) {
        off.push_back(int(iters.size()));
        for (int ob = 0; ob < NOBx; ++ob) {
            bool any = false;
            int first_scale = -1;
            for (int delta = 0; delta <= (r + 1 < R ? 1 : 0); ++delta) {
                const int sc = blockscale(r, delta, ob);
                if (first_scale < 0) first_scale = sc;
                // present segments of this (part, ob), in pair order: the K steps from the
                // first to the last nonzero block of p (zero blocks in between are stored)
                struct Seg { int p, lo, hi; };
                std::vector<Seg> segs;
                for (auto& pr : pairs)
                    for (int side = 0; side < 2; ++side) {
                        const int p = side ? pr.second : pr.first;
                        if (p < 0) continue;
                        int lo = -1, hi = -1;
                        for (int ks = p / KW; ks < KSx; ++ks) {
                            bool nz = false;
                            for (int o = ob * RB; o < std::min(NO, ob * RB + RB) && !nz; ++o)
                                for (int q = std::max(p, ks * KW); q < std::min(P, ks * KW + KW); ++q)
                                    if (part(t, r, delta, o, p, q) != 0.0) { nz = true; break; }
                            if (nz) {
                                if (lo < 0) lo = ks;
                                hi = ks;
                            }
                        }
                        // the kernels run every segment to the last K step
                        if (lo >= 0) segs.push_back({p, lo, KSx - 1});
                        (void)hi;
                    }
                for (size_t s0 = 0; s0 < segs.size(); s0 += SEG) {
                    IterDesc d{};
                    d.ob = ob;
                    d.delta = delta;
                    d.scale = sc;
                    d.frag = nfrag;
                    d.nseg = int(std::min<size_t>(SEG, segs.size() - s0));
                    for (int j = 0; j < d.nseg; ++j) {
                        d.p[j] = segs[s0 + j].p;
                        d.lo[j] = segs[s0 + j].lo;
                        d.hi[j] = segs[s0 + j].hi;
                        for (int ks = d.lo[j]; ks <= d.hi[j]; ++ks) {
                            emit(r, delta, ob, d.p[j], ks);
                            ++nfrag;
                        }
                    }
                    d.nfrag = nfrag - d.frag;
                    iters.push_back(d);
                    any = true;
                }
            }
            if (!any) {
                // a row block with no stored fragment still has its (zero) rows written
                IterDesc d{};
                d.ob = ob;
                d.frag = nfrag;
                d.scale = std::max(0, first_scale);
                iters.push_back(d);
            }
        }
        cnt.push_back(int(iters.size()) - off.back());
        IterDesc sentinel{};
        sentinel.ob = -1;
        sentinel.frag = nfrag;
        iters.push_back(sentinel);
        iters.push_back(sentinel);
    }
}

static int pack_tensor(gd_tensor* t)
{
    if (t->packed) return GD_OK;
    const int P = t->P, NO = t->n_out, R = t->R, K1 = t->k + 1;
    t->KS = cdiv(P, 16);
    t->NOB = cdiv(NO, 32);
    t->KS4 = cdiv(P, 4);
    t->NOB16 = cdiv(NO, 16);
    int rc;

    std::vector<double> h(t->N);
    for (int j = 0; j < t->N; ++j) h[j] = t->host.edges[j + 1] - t->host.edges[j];
    if ((rc = upload(t->bufs, h, &t->h, &t->bytes))) return rc;

    // ---------------- scaling of the split path.  U = Tf / (h_l h_m).
    // rowscale_o = 2^ceil(log2 max |U[o]|) over all levels; colscale_q = 2^ceil(log2 of
    // the largest |U[.][.][q]| / rowscale) over all levels.  T is divided by both and the
    // state multiplied by colscale, so that columns whose entries are large (small
    // colliding masses) do not meet the FP16 absolute floor of small state values.
    auto U = [&](int r, int delta, int o, int p, int q) { return part(t, r, delta, o, p, q) / (h[p / K1] * h[q / K1]); };
    std::vector<double> rs(size_t(t->NOB) * 32, 1.0), colmax(P, 0.0);
    for (int o = 0; o < NO; ++o) {
        double mx = 0.0;
        for (int r = 0; r < R; ++r)
            for (int p = 0; p < P; ++p)
                for (int q = p; q < P; ++q) mx = std::max(mx, std::fabs(U(r, 0, o, p, q)));
        if (mx > 0.0) rs[o] = std::ldexp(1.0, pow2_exp(mx));
        for (int r = 0; r < R; ++r)
            for (int p = 0; p < P; ++p)
                for (int q = p; q < P; ++q) colmax[q] = std::max(colmax[q], std::fabs(U(r, 0, o, p, q)) / rs[o]);
    }
    std::vector<double> cs(P, 1.0);
    for (int q = 0; q < P; ++q)
        if (colmax[q] > 0.0) cs[q] = std::ldexp(1.0, pow2_exp(colmax[q]));
    if ((rc = upload(t->bufs, cs, &t->colscale, &t->bytes))) return rc;
    if ((rc = upload(t->bufs, rs, &t->rowscale, &t->bytes))) return rc;
    auto Ut = [&](int r, int delta, int o, int p, int q) { return U(r, delta, o, p, q) / (cs[q] * rs[o]); };

    // ---------------- split-FP16 schedule (32 rows x 16 K per fragment)
    {
        std::vector<IterDesc> iters;
        std::vector<int> off, cnt;
        std::vector<float> scale;
        std::vector<uint16_t> frag;
        std::vector<double> sblk_cur;
        // block scale of (part, ob): the largest |Ut| of every (row block, p) lands in [2^14, 2^15)
        std::vector<double> sblk;   // parallel to scale: the block scale itself
        auto blockscale = [&](int r, int delta, int ob) {
            const int base = int(scale.size());
            for (int p = 0; p < P; ++p) {
                double mx = 0.0;
                for (int o = ob * 32; o < std::min(NO, ob * 32 + 32); ++o)
                    for (int q = p; q < P; ++q) mx = std::max(mx, std::fabs(Ut(r, delta, o, p, q)));
                const double s = (mx > 0.0) ? std::ldexp(1.0, std::max(-1000, pow2_exp(mx) - 15)) : 1.0;
                sblk.push_back(s);
                // stage-2 factor: block scale over the column factor of p
                scale.push_back((float)(s / cs[p]));
            }
            return base;
        };
        auto emit = [&](int r, int delta, int ob, int p, int ks) {
            const double s = sblk[sblk.size() - size_t(P) + p];   // current (part, ob) block
            const size_t f = frag.size() / 1024;
            frag.resize(frag.size() + 1024, 0);
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                    const int o = ob * 32 + (l & 31), q = ks * 16 + 8 * (l >> 5) + j;
                    double v = 0.0;
                    if (o < NO && q < P && q >= p) v = Ut(r, delta, o, p, q) / s;
                    const _Float16 hi = (_Float16)v;
                    const _Float16 lo = (_Float16)(v - (double)hi);
                    uint16_t bh, bl;
                    std::memcpy(&bh, &hi, 2);
                    std::memcpy(&bl, &lo, 2);
                    frag[f * 1024 + l * 8 + j] = bh;
                    frag[f * 1024 + 512 + l * 8 + j] = bl;
                }
        };
        build_schedule(t, 32, 16, segs_per_iter(t->KS), iters, off, cnt, emit, blockscale);
        const uint16_t* dfrag = nullptr;
        if ((rc = upload(t->bufs, frag, &dfrag, &t->bytes))) return rc;
        t->mixed.frag = dfrag;
        t->mixed.frags = (long long)(frag.size() / 1024);
        t->mixed.iters_total = (long long)iters.size();
        if ((rc = upload(t->bufs, iters, &t->mixed.iters, &t->bytes))) return rc;
        if ((rc = upload(t->bufs, off, &t->mixed.iter_off, &t->bytes))) return rc;
        if ((rc = upload(t->bufs, cnt, &t->mixed.iter_cnt, &t->bytes))) return rc;
        if ((rc = upload(t->bufs, scale, &t->mixed.scale, &t->bytes))) return rc;
    }

    // ---------------- FP64 schedule (16 rows x 16 K per fragment as four 4-column steps), T as built
    {
        std::vector<IterDesc> iters;
        std::vector<int> off, cnt;
        std::vector<double> frag;
        auto blockscale = [&](int, int, int) { return 0; };
        auto emit = [&](int r, int delta, int ob, int p, int ks) {
            const size_t f = frag.size() / 256;
            frag.resize(frag.size() + 256, 0.0);
            for (int j = 0; j < 4; ++j)
                for (int l = 0; l < 64; ++l) {
                    const int o = ob * 16 + (l & 15), q = ks * 16 + 4 * j + (l >> 4);
                    if (o < NO && q < P && q >= p) frag[f * 256 + j * 64 + l] = part(t, r, delta, o, p, q);
                }
        };
        build_schedule(t, 16, 16, segs_per_iter(t->KS), iters, off, cnt, emit, blockscale);
        const double* dfrag = nullptr;
        if ((rc = upload(t->bufs, frag, &dfrag, &t->bytes))) return rc;
        t->f64.frag = dfrag;
        t->f64.frags = (long long)(frag.size() / 256);
        t->f64.iters_total = (long long)iters.size();
        if ((rc = upload(t->bufs, iters, &t->f64.iters, &t->bytes))) return rc;
        if ((rc = upload(t->bufs, off, &t->f64.iter_off, &t->bytes))) return rc;
        if ((rc = upload(t->bufs, cnt, &t->f64.iter_cnt, &t->bytes))) return rc;
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
    if (frag->kind != GD_FRAG_NONE && (frag->n_levels < 1 || frag->n_levels > 64 || !frag->levels))
        return fail(GD_EINVAL, "fragmentation needs 1..64 threshold levels");
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

// ============================================================================ plans
struct Group {
    const gd_tensor* t = nullptr;
    int C = 0;
    long long cell0 = 0, val0 = 0;
    int n_slots = 0, tiles32 = 0, tiles16 = 0;
    int* perm = nullptr;        // slot -> cell within the group (nullptr: identity)
    int* slot_level = nullptr;  // [n_slots]
    double* theta = nullptr;    // [n_slots]
    std::vector<int> h_perm;
    uint4* mfrag = nullptr;
    float* mt = nullptr;
    int* eslot = nullptr;
    float* Yf = nullptr;
    double* Yd = nullptr;
    int ystride = 0;
};

struct KernelTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
};

struct gd_plan {
    std::vector<Group> groups;
    int prec = GD_PREC_FP64;
    hipStream_t stream = nullptr;
    long long n_cells = 0, n_values = 0;
    double* y1 = nullptr;
    double* y2 = nullptr;
    unsigned long long* viol = nullptr;
    bool timing = false;
    KernelTimer timer;
    std::vector<void*> allocs;
    ~gd_plan()
    {
        for (auto& e : timer.ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
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

template <class T>
static int dcopy(gd_plan* pl, T** p, const std::vector<T>& v)
{
    int rc = dalloc(pl, p, v.size());
    if (rc) return rc;
    if (!v.empty()) HIP_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return GD_OK;
}

// cells are grouped into threshold brackets of 256 slots so that every contraction
// workgroup reads one level
static constexpr int kSlotGranule = 256;

extern "C" int gd_plan_create(const gd_tensor* const* tensors, const int* cells_per_group, int n_groups,
                              int precision, const double* vfrag, void* stream, gd_plan** out)
{
    if (!tensors || !cells_per_group || n_groups < 1 || !out) return fail(GD_EINVAL, "null argument");
    if (precision != GD_PREC_FP64 && precision != GD_PREC_MIXED_F16X3) return fail(GD_EINVAL, "unknown precision");
    auto pl = std::unique_ptr<gd_plan>(new (std::nothrow) gd_plan());
    if (!pl) return fail(GD_ENOMEM, "host allocation");
    pl->prec = precision;
    pl->stream = (hipStream_t)stream;
    int rc;
    for (int g = 0; g < n_groups; ++g) {
        if (!tensors[g] || cells_per_group[g] < 0) return fail(GD_EINVAL, "bad group");
        if ((rc = pack_tensor(const_cast<gd_tensor*>(tensors[g])))) return rc;
        Group G;
        G.t = tensors[g];
        G.C = cells_per_group[g];
        G.cell0 = pl->n_cells;
        G.val0 = pl->n_values;
        pl->n_cells += G.C;
        pl->n_values += (long long)G.C * G.t->P;
        pl->groups.push_back(std::move(G));
    }
    for (Group& G : pl->groups) {
        const gd_tensor* t = G.t;
        if (t->R > 1) {
            // bracket r and blend weight theta of every cell: levels[r] <= v < levels[r+1],
            // theta = (v - levels[r]) / (levels[r+1] - levels[r]) clamped to [0,1]
            const std::vector<double>& lv = t->spec.levels;
            std::vector<std::vector<std::pair<int, double>>> br(t->R - 1);
            for (int c = 0; c < G.C; ++c) {
                const double v = vfrag ? vfrag[G.cell0 + c] : lv[0];
                int r = 0;
                while (r < t->R - 2 && v >= lv[r + 1]) ++r;
                double th = (v - lv[r]) / (lv[r + 1] - lv[r]);
                th = std::min(1.0, std::max(0.0, th));
                br[r].push_back({c, th});
            }
            std::vector<int> perm, level;
            std::vector<double> theta;
            for (int r = 0; r < t->R - 1; ++r) {
                if (br[r].empty()) continue;
                for (auto& ct : br[r]) {
                    perm.push_back(ct.first);
                    level.push_back(r);
                    theta.push_back(ct.second);
                }
                while (perm.size() % kSlotGranule) {
                    perm.push_back(-1);
                    level.push_back(r);
                    theta.push_back(0.0);
                }
            }
            G.n_slots = int(perm.size());
            G.h_perm = perm;
            if ((rc = dcopy(pl.get(), &G.perm, perm))) return rc;
            if ((rc = dcopy(pl.get(), &G.slot_level, level))) return rc;
            if ((rc = dcopy(pl.get(), &G.theta, theta))) return rc;
        } else {
            G.n_slots = G.C;
        }
        G.tiles32 = cdiv(G.n_slots, 32);
        G.tiles16 = cdiv(G.n_slots, 16);
        if (precision == GD_PREC_MIXED_F16X3) {
            G.ystride = t->NOB * 32;
            if ((rc = dalloc(pl.get(), &G.mfrag, size_t(G.tiles32) * t->KS * 128))) return rc;
            if ((rc = dalloc(pl.get(), &G.mt, size_t(G.tiles32) * 32 * t->P))) return rc;
            if ((rc = dalloc(pl.get(), &G.eslot, size_t(G.n_slots)))) return rc;
            if ((rc = dalloc(pl.get(), &G.Yf, size_t(G.n_slots) * G.ystride))) return rc;
        } else {
            G.ystride = t->NOB16 * 16;
            if ((rc = dalloc(pl.get(), &G.Yd, size_t(G.n_slots) * G.ystride))) return rc;
        }
    }
    if ((rc = dalloc(pl.get(), &pl->y1, pl->n_values))) return rc;
    if ((rc = dalloc(pl.get(), &pl->y2, pl->n_values))) return rc;
    if ((rc = dalloc(pl.get(), &pl->viol, 1))) return rc;
    HIP_TRY(hipMemset(pl->viol, 0, sizeof(unsigned long long)));
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

static StageArgs stage_args(const gd_plan* pl, const Group& G, int mode, int limit, const double* kscale,
                            const double* gn, const double* gs, double* out, double dt, double* raw)
{
    const gd_tensor* t = G.t;
    const bool mixed = pl->prec == GD_PREC_MIXED_F16X3;
    StageArgs a{};
    a.mode = mode;
    a.limit = limit;
    a.split = mixed ? 1 : 0;
    a.Yf = mixed ? G.Yf : nullptr;
    a.Yd = mixed ? nullptr : G.Yd;
    a.rowscale = t->rowscale;
    a.eslot = G.eslot;
    a.perm = G.perm;
    a.kscale = kscale ? kscale + G.cell0 : nullptr;
    a.gn = gn;
    a.gs = gs;
    a.out = out;
    a.raw = raw;
    a.h = t->h;
    a.colscale = t->colscale;
    a.mfrag = G.mfrag;
    a.mt = G.mt;
    a.viol = pl->viol;
    a.dt = dt;
    a.n_slots = G.n_slots;
    a.n_tiles = G.tiles32;
    a.N = t->N;
    a.k = t->k;
    a.P = t->P;
    a.KS = t->KS;
    a.n_out = t->n_out;
    a.ystride = G.ystride;
    a.conservative = t->spec.conservative;
    return a;
}

// the contraction of group G on stage state gs (the split path reads the fragments
// the previous stage kernel wrote from gs)
static int contract_group(gd_plan* pl, Group& G, const double* gs)
{
    const gd_tensor* t = G.t;
    hipStream_t s = pl->stream;
    int rc;
    hipEvent_t ev_end = nullptr;
    if (pl->timing) {
        KernelTimer& T = pl->timer;
        if (T.used == T.ev.size()) {
            hipEvent_t e0, e1;
            HIP_TRY(hipEventCreate(&e0));
            HIP_TRY(hipEventCreate(&e1));
            T.ev.push_back({e0, e1});
        }
        HIP_TRY(hipEventRecord(T.ev[T.used].first, s));
        ev_end = T.ev[T.used].second;
        ++T.used;
    }
    if (pl->prec == GD_PREC_MIXED_F16X3) {
        MixedArgs ma{};
        ma.frag = static_cast<const uint4*>(t->mixed.frag);
        ma.iters = t->mixed.iters;
        ma.iter_off = t->mixed.iter_off;
        ma.iter_cnt = t->mixed.iter_cnt;
        ma.scale = t->mixed.scale;
        ma.slot_level = G.slot_level;
        ma.theta = G.theta;
        ma.mfrag = G.mfrag;
        ma.mt = G.mt;
        ma.Y = G.Yf;
        ma.KS = t->KS;
        ma.n_tiles = G.tiles32;
        ma.n_slots = G.n_slots;
        ma.P = t->P;
        ma.ystride = G.ystride;
        if ((rc = launch_contract_mixed(ma, s))) return rc;
    } else {
        F64Args fa{};
        fa.frag = static_cast<const uint4*>(t->f64.frag);
        fa.iters = t->f64.iters;
        fa.iter_off = t->f64.iter_off;
        fa.iter_cnt = t->f64.iter_cnt;
        fa.slot_level = G.slot_level;
        fa.theta = G.theta;
        fa.perm = G.perm;
        fa.g = gs;
        fa.Y = G.Yd;
        fa.KS = t->KS;
        fa.n_tiles = G.tiles16;
        fa.n_slots = G.n_slots;
        fa.P = t->P;
        fa.ystride = G.ystride;
        if ((rc = launch_contract_fp64(fa, s))) return rc;
    }
    if (ev_end) HIP_TRY(hipEventRecord(ev_end, s));
    return GD_OK;
}

extern "C" int gd_collision_rhs(gd_plan* pl, const double* g, const double* kscale, double* rhs, double* raw)
{
    if (!pl || !g || !rhs) return fail(GD_EINVAL, "null argument");
    long long rawoff = 0;
    int rc;
    for (Group& G : pl->groups) {
        const long long off = rawoff;
        rawoff += (long long)G.C * G.t->n_out;
        if (G.C == 0) continue;
        const double* gs = g + G.val0;
        if (pl->prec == GD_PREC_MIXED_F16X3) {
            // split of the input state (no limiting: the state is read only)
            StageArgs a = stage_args(pl, G, -1, 0, kscale, nullptr, gs, nullptr, 0.0, nullptr);
            if ((rc = launch_stage(a, pl->stream))) return rc;
        }
        if ((rc = contract_group(pl, G, gs))) return rc;
        StageArgs b = stage_args(pl, G, 0, 0, kscale, nullptr, gs, rhs + G.val0, 0.0, raw ? raw + off : nullptr);
        b.split = 0;
        if ((rc = launch_stage(b, pl->stream))) return rc;
    }
    return GD_OK;
}

extern "C" int gd_rk_step(gd_plan* pl, double* g, const double* kscale, double dt, int n_steps,
                          long long* violations)
{
    if (!pl || !g || n_steps < 0) return fail(GD_EINVAL, "bad argument");
    int rc;
    hipStream_t s = pl->stream;
    if ((rc = launch_fill_u64(pl->viol, 1, s))) return rc;
    // limiter on the start state (and its split for the first contraction)
    for (Group& G : pl->groups) {
        if (G.C == 0) continue;
        StageArgs a = stage_args(pl, G, -1, 1, kscale, nullptr, g + G.val0, nullptr, dt, nullptr);
        if ((rc = launch_stage(a, s))) return rc;
    }
    for (int n = 0; n < n_steps; ++n) {
        for (Group& G : pl->groups) {
            if (G.C == 0) continue;
            double* gn = g + G.val0;
            double* y1 = pl->y1 + G.val0;
            double* y2 = pl->y2 + G.val0;
            // y1 = gn + dt L(gn); y2 = 3/4 gn + 1/4 (y1 + dt L(y1)); gn = 1/3 gn + 2/3 (y2 + dt L(y2)),
            // each stage limited (and split for the next contraction) as it is written
            if ((rc = contract_group(pl, G, gn))) return rc;
            if ((rc = launch_stage(stage_args(pl, G, 1, 1, kscale, gn, gn, y1, dt, nullptr), s))) return rc;
            if ((rc = contract_group(pl, G, y1))) return rc;
            if ((rc = launch_stage(stage_args(pl, G, 2, 1, kscale, gn, y1, y2, dt, nullptr), s))) return rc;
            if ((rc = contract_group(pl, G, y2))) return rc;
            if ((rc = launch_stage(stage_args(pl, G, 3, 1, kscale, gn, y2, gn, dt, nullptr), s))) return rc;
        }
    }
    if (violations) {
        unsigned long long v = 0;
        HIP_TRY(hipMemcpyAsync(&v, pl->viol, sizeof(v), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *violations = (long long)v;
    }
    return GD_OK;
}

// ============================================================================ projection
static constexpr int kProjPts = 16;

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
        double Pm = 1.0, Pc = s[a];   // P_{i-2}, P_{i-1}
        for (int i = 0; i < K1; ++i) {
            double Pi;
            if (i == 0) Pi = 1.0;
            else if (i == 1) Pi = s[a];
            else {
                Pi = ((2 * i - 1) * s[a] * Pc - (i - 1) * Pm) / i;
                Pm = Pc;
                Pc = Pi;
            }
            wP[size_t(i) * kProjPts + a] = 0.5 * (2 * i + 1) * w[a] * Pi;
        }
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, wP.size() * sizeof(double)));
    hipStream_t st = (hipStream_t)stream;
    int rc = GD_OK;
    hipError_t e = hipMemcpyAsync(d, wP.data(), wP.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) rc = launch_project(samples, d, coef, n_cells, t->N, t->k, st);
    if (e == hipSuccess && rc == GD_OK) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GD_EHIP, std::string("gd_project: ") + hipGetErrorString(e));
    return rc;
}

// ============================================================================ timing
extern "C" int gd_plan_timing(gd_plan* pl, int enable)
{
    if (!pl) return fail(GD_EINVAL, "null plan");
    pl->timing = enable != 0;
    pl->timer.used = 0;
    return GD_OK;
}

extern "C" int gd_plan_contraction_time(gd_plan* pl, double* total_ms, int* launches)
{
    if (!pl || !total_ms || !launches) return fail(GD_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(pl->stream));
    double tot = 0.0;
    for (size_t i = 0; i < pl->timer.used; ++i) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pl->timer.ev[i].first, pl->timer.ev[i].second));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int)pl->timer.used;
    pl->timer.used = 0;
    return GD_OK;
}

extern "C" int gd_plan_schedule_stats(const gd_plan* pl, int group, long long* frags_mixed, long long* frags_fp64,
                                      int* n_slots)
{
    if (!pl || group < 0 || group >= (int)pl->groups.size()) return fail(GD_EINVAL, "bad group");
    const Group& G = pl->groups[group];
    if (frags_mixed) *frags_mixed = G.t->mixed.frags;
    if (frags_fp64) *frags_fp64 = G.t->f64.frags;
    if (n_slots) *n_slots = G.n_slots;
    return GD_OK;
}
