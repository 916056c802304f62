// The right-hand side of Eq. evo for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the same kernels as gd_collision_rhs, with every buffer the
// contraction and the stage kernel need beyond the caller's inputs and outputs
// (the group descriptor, the work items, the split B operands and weights, the
// per-slot exponents, the raw flux vector, the violation counter) placed in one
// file-scope device array instead of a plan's allocations.
#include <algorithm>
#include <mutex>

#include "gd_internal.h"

namespace gd {

// 16 MiB per device, held until the process ends.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// device address of this device's copy of the array (looked up once per device,
// with that device current; the array's name is not a device address on the host)
int scratch_base(unsigned char** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GD_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GD_EHIP, "no device address for the static scratch");
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return GD_OK;
}

struct ObOrder {
    int ob[16];   // row blocks, costliest first
};

// Writes the group descriptor and the work items (one per row block and chunk of W
// tiles, row blocks costliest first) into the scratch, and clears the counter.
__global__ void k_noalloc_setup(GroupDev gd, GroupDev* dst, int4* items, int n_items, int ntiles, int W,
                                ObOrder order, unsigned long long* viol)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *dst = gd;
        *viol = 0ull;
    }
    if (i < n_items) {
        const int chunks = (ntiles + W - 1) / W;
        const int ob = order.ob[i / chunks], tile = (i % chunks) * W;
        const int nt = min(W, ntiles - tile);
        items[i] = make_int4(0, 0, ob | ((ob + 1) << 10) | (nt << 20), tile);
    }
}

size_t up256(size_t n) { return (n + 255) & ~size_t(255); }

} // namespace
} // namespace gd

using namespace gd;

extern "C" int gd_collision_rhs_noalloc(const gd_tensor* t, int precision, int n_cells, const double* g,
                                        const double* kscale, double* rhs, double* raw, void* stream)
{
    if (!t || n_cells < 0 || (n_cells > 0 && (!g || !rhs))) return fail(GD_EINVAL, "null argument");
    if (precision != GD_PREC_FP64 && precision != GD_PREC_MIXED_F16X3) return fail(GD_EINVAL, "unknown precision");
    if (!t->packed) return fail(GD_EINVAL, "tensor not on the device yet: call gd_tensor_upload (or create a plan) first");
    if (n_cells == 0) return GD_OK;
    const bool mixed = precision == GD_PREC_MIXED_F16X3;
    const Schedule& S = mixed ? t->mixed : t->f64;
    const int P = t->P, KS = t->KS, NOB = S.NOB;
    const int tiles32 = cdiv(n_cells, 32), tiles16 = cdiv(n_cells, 16);
    const int ystride = mixed ? t->NOB * 32 : t->NOB16 * 16;
    const int W = 8, ntiles = mixed ? tiles32 : tiles16;
    const int n_items = NOB * cdiv(ntiles, W);
    if (NOB > 16) return fail(GD_EUNSUPPORTED, "too many row blocks for the no-allocation path");
    // scratch layout
    size_t off = 0;
    const size_t o_group = off;  off += up256(sizeof(GroupDev));
    const size_t o_viol = off;   off += 256;
    const size_t o_items = off;  off += up256(size_t(n_items) * sizeof(int4));
    size_t o_mfrag = 0, o_mt = 0, o_eslot = 0, o_y = 0;
    if (mixed) {
        o_mfrag = off; off += up256(size_t(tiles32) * KS * 128 * sizeof(uint4));
        o_mt = off;    off += up256(size_t(tiles32) * 32 * P * sizeof(float));
        o_eslot = off; off += up256(size_t(n_cells) * sizeof(int));
        o_y = off;     off += up256(size_t(n_cells) * ystride * sizeof(float));
    } else {
        o_y = off;     off += up256(size_t(n_cells) * ystride * sizeof(double));
    }
    if (off > kScratchBytes)
        return fail(GD_EINVAL, "n_cells too large for the 16 MiB static scratch of the no-allocation path");
    unsigned char* base = nullptr;
    int rc = scratch_base(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;

    GroupDev d{};
    d.frag = static_cast<const uint4*>(S.frag);
    d.iters = S.iters;
    d.list_off = S.list_off;
    d.list_cnt = S.list_cnt;
    d.scale = S.scale;
    d.h = t->h;
    d.colscale = t->colscale;
    d.rowscale = t->rowscale;
    d.perm = nullptr;          // slots are the caller's cells
    d.theta = nullptr;         // level 0 for every cell
    if (mixed) {
        d.mfrag = reinterpret_cast<uint4*>(base + o_mfrag);
        d.mt = reinterpret_cast<float*>(base + o_mt);
        d.eslot = reinterpret_cast<int*>(base + o_eslot);
        d.Yf = reinterpret_cast<float*>(base + o_y);
    } else {
        d.Yd = reinterpret_cast<double*>(base + o_y);
    }
    d.N = t->N;
    d.k = t->k;
    d.P = P;
    d.KS = KS;
    d.n_out = t->n_out;
    d.NOB = NOB;
    d.ystride = ystride;
    d.n_slots = n_cells;
    d.tiles32 = tiles32;
    d.tiles16 = tiles16;
    d.conservative = t->spec.conservative;
    d.R = t->R;
    d.n_frag = S.frags;
    d.n_iters = S.iters_total;
    d.n_cells = n_cells;       // checks: nullptr, the path keeps no check word

    // row blocks of level 0, costliest first
    ObOrder order{};
    {
        int idx[16];
        for (int ob = 0; ob < NOB; ++ob) idx[ob] = ob;
        std::stable_sort(idx, idx + NOB, [&](int a, int b) { return S.list_cost[a] > S.list_cost[b]; });
        for (int i = 0; i < NOB; ++i) order.ob[i] = idx[i];
    }
    GroupDev* gdev = reinterpret_cast<GroupDev*>(base + o_group);
    int4* items = reinterpret_cast<int4*>(base + o_items);
    unsigned long long* viol = reinterpret_cast<unsigned long long*>(base + o_viol);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(cdiv(std::max(1, n_items), 256)), dim3(256), 0, s, d, gdev, items,
                       n_items, ntiles, W, order, viol);
    HIP_TRY(hipGetLastError());

    StageArgs a{};
    a.groups = gdev;
    a.n_groups = 1;
    a.n_tiles = tiles32;
    a.max_p = P;
    a.kscale = kscale;
    a.viol = viol;
    if (mixed) {
        // split of the input state (read only), then the contraction
        a.mode = -1;
        a.split = 1;
        a.gs = g;
        if ((rc = launch_stage(a, s))) return rc;
    }
    ContractArgs c{gdev, items, g, n_items};
    rc = mixed ? launch_contract_mixed(c, KS, W, 1, s) : launch_contract_fp64(c, KS, W, s);
    if (rc) return rc;
    // fluxes -> L (Eq. evo), and the raw vector if asked for
    a.mode = 0;
    a.split = 0;
    a.gs = g;
    a.out = rhs;
    a.raw = raw;
    return launch_stage(a, s);
}
