// Internal declarations shared by the translation units of libgracedg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/gracedg.h"
#include "tensor_build.h"

namespace gd {

// ------------------------------------------------------------------ errors
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::gd::fail(GD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Pointers read from the group table are generic; the kernels re-type them so that
// read-only tables with uniform indices go through scalar loads (constant address
// space) and the per-lane data through global (not flat) memory instructions.
#if defined(__HIP_DEVICE_COMPILE__)
#define GD_CONST __attribute__((address_space(4)))
#define GD_GLOBAL __attribute__((address_space(1)))
#else
#define GD_CONST
#define GD_GLOBAL
#endif
template <class T>
__device__ __forceinline__ const GD_CONST T* cptr(const T* p)
{
    return (const GD_CONST T*)p;
}
template <class T>
__device__ __forceinline__ GD_GLOBAL T* gptr(T* p)
{
    return (GD_GLOBAL T*)p;
}


// ------------------------------------------------------------------ schedules
// The contraction of one tensor level r and one row block ob is a list of
// iterations.  An iteration carries up to kSegMax p values ("segments") of one part
// (the level itself, or the difference of the next level and this one) whose
// fragments together fit one LDS buffer of frag_budget(KS) fragments of 2 KB (12, or
// KS when a single chain is longer).  Segment s
// covers the K steps lo[s]..KS-1 (16 columns q each) of p[s]: blocks before lo are
// structural zeros, zero blocks after it are stored as zero fragments.  Fragments
// of an iteration are contiguous, segment by segment, K step ascending.  Every list
// is followed by two empty descriptors (nseg = 0) so that the kernels can read the
// descriptors two iterations ahead; a list with no fragment holds one empty
// iteration.
constexpr int kSegMax = 4;
constexpr int kFragBudget = 12;
constexpr int kMaxKS = 13;            // K steps of 16: P = bins * (order + 1) <= 208
constexpr int kMaxP = 16 * kMaxKS;
constexpr int frag_budget(int ks) { return ks > kFragBudget ? ks : kFragBudget; }
struct IterDesc {
    int ob;
    int delta;           // 1: level-difference part, weighted by the cell's blend factor
    int scale;           // offset of (part, ob) in the stage-2 scale table (split path)
    int frag;            // first fragment of the iteration (absolute index)
    int nfrag;
    int nseg;
    int pad0, pad1;
    int p[kSegMax];
    int lo[kSegMax];
    int hi[kSegMax];
    int pad2[kSegMax];
};

// Device layouts of one tensor for one contraction precision.
struct Schedule {
    const void* frag = nullptr;           // 2 KB fragments: split (hi 64 lanes, lo 64 lanes) or FP64 (4 K steps)
    const IterDesc* iters = nullptr;      // all lists, concatenated
    const int* list_off = nullptr;        // [levels * row blocks] first iteration of list (r, ob)
    const int* list_cnt = nullptr;        // [levels * row blocks] iterations of the list
    const float* scale = nullptr;         // split path: stage-2 factors
    std::vector<long long> list_cost;     // host: fragments + iterations of every list
    std::vector<long long> list_frags;    // host: fragments of every list
    std::vector<int> list_n;              // host: iterations of every list (adjoint: 0 = empty list)
    int NOB = 0;                          // row blocks
    long long frags = 0;                  // stored fragments (all levels)
    long long iters_total = 0;
};

// Device-side checks, compiled in with -DGD_CHECKS (the second build of the library,
// libgracedg_checks.so): before using them, the kernels test the work items,
// iteration descriptors, fragment and iteration ranges and slot -> cell indices
// against the sizes in the group descriptor, skip the work on a failure and record
// it as a bit of the plan's check word; the stage kernel also flags non-finite new
// states.  Without the flag the tests compile away.
enum : unsigned { kCheckItem = 1u, kCheckDesc = 2u, kCheckSlot = 4u, kCheckNonFinite = 8u };
#ifdef GD_CHECKS
constexpr bool kChecks = true;
#else
constexpr bool kChecks = false;
#endif

// One group of a plan as the kernels see it: the tensor of the group in the plan's
// precision and the group's slot buffers.  Slots are the cells of the group sorted
// by threshold bracket, each bracket padded to a multiple of 32 slots.
struct GroupDev {
    const uint4* frag;
    const IterDesc* iters;
    const int* list_off;
    const int* list_cnt;
    const float* scale;
    const double* h;           // [N] bin widths
    const double* colscale;    // [P]   split path column factors
    const double* rowscale;    // [NOB*32] split path row factors (by position in Y)
    const int* perm;           // [n_slots] slot -> cell of the group (-1: padding); nullptr: identity
    const double* theta;       // [n_slots] blend weight; nullptr: 0
    uint4* mfrag;              // split path B operands [tiles32][KS][hi|lo][64 lanes]
    float* mt;                 // split path stage-2 weights [tiles32][P][32]
    int* eslot;                // split path per-slot exponent [n_slots]
    float* Yf;                 // split path raw vector [n_slots][ystride], rows bin by bin
    double* Yd;                // FP64 raw vector [n_slots][ystride], rows bin by bin
    long long val0;            // first state value of the group in the plan-wide arrays
    long long raw0;            // first raw-vector value of the group
    int cell0;                 // first cell of the group
    int N, k, P, KS, n_out, NOB, ystride;
    int n_slots, tiles32, tiles16;
    int tile_off;              // first 32-slot tile of the group in the stage launch
    int conservative;
    int R;                     // threshold levels of the tensor
    long long gam0;            // first bin of the group in per-bin arrays (cells * N per group)
    // reverse mode (allocated by the first adjoint call)
    const uint4* afrag;        // FP64 transposed fragments of the vector-Jacobian product
    const IterDesc* aiters;
    const int* alist_off;      // [R * NQB]
    const int* alist_cnt;
    int KSO, NQB, NPS;         // K steps of 16 rows o; blocks of 16 coefficients q; ranges of p
    double* nu;                // [n_slots][KSO*16] cotangent of the raw flux vector
    double* G2;                // [NPS][n_slots][P] second-sum partials (one per p range)
    double* G1p;               // [parts][NQB][n_slots][P] first-sum partials
    double* Dth;               // [NPS][NQB][n_slots] blend-weight partials
    const double* dthdv;       // [n_slots] d theta / d v_frag of the slot's cell
    // sizes the device checks test against (GD_CHECKS), and the word they set
    unsigned* checks;
    long long n_frag;          // 2 KB fragments of the schedule (all levels)
    long long n_iters;         // iteration descriptors of the schedule (with the sentinels)
    int n_cells;               // cells of the group
};

// record a failed device check (any thread; the word is the plan's)
__device__ __forceinline__ void check_fail(unsigned* word, unsigned bit)
{
    if (word) atomicOr(word, bit);
}

// One contraction workgroup: {group, level, ob0 | ob1 << 10 | ntile << 20, first
// tile}.  The workgroup's waves take consecutive tiles (32 slots split path, 16 slots
// FP64), the first ntile of them inside the bracket of the level, and run the lists
// (level, ob0..ob1-1) of the group's tensor.
struct ContractArgs {
    const GroupDev* groups;
    const int4* items;
    const double* g;           // FP64 path: plan-wide stage state (cell order)
    int n_items;
};

// One kernel per RK stage boundary over every group of a plan, one workgroup per
// tile of 32 slots:
//  1. (mode >= 0) fluxes from the raw vector Y, L (Eq. evo) and, for modes 1-3, the
//     SSP-RK3 stage combination (Eq. RK3); mode -1 takes the state gs as it is;
//  2. (limit) the scaling limiter on the new state, written back;
//  3. (split) the per-slot scale and the split FP16 B operands / FP32 weights of the
//     new state for the next contraction.
// State pointers are plan-wide; every group adds its own offsets.
struct StageArgs {
    double* gamma;             // optional limiter factors [bins] (cell order per group)
    const GroupDev* groups;
    int n_groups;
    int tile0, n_tiles;        // the launch covers 32-slot tiles [tile0, tile0 + n_tiles) over all groups
    int max_p;                 // largest P over the groups (sets the LDS size)
    int mode;                  // -1 none, 0: out = L, 1..3: RK stage into out
    int limit, split;
    const double* kscale;      // [cells] or nullptr
    const double* gn;          // RK base state
    const double* gs;          // stage input state
    double* out;               // new state (or L); mode -1 with limit: gs itself
    double* raw;               // optional FP64 raw output [cells][n_out]
    unsigned long long* viol;
    double dt;                 // the step; with adapt set, the largest step dt_max
    // per-cell steps under the CFL bound (adapt = 1): mode 1 sets dtc[cell] =
    // min(dt, t_end - tcell[cell], cfl * bound), modes 2 and 3 read it, mode 3
    // advances tcell; a cell with dtc = 0 keeps its state (cells in caller order over
    // all groups, GroupDev::cell0 + cell)
    int adapt;
    double cfl, t_end, floor;  // floor: outflows <= floor * (largest edge flux) do not bound
    double* tcell;
    double* dtc;
};

// Kernels of the reverse step (see adjoint.hip).
constexpr int kAdjThreads = 256;
constexpr int kAdjSlots = 8;   // slots per workgroup of the per-slot reverse kernels (4 per tile)
constexpr int kAdjPs = 32;     // values of p per list of the vector-Jacobian product
constexpr int kAdjWaves = 4;   // waves per workgroup of the vector-Jacobian product
struct AdjStageArgs {
    const GroupDev* groups;
    int n_groups;
    int n_tiles;               // 32-slot tiles over all groups
    int max_p;                 // largest P over the groups (sets the LDS size)
    int combine;               // add s G of the previous contraction (linearised at ylin) to mu
    const double* ylin;
    const double* mu;          // cotangent of the stage's output (before the combine and the limiter VJP)
    const double* gamma;       // limiter factors of the stage, or nullptr (no limiter)
    const double* ylim;        // limited state of the stage (with gamma)
    double* out;               // if set: the cotangent after the limiter goes here, nothing else
    double* acc;               // acc (=|+=) a lam (or nullptr)
    int acc_add;
    double a;
    double* prev;              // prev (=|+=) b lam (or nullptr)
    int prev_add;
    double b;
    double bdt;                // b dt: nu = A^T (b dt lam)
    const double* kscale;
    double* dkscale;           // combine outputs (+=), [cells] or nullptr
    double* dvfrag;
};

// ------------------------------------------------------------------ tensors
// device buffer owned by a tensor
struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

} // namespace gd

// The library's tensor handle (opaque in the C ABI).
struct gd_tensor {
    gd::TensorSpec spec;
    gd::HostTensor host;
    int N = 0, k = 0, P = 0, n_out = 0, R = 0;
    int KS = 0, NOB = 0;       // split-FP16 path: K steps of 16, row blocks of 32
    int KS4 = 0, NOB16 = 0;    // FP64 path: K steps of 4, row blocks of 16
    long long nnz = 0;
    std::vector<long long> nnz_level, nnz_delta;   // per level r: folded level, level r+1 minus r
    size_t bytes = 0;
    bool packed = false;       // device layouts uploaded (by the first plan)
    std::vector<std::unique_ptr<gd::DevBuf>> bufs;
    const double* h = nullptr;
    const double* colscale = nullptr;   // [P]
    const double* rowscale = nullptr;   // [NOB*32]
    gd::Schedule mixed, f64;
    gd::Schedule adj;              // FP64 transposed layout of the vector-Jacobian product
    // Rows of the forward schedules are ordered bin by bin (V_{0,1..k}, then F_j with
    // V_{j,1..k} for j = 1..N-1, then F_N if non-conservative), so that a row block
    // covers neighbouring masses and its nonzero (p, q) blocks are few: F_j sits at
    // position j(k+1)-1 and V_{j,i} at j(k+1)+i-1 of the raw buffers (the stage kernel
    // reads them there).  rowperm[position] = row o.
    std::vector<int> rowperm;
    bool adj_packed = false;
    int KSO = 0;               // K steps of 16 output rows o (adjoint contraction)
    int NPS = 0;               // ranges of p per q block (adjoint contraction)
};

namespace gd {

// ------------------------------------------------------------------ launchers
int launch_stage(const StageArgs& a, hipStream_t s);
int launch_count_below(const double* t, long long n, double t_end, unsigned long long* count, hipStream_t s);
int launch_fill_u64(unsigned long long* p, int n, hipStream_t s);
int launch_project(const double* samples, const double* wP, double* coef, int C, int N, int k, hipStream_t s);
// ksmax: largest KS of the plan; waves: 4 or 8 per workgroup
int launch_contract_mixed(const ContractArgs& a, int ksmax, int waves, int tpw, hipStream_t s);
int launch_contract_fp64(const ContractArgs& a, int ksmax, int waves, hipStream_t s);
int launch_adjoint_fp64(const ContractArgs& a, int ksomax, hipStream_t s);
int launch_adj_boundary(const AdjStageArgs& a, hipStream_t s);
int launch_fill_f64(double* p, long long n, double v, hipStream_t s);
int launch_advect(const double* g, double* out, const double* courant, long long C, int N, int K1, int periodic,
                  hipStream_t s);

} // namespace gd
