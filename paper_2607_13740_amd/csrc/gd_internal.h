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

// ------------------------------------------------------------------ schedules
// One iteration of the contraction: a row block ob and up to kSegMax p values of
// one part (a level, or the difference of two neighbouring levels).  Segment s
// covers the K steps lo[s]..KS-1 (16 columns q each) of p[s] (hi[s] = KS-1); zero
// blocks inside the range are stored as zero fragments, blocks before lo are
// structural zeros.
// Fragments of an iteration are contiguous, segment by segment, K step ascending.
// Every level's list ends with two empty descriptors (nseg = 0, ob = -1) so that the
// kernels can always read the descriptors two iterations ahead.
constexpr int kSegMax = 4;
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
    const IterDesc* iters = nullptr;      // all levels, concatenated
    const int* iter_off = nullptr;        // [levels] first iteration of the level
    const int* iter_cnt = nullptr;        // [levels] iterations of the level
    const float* scale = nullptr;         // mixed: stage-2 factors
    long long frags = 0;                  // stored fragments (all levels)
    long long iters_total = 0;
};

// ------------------------------------------------------------------ kernel arguments
struct MixedArgs {
    const uint4* frag;
    const IterDesc* iters;
    const int* iter_off;
    const int* iter_cnt;
    const float* scale;
    const int* slot_level;     // [n_slots] (nullptr: level 0)
    const double* theta;       // [n_slots] blend weight (nullptr: 0)
    const uint4* mfrag;
    const float* mt;
    float* Y;                  // [n_slots][ystride]
    int KS, n_tiles, n_slots, P, ystride;
};

struct F64Args {
    const uint4* frag;
    const IterDesc* iters;
    const int* iter_off;
    const int* iter_cnt;
    const int* slot_level;
    const double* theta;
    const int* perm;
    const double* g;           // caller state
    double* Y;                 // [n_slots][ystride]
    int KS, n_tiles, n_slots, P, ystride;
};

// One kernel per RK stage boundary, one workgroup per tile of 32 slots:
//  1. (mode >= 0) fluxes from the raw vector Y, L (Eq. evo) and, for modes 1-3, the
//     SSP-RK3 stage combination (Eq. RK3); mode -1 takes the state gs as it is;
//  2. (limit) the scaling limiter on the new state, written back;
//  3. (split) the per-slot scale and the split FP16 B operands / FP32 weights of the
//     new state for the next contraction.
struct StageArgs {
    int mode;                  // -1 none, 0: out = L, 1..3: RK stage into out
    int limit, split;
    const float* Yf;           // split path raw vector (scaled)   or nullptr
    const double* Yd;          // FP64 raw vector                 or nullptr
    const double* rowscale;
    int* eslot;                // per-slot exponent: read for Y, then rewritten by the split
    const int* perm;
    const double* kscale;      // [cells] or nullptr
    const double* gn;          // RK base state (cell order)
    const double* gs;          // stage input state
    double* out;               // new state (or L); mode -1 with limit: gs itself
    double* raw;               // optional FP64 raw output [cells][n_out]
    const double* h;
    const double* colscale;
    uint4* mfrag;
    float* mt;
    unsigned long long* viol;
    double dt;
    int n_slots, n_tiles, N, k, P, KS, n_out, ystride, conservative;
};

// ------------------------------------------------------------------ launchers
int launch_stage(const StageArgs& a, hipStream_t s);
int launch_fill_u64(unsigned long long* p, int n, hipStream_t s);
int launch_project(const double* samples, const double* wP, double* coef, int C, int N, int k, hipStream_t s);
int launch_contract_mixed(const MixedArgs& a, hipStream_t s);
int launch_contract_fp64(const F64Args& a, hipStream_t s);
// p segments per iteration used by the contraction kernels for a given count of
// 16-column K steps; the schedules are built with the same number
int segs_per_iter(int KS);
// cells per contraction workgroup (row blocks of 32: split path; 16: FP64 path)
int slots_per_wg(int rows);

} // namespace gd
