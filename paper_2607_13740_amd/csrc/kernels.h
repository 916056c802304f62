// Device-side argument blocks shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

// Split-FP16 contraction (32x32x16 MFMA): rows of T in blocks of 32, K in steps of 16.
struct MixedLevel {
    const uint4* frag;       // fragments (hi 64 lanes x 16 B, then lo) in schedule order
    const int* pair_off;     // [n_pairs + 1] fragment prefix within one row block
    int frags_per_ob;        // fragments per row block
    const float* scale;      // [NOB][P] power-of-two factor of each (row block, p)
    const double* rowscale;  // [NOB*32] power-of-two factor of each row
};

// FP64 contraction (16x16x4 MFMA): rows in blocks of 16, K in steps of 4.
struct F64Level {
    const double* frag;      // fragments (64 lanes x 8 B) in schedule order
    const int* pair_off;     // [n_pairs + 1]
    int frags_per_ob;
};

struct GroupGeom {
    int N, k, P, n_out;
    int conservative;
    int n_pairs;
    const int4* sched;       // [n_pairs] (p_a, ks0_a, p_b, ks0_b); p_b < 0: no second segment
    const double* h;         // [N] bin widths
};

} // namespace gd
