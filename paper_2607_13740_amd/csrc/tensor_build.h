// Host-side description and FP64 construction of the collision tensor.
#pragma once

#include <vector>

#include "../../include/gracedg.h"

namespace gd {

struct TensorSpec {
    int kernel = GD_KERNEL_CONST;
    double v0 = 1.0;
    double v_bounce = 0.0;
    int frag = GD_FRAG_NONE;
    double alpha = -11.0 / 6.0;
    std::vector<double> levels{1e300};   // fragmentation thresholds (>= 1 entry)
    int bins = 0, order = 0, quad_points = 0;
    double x_min = 0.0, x_max = 0.0;
    int conservative = 0;
};

struct HostTensor {
    int P = 0, n_out = 0, n_levels = 0;
    std::vector<double> edges;   // bins + 1
    std::vector<double> T;       // [level][n_out][P][P], unfolded
};

int n_out_rows(const TensorSpec& sp);
std::vector<double> make_edges(int N, double x_min, double x_max);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void build_tensor(const TensorSpec& sp, HostTensor& out);

} // namespace gd
