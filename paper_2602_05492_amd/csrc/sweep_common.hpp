// sweep_common.hpp - geometry of the outer boundary and layout constants
// shared by the kernels of the forward, adjoint and normal-equation paths.
#pragma once

#include "common.hpp"

namespace bem {

// Sums kept per handle segment by the adjoint: d/da (2), d/db (2) of the
// cotangent-weighted handle term, and sum_x gbar_c M_m for the four moments
// m = Md_a, Md_b, Ms_a, Ms_b and three channels c (12).
constexpr int kSegVjpVals = 16;

// Element i of the counter-clockwise unit square with m elements per side.
__device__ inline void square_element(int i, int m, double& ax, double& ay, double& bx, double& by)
{
    const int side = i / m, k = i % m;
    const double t0 = (double)k / (double)m, t1 = (double)(k + 1) / (double)m;
    const double cx0 = (side == 1 || side == 2) ? 1.0 : 0.0;
    const double cy0 = (side >= 2) ? 1.0 : 0.0;
    const double dx = side == 0 ? 1.0 : (side == 2 ? -1.0 : 0.0);
    const double dy = side == 1 ? 1.0 : (side == 3 ? -1.0 : 0.0);
    ax = cx0 + t0 * dx; ay = cy0 + t0 * dy;
    bx = cx0 + t1 * dx; by = cy0 + t1 * dy;
}

}  // namespace bem
