// String method on the device: the reaction-path workload of the paper's
// replica layer (Section 3.2: images of a path, each image's BO energy and
// force evaluated in parallel, the path updated between force calls), as the
// simplified string method of E, Ren and Vanden-Eijnden (2007):
//   evolution   x_i <- x_i + h F_i for every movable image (F = -dE/dx);
//   reparametrisation: the images redistributed to equal arc length along
//   the piecewise-linear curve through them (cumulative chord lengths s_j,
//   image i to arc length i L / (n - 1) by linear interpolation on the
//   segment s_j <= t < s_{j+1}); the end images keep their positions, a
//   zero-length segment gives weight 0 and a string of zero length stays.
#pragma once
#include <hip/hip_runtime.h>

namespace bscf {

constexpr int kStringMaxImages = 2048;   // arc positions held in LDS

// x [n][ncol] += h * fsign * F [n][ncol] for the movable images (all, or
// without the two ends when fix_ends)
void launch_string_evolve(int n, int ncol, double* x, const double* F, double fsign, double h,
                          int fix_ends, hipStream_t s);
// out = the equal-arc-length redistribution of x (n images of ncol
// coordinates); arc[n] receives the normalised arc positions s_j / L of x
void launch_string_reparam(int n, int ncol, const double* x, double* out, double* arc,
                           hipStream_t s);

}  // namespace bscf
