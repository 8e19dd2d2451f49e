// String-method kernels (see string_method.h).  The path is small (images x
// 3N coordinates), so the reparametrisation is one workgroup: the segment
// lengths by block reductions, their prefix sums in LDS, then every
// (image, coordinate) interpolated in parallel.
#include "string_method.h"

#include <algorithm>

namespace bscf {
namespace {

__global__ void string_evolve_kernel(int n, int ncol, double* __restrict__ x,
                                     const double* __restrict__ F, double fsign, double h,
                                     int fix_ends) {
  const long total = (long)n * ncol;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total;
       k += (long)gridDim.x * blockDim.x) {
    const int i = (int)(k / ncol);
    if (fix_ends && (i == 0 || i == n - 1)) continue;
    x[k] += h * (fsign * F[k]);
  }
}

__global__ __launch_bounds__(256) void string_reparam_kernel(int n, int ncol,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ out,
                                                             double* __restrict__ arc) {
  __shared__ double s[kStringMaxImages];
  __shared__ double red[256];
  const int t = threadIdx.x;
  if (t == 0) s[0] = 0.0;
  // chord length of every segment, one block reduction each
  for (int j = 0; j + 1 < n; ++j) {
    double acc = 0.0;
    for (int c = t; c < ncol; c += 256) {
      const double d = x[(long)(j + 1) * ncol + c] - x[(long)j * ncol + c];
      acc += d * d;
    }
    red[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) s[j + 1] = sqrt(red[0]);
    __syncthreads();
  }
  if (t == 0)
    for (int j = 1; j < n; ++j) s[j] += s[j - 1];   // cumulative arc length
  __syncthreads();
  const double L = s[n - 1];
  for (int j = t; j < n; j += 256) arc[j] = L > 0.0 ? s[j] / L : 0.0;
  const long total = (long)n * ncol;
  for (long k = t; k < total; k += 256) {
    const int i = (int)(k / ncol), c = (int)(k - (long)i * ncol);
    if (n < 3 || L == 0.0 || i == 0 || i == n - 1) {
      out[k] = x[k];
      continue;
    }
    const double tt = i * L / (n - 1);
    // the segment with s_j <= tt < s_{j+1} (the last one at most)
    int lo = 0, hi = n - 2;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (s[mid + 1] <= tt) lo = mid + 1;
      else hi = mid;
    }
    const double d = s[lo + 1] - s[lo];
    const double w = d > 0.0 ? (tt - s[lo]) / d : 0.0;
    out[k] = (1.0 - w) * x[(long)lo * ncol + c] + w * x[(long)(lo + 1) * ncol + c];
  }
}

}  // namespace

void launch_string_evolve(int n, int ncol, double* x, const double* F, double fsign, double h,
                          int fix_ends, hipStream_t s) {
  const long total = (long)n * ncol;
  const int blocks = (int)std::min<long>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(string_evolve_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, ncol,
                     x, F, fsign, h, fix_ends);
}

void launch_string_reparam(int n, int ncol, const double* x, double* out, double* arc,
                           hipStream_t s) {
  hipLaunchKernelGGL(string_reparam_kernel, dim3(1), dim3(256), 0, s, n, ncol, x, out, arc);
}

}  // namespace bscf
