// Ring-polymer integrator kernels (see pimd.h for the scheme and conventions).
//
// The work per step is tiny (two P x P transforms per coordinate column), so
// the kernels are plain: one 64-thread block per column (atom, xyz), thread t
// holding bead t or mode t, the column's vector staged in LDS for the
// transforms.  What matters is that the state never leaves the device between
// steps except for the positions the next force call needs.
#include "pimd.h"

#include <cmath>

namespace bscf {
namespace {

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw 2011): multipliers
// 0xD2511F53 and 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85.
__device__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = (uint64_t)0xD2511F53u * c[0];
    const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)b;
    c[2] = n2;
    c[3] = (uint32_t)a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Standard normal deviate number i of half-step h (Box-Muller on the two
// 53-bit uniforms of one Philox block; even i the cosine, odd i the sine).
__device__ double gaussian(uint64_t seed, uint64_t h, long i) {
  uint32_t c[4] = {(uint32_t)(i >> 1), (uint32_t)h, (uint32_t)(h >> 32), 0x50494d44u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = (double)((((uint64_t)c[0] << 32) | c[1]) >> 11) * 0x1p-53 + 0x1p-54;
  const double u2 = (double)((((uint64_t)c[2] << 32) | c[3]) >> 11) * 0x1p-53 + 0x1p-54;
  const double r = sqrt(-2.0 * log(u1));
  const double t = 2.0 * M_PI * u2;
  return (i & 1) ? r * sin(t) : r * cos(t);
}

__global__ __launch_bounds__(64) void pimd_ob_kernel(PimdArgs a, const double* __restrict__ F,
                                                     double fsign, int thermostat, uint64_t h,
                                                     int order) {
  __shared__ double sv[kPimdMaxBeads];
  const int col = blockIdx.x, t = threadIdx.x, P = a.P;
  const bool on = t < P;
  const long at = (long)t * a.ncol + col;
  double pj = on ? a.p[at] : 0.0;
  const double kick = on ? 0.5 * a.dt * (fsign * F[at]) / P : 0.0;
  if (order == 1) pj += kick;
  if (thermostat) {
    sv[t] = pj;
    __syncthreads();
    double pk = 0.0;
    if (on) {
      for (int j = 0; j < P; ++j) pk += a.C[j * P + t] * sv[j];
      pk = a.c1[t] * pk + a.sig[col / 3] * a.c2[t] * gaussian(a.seed, h, at);
    }
    __syncthreads();
    sv[t] = pk;
    __syncthreads();
    if (on) {
      pj = 0.0;
      for (int k = 0; k < P; ++k) pj += a.C[t * P + k] * sv[k];
    }
  }
  if (order == 0) pj += kick;
  if (on) a.p[at] = pj;
}

__global__ __launch_bounds__(64) void pimd_a_kernel(PimdArgs a) {
  __shared__ double sx[kPimdMaxBeads], sp[kPimdMaxBeads];
  const int col = blockIdx.x, t = threadIdx.x, P = a.P;
  const bool on = t < P;
  const long at = (long)t * a.ncol + col;
  sx[t] = on ? a.x[at] : 0.0;
  sp[t] = on ? a.p[at] : 0.0;
  __syncthreads();
  double q = 0.0, p = 0.0;
  if (on) {
    for (int j = 0; j < P; ++j) {
      q += a.C[j * P + t] * sx[j];
      p += a.C[j * P + t] * sp[j];
    }
    const double m = a.mass[col / 3], w = a.w[t];
    if (t == 0 || w == 0.0) {
      q += a.dt * p / m;
    } else {
      const double c = cos(w * a.dt), s = sin(w * a.dt), mw = m * w;
      const double pn = c * p - mw * s * q;
      q = c * q + s * p / mw;
      p = pn;
    }
  }
  __syncthreads();
  sx[t] = q;
  sp[t] = p;
  __syncthreads();
  if (on) {
    double xj = 0.0, pj = 0.0;
    for (int k = 0; k < P; ++k) {
      xj += a.C[t * P + k] * sx[k];
      pj += a.C[t * P + k] * sp[k];
    }
    a.x[at] = xj;
    a.p[at] = pj;
  }
}

}  // namespace

void launch_pimd_ob(const PimdArgs& a, const double* F, double fsign, int thermostat, uint64_t h,
                    int order, hipStream_t s) {
  hipLaunchKernelGGL(pimd_ob_kernel, dim3(a.ncol), dim3(64), 0, s, a, F, fsign, thermostat, h, order);
}

void launch_pimd_a(const PimdArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(pimd_a_kernel, dim3(a.ncol), dim3(64), 0, s, a);
}

}  // namespace bscf
