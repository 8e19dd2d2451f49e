// Device Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt, m = 0..L.
//
// T < 40: eight-term Taylor expansion of F_L about the nearest grid point
// T_k = 0.1 k (|T - T_k| <= 0.05) from a table of F_m(T_k), then the stable
// downward recursion F_m = (2T F_{m+1} + exp(-T)) / (2m+1), with exp(-T)
// = exp(-T_k) exp(-(T - T_k)) also from the table.  T >= 40: F_0 =
// sqrt(pi/T)/2 (erf(sqrt T) = 1 to double precision) and the upward recursion
// F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T).  The table is built on the host by
// Gauss-Legendre quadrature of the defining integral.
#pragma once
#include "common.h"

namespace bscf {

// Taylor sum_{j<n} a_j x^j / j! in Horner form, a_j = row[j]
template <int N, typename R>
__device__ __forceinline__ R taylor_row(const R* __restrict__ row, R x) {
  R s = row[N - 1];
#pragma unroll
  for (int j = N - 2; j >= 0; --j) s = fma(s, x * (R(1) / R(j + 1)), row[j]);
  return s;
}

template <int N, typename R>
__device__ __forceinline__ R taylor_exp(R x) {
  R s = R(1);
#pragma unroll
  for (int j = N - 1; j >= 1; --j) s = fma(s, x * (R(1) / R(j)), R(1));
  return s;
}

// F[m] = scale * F_m(T), m = 0..L (FP64)
template <int L>
__device__ __forceinline__ void boys_f64(double T, double scale, const double* __restrict__ tab,
                                         double* F) {
  if (T < kBoysTmax) {
    const int k = __double2int_rn(T * (1.0 / kBoysStep));
    const double d = T - kBoysStep * k;
    const double* row = tab + k * kBoysCols;
    double f = taylor_row<8>(row + L, -d);
    if constexpr (L == 0) {
      F[0] = scale * f;
    } else {
      const double e = row[kBoysExpCol] * taylor_exp<9>(-d);
      F[L] = scale * f;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) {
        f = fma(2.0 * T, f, e) * (1.0 / (2 * m + 1));
        F[m] = scale * f;
      }
    }
  } else {
    const double rt = rsqrt(T);
    double f = 0.886226925452758014 * rt;  // sqrt(pi)/2
    F[0] = scale * f;
    if constexpr (L > 0) {
      const double e = exp(-T);
      const double h = 0.5 * rt * rt;
#pragma unroll
      for (int m = 0; m < L; ++m) {
        f = fma(double(2 * m + 1), f, -e) * h;
        F[m + 1] = scale * f;
      }
    }
  }
}

// FP32 body: five-term Taylor on an FP32 copy of the table; the large-T branch
// and exp(-T) tails stay in FP64 where FP32 would lose relative accuracy.
template <int L>
__device__ __forceinline__ void boys_f32(double T, double scale, const float* __restrict__ tab,
                                         float* F) {
  if (T < kBoysTmax) {
    const int k = __double2int_rn(T * (1.0 / kBoysStep));
    const float d = float(T - kBoysStep * k);
    const float* row = tab + k * kBoysCols;
    float f = taylor_row<5>(row + L, -d);
    const float s = float(scale);
    if constexpr (L == 0) {
      F[0] = s * f;
    } else {
      const float e = row[kBoysExpCol] * taylor_exp<5>(-d);
      const float tt = float(2.0 * T);
      F[L] = s * f;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) {
        f = fmaf(tt, f, e) * (1.0f / (2 * m + 1));
        F[m] = s * f;
      }
    }
  } else {
    const double rt = rsqrt(T);
    double f = 0.886226925452758014 * rt;
    F[0] = float(scale * f);
    if constexpr (L > 0) {
      const double e = exp(-T);
      const double h = 0.5 * rt * rt;
#pragma unroll
      for (int m = 0; m < L; ++m) {
        f = fma(double(2 * m + 1), f, -e) * h;
        F[m + 1] = float(scale * f);
      }
    }
  }
}

}  // namespace bscf
