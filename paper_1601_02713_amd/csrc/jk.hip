// Ket-list-position buffers of the Fock build: the gather of the ket-side
// density block before the class kernels and the fold of the ket-side J block
// into J after them.  Each (position, component) maps to one element of one
// shell-pair block, and every pair occupies one position, so the fold writes
// each J element at most once and needs no atomics.
#include "kernels.h"

namespace bscf {
namespace {

struct PosElem {
  long long idx;   // element offset in the per-instance matrices
  bool ok;
};

__device__ __forceinline__ PosElem pos_elem(const KetPosArgs& a, int e, int pos) {
  const ShellPair pr = a.pairs[a.kets[pos]];
  const Shell sc = a.shells[pr.a], sd = a.shells[pr.b];
  const int nd = ncart(sd.l);
  if (e >= ncart(sc.l) * nd) return {0, false};
  const int k = e / nd, l = e - k * nd;
  const int n = a.nbf[sc.inst];
  return {a.moff[sc.inst] + (long long)(sc.bf + k) * n + sd.bf + l, true};
}

__global__ __launch_bounds__(256) void gather_pk_kernel(KetPosArgs a, int max_ncd,
                                                        const double* __restrict__ P,
                                                        double* __restrict__ Pk) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)max_ncd * a.nk_total) return;
  const int e = (int)(t / a.nk_total), pos = (int)(t - (long long)e * a.nk_total);
  const PosElem x = pos_elem(a, e, pos);
  if (x.ok) Pk[t] = P[x.idx];
}

__global__ __launch_bounds__(256) void jk_finalize_kernel(KetPosArgs a, int max_ncd,
                                                          double* __restrict__ Jk,
                                                          double* __restrict__ J) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)max_ncd * a.nk_total) return;
  const int e = (int)(t / a.nk_total), pos = (int)(t - (long long)e * a.nk_total);
  const PosElem x = pos_elem(a, e, pos);
  if (!x.ok) return;
  J[x.idx] += Jk[t];
  Jk[t] = 0.0;
}

__global__ __launch_bounds__(256) void gather_prims_kernel(int n, const int* __restrict__ map,
                                                           const PrimPair* __restrict__ src,
                                                           PrimPair* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[map[t]];
}

}  // namespace

void launch_gather_prims(int n, const int* map, const PrimPair* src, PrimPair* dst, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(gather_prims_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, map, src, dst);
}

void launch_gather_pk(const KetPosArgs& a, int max_ncd, const double* P, double* Pk,
                      hipStream_t s) {
  const long long n = (long long)max_ncd * a.nk_total;
  if (n == 0) return;
  hipLaunchKernelGGL(gather_pk_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     max_ncd, P, Pk);
}

void launch_jk_finalize(const KetPosArgs& a, int max_ncd, double* Jk, double* J, hipStream_t s) {
  const long long n = (long long)max_ncd * a.nk_total;
  if (n == 0) return;
  hipLaunchKernelGGL(jk_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     max_ncd, Jk, J);
}

}  // namespace bscf
