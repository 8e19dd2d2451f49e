// Ket-list-position buffers of the Fock build: the gather of the ket-side
// density block before the class kernels and the fold of the ket-side J block
// into J after them.  Each (position, component) maps to one element of one
// shell-pair block, and every pair occupies one position, so the fold writes
// each J element at most once and needs no atomics.
#include "kernels.h"

#include <algorithm>

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

// deterministic builds: the same fold in fixed point (Jfx += Jkfx with the
// carry of the low word, then Jkfx cleared)
__global__ __launch_bounds__(256) void jk_finalize_fx_kernel(KetPosArgs a, int max_ncd,
                                                             unsigned long long* __restrict__ Jk,
                                                             unsigned long long* __restrict__ J) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)max_ncd * a.nk_total) return;
  const int e = (int)(t / a.nk_total), pos = (int)(t - (long long)e * a.nk_total);
  const PosElem x = pos_elem(a, e, pos);
  if (!x.ok) return;
  const unsigned long long lo = J[2 * x.idx], add = Jk[2 * t];
  J[2 * x.idx] = lo + add;
  J[2 * x.idx + 1] += Jk[2 * t + 1] + (lo + add < lo ? 1ull : 0ull);
  Jk[2 * t] = 0ull;
  Jk[2 * t + 1] = 0ull;
}

__global__ __launch_bounds__(256) void fx_to_double_kernel(long long n,
                                                           const unsigned long long* __restrict__ fx,
                                                           double* __restrict__ out) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    out[t] = fx_value(fx + 2 * t);
}

__global__ __launch_bounds__(256) void fill_u64_kernel(long long n, unsigned long long* __restrict__ p) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = 0ull;
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

namespace {
// largest |P| of every shell-pair block of every instance
__global__ void shell_pmax_kernel(const int* shell_off, const int* nsh, const long long* pm_off,
                                  const Shell* shells, const long long* moff, const int* nbf,
                                  const double* P, double* Pm) {
  const int inst = blockIdx.y, ns = nsh[inst];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ns * ns) return;
  const int s = e / ns, t = e - s * ns;
  const Shell a = shells[shell_off[inst] + s], b = shells[shell_off[inst] + t];
  const int na = (a.l + 1) * (a.l + 2) / 2, nb = (b.l + 1) * (b.l + 2) / 2, n = nbf[inst];
  const double* M = P + moff[inst];
  double m = 0.0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) m = fmax(m, fabs(M[(long long)(a.bf + i) * n + b.bf + j]));
  Pm[pm_off[inst] + e] = m;
}
}  // namespace

void launch_shell_pmax(int ninst, int max_nsh, const int* shell_off, const int* nsh,
                       const long long* pm_off, const Shell* shells, const long long* moff,
                       const int* nbf, const double* P, double* Pm, hipStream_t s) {
  if (ninst == 0 || max_nsh == 0) return;
  const long long nn = (long long)max_nsh * max_nsh;
  hipLaunchKernelGGL(shell_pmax_kernel, dim3((unsigned)((nn + 255) / 256), ninst), dim3(256), 0, s,
                     shell_off, nsh, pm_off, shells, moff, nbf, P, Pm);
}

void launch_gather_pk(const KetPosArgs& a, int max_ncd, const double* P, double* Pk,
                      hipStream_t s) {
  const long long n = (long long)max_ncd * a.nk_total;
  if (n == 0) return;
  hipLaunchKernelGGL(gather_pk_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     max_ncd, P, Pk);
}

void launch_jk_finalize_fx(const KetPosArgs& a, int max_ncd, unsigned long long* Jk,
                           unsigned long long* J, hipStream_t s) {
  const long long n = (long long)max_ncd * a.nk_total;
  if (n == 0) return;
  hipLaunchKernelGGL(jk_finalize_fx_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     max_ncd, Jk, J);
}

void launch_fx_to_double(long long n, const unsigned long long* fx, double* out, hipStream_t s) {
  if (n == 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fx_to_double_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, fx, out);
}

void launch_fill_u64(long long n, unsigned long long* p, hipStream_t s) {
  if (n == 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, n, p);
}

void launch_jk_finalize(const KetPosArgs& a, int max_ncd, double* Jk, double* J, hipStream_t s) {
  const long long n = (long long)max_ncd * a.nk_total;
  if (n == 0) return;
  hipLaunchKernelGGL(jk_finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                     max_ncd, Jk, J);
}

// Kets of each work row that pass an incremental build's test
// Q_ab Q_cd min(dpmax[inst], 1) >= tau: the row's kets run in descending
// Schwarz bound, so the count is a binary search.  One thread per row, the
// rows of every class in one launch (set.cls[c] owns the blocks from its
// block0 on); rows of instances that are not active are left alone.  When
// keep is given the count goes there; the kept quartets and primitive
// quartets (and, with c32, the kept quartets past the row's FP64 prefix of
// w.pad kets) are added to cq[inst], cpq[inst] (c32[inst]).
__global__ void row_keep_kernel(RowKeepSet set, const int* __restrict__ kets,
                                const ShellPair* __restrict__ pairs,
                                const Shell* __restrict__ shells, const double* __restrict__ Q,
                                const double* __restrict__ dpmax, const int* __restrict__ active,
                                double tau, int ninst) {
  extern __shared__ double part[];   // [3][ninst]
  int ci = 0;
  while (ci + 1 < set.nclass && (int)blockIdx.x >= set.cls[ci + 1].block0) ++ci;
  const RowKeepClass& C = set.cls[ci];
  for (int k = threadIdx.x; k < 3 * ninst; k += blockDim.x) part[k] = 0.0;
  __syncthreads();
  const int r = ((int)blockIdx.x - C.block0) * blockDim.x + threadIdx.x;
  if (r < C.nrows) {
    const WorkRow w = C.rows[r];
    const ShellPair bra = pairs[w.bra];
    const int inst = shells[bra.a].inst;
    if (active[inst]) {
      const double qd = Q[w.bra] * fmin(dpmax[inst], 1.0);
      int lo = 0, hi = w.nket;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (qd * Q[kets[w.ket0 + mid]] >= tau) lo = mid + 1;
        else hi = mid;
      }
      if (C.keep) C.keep[r] = lo;
      if (lo > 0) {
        const int knp = pairs[kets[w.ket0]].nprim;   // one primitive count per row
        atomicAdd(&part[inst], double(lo));
        atomicAdd(&part[ninst + inst], double(lo) * bra.nprim * knp);
        if (C.c32) atomicAdd(&part[2 * ninst + inst], double(max(0, lo - w.pad)));
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ninst; k += blockDim.x) {
    if (part[k] != 0.0) atomicAdd(&C.cq[k], part[k]);
    if (part[ninst + k] != 0.0) atomicAdd(&C.cpq[k], part[ninst + k]);
    if (C.c32 && part[2 * ninst + k] != 0.0) atomicAdd(&C.c32[k], part[2 * ninst + k]);
  }
}

void launch_row_keep(const RowKeepClass* cls, int ncls, const int* kets, const ShellPair* pairs,
                     const Shell* shells, const double* Q, const double* dpmax, const int* active,
                     double tau, int ninst, hipStream_t s) {
  for (int c0 = 0; c0 < ncls; c0 += kRowKeepMaxClasses) {
    RowKeepSet set;
    set.nclass = 0;
    int blocks = 0;
    for (int c = c0; c < std::min(ncls, c0 + kRowKeepMaxClasses); ++c) {
      if (cls[c].nrows <= 0) continue;
      RowKeepClass& d = set.cls[set.nclass++];
      d = cls[c];
      d.block0 = blocks;
      blocks += (cls[c].nrows + 255) / 256;
    }
    if (blocks == 0) continue;
    hipLaunchKernelGGL(row_keep_kernel, dim3(blocks), dim3(256), sizeof(double) * 3 * ninst, s, set,
                       kets, pairs, shells, Q, dpmax, active, tau, ninst);
  }
}

}  // namespace bscf
