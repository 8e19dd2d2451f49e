// Dense per-instance kernels of the SCF step: Fock assembly and energy,
// commutator error, Pulay DIIS, convergence flags, density commit, nuclear
// repulsion, and the host-side Boys table.
//
// Fock matrix and energy of closed-shell Hartree-Fock:
//   F = H + J - K/2,  E = Tr[P(H+F)]/2 + E_nuc  (Szabo and Ostlund, 3.4).
// The J and K accumulated by the class kernels are symmetrised here.
// Pulay DIIS (Pulay 1980/1982): B_ij = <e_i, e_j>, minimise |sum c_i e_i| with
// sum c_i = 1, Fbar = sum c_i F_i.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace bscf {

namespace {

__global__ void fill_kernel(double* p, long long n, double v) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <typename T>
__device__ T block_sum(T v, T* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
  __syncthreads();
  return s;  // valid in thread 0
}

// grid: (max_n rows, ninst); writes row partials of Tr[P(H+F)]/2 to rowE
__global__ void fock_assemble_kernel(BatchInfo b, const double* H, const double* J,
                                     const double* K, const double* P, double* F, double* rowE) {
  __shared__ double sh[8];
  const int inst = blockIdx.y, i = blockIdx.x;
  const int n = b.nbf[inst];
  // a converged (masked) instance keeps the F and E of its last build
  if (i >= n || (b.active && !b.active[inst])) return;
  const long long o = b.moff[inst];
  double e = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const long long ij = o + (long long)i * n + j, ji = o + (long long)j * n + i;
    const double f = H[ij] + 0.5 * (J[ij] + J[ji]) - 0.25 * (K[ij] + K[ji]);
    F[ij] = f;
    e += P[ij] * (H[ij] + f);
  }
  e = block_sum(e, sh);
  if (threadIdx.x == 0) rowE[(long long)inst * gridDim.x + i] = 0.5 * e;
}

__global__ void energy_sum_kernel(int ninst, int max_n, const int* nbf, const int* active,
                                  const double* rowE, const double* Enuc, double* E) {
  __shared__ double sh[8];
  const int inst = blockIdx.x;
  if (active && !active[inst]) return;
  const int n = nbf[inst];
  double e = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) e += rowE[(long long)inst * max_n + i];
  e = block_sum(e, sh);
  if (threadIdx.x == 0) E[inst] = e + Enuc[inst];
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), __double_as_longlong(v));
}

// e = A - A^T written to A's antisymmetric copy out; emax over active instances
__global__ void antisym_kernel(BatchInfo b, const double* A, double* out, double* emax) {
  const int inst = blockIdx.y, i = blockIdx.x;
  const int n = b.nbf[inst];
  if (i >= n) return;
  const long long o = b.moff[inst];
  double m = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = A[o + (long long)i * n + j] - A[o + (long long)j * n + i];
    out[o + (long long)i * n + j] = v;
    m = fmax(m, fabs(v));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(&emax[inst], m);
}

// DIIS: copy F, e into the slot head[inst]
__global__ void diis_copy_kernel(DiisArgs d, const double* F, const double* e) {
  const int inst = blockIdx.y;
  if (!d.active[inst]) return;
  const int n = d.nbf[inst];
  const long long o = d.moff[inst], nn = (long long)n * n;
  const int slot = d.head[inst];
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    d.Fhist[slot * d.stride + o + k] = F[o + k];
    d.Ehist[slot * d.stride + o + k] = e[o + k];
  }
}

// B[inst][slot][j] = <e_slot, e_j> for stored j (grid: (max_vec, ninst))
__global__ void diis_dot_kernel(DiisArgs d) {
  __shared__ double sh[8];
  const int inst = blockIdx.y, j = blockIdx.x;
  if (!d.active[inst]) return;
  const int cnt = min(d.count[inst] + 1, d.max_vec);
  const int slot = d.head[inst];
  // stored slots are slot, slot-1, ..., slot-cnt+1 (mod max_vec)
  bool used = false;
  for (int k = 0; k < cnt; ++k)
    if ((slot - k + d.max_vec) % d.max_vec == j) used = true;
  if (!used) return;
  const int n = d.nbf[inst];
  const long long o = d.moff[inst], nn = (long long)n * n;
  double s = 0.0;
  for (long long k = threadIdx.x; k < nn; k += blockDim.x)
    s += d.Ehist[slot * d.stride + o + k] * d.Ehist[j * d.stride + o + k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    double* B = d.B + (long long)inst * d.max_vec * d.max_vec;
    B[slot * d.max_vec + j] = s;
    B[j * d.max_vec + slot] = s;
  }
}

__global__ void diis_advance_kernel(DiisArgs d) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= d.ninst || !d.active[inst]) return;
  d.count[inst] = min(d.count[inst] + 1, d.max_vec);
  d.head[inst] = (d.head[inst] + 1) % d.max_vec;
}

// Solve the DIIS system per instance; drop the oldest vector while the
// elimination meets a pivot below 1e-14 of the largest |B| entry.
__global__ void diis_solve_kernel(DiisArgs d) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= d.ninst || !d.active[inst]) return;
  const int mv = d.max_vec;
  const double* B = d.B + (long long)inst * mv * mv;
  double* c = d.coef + (long long)inst * mv;
  for (int k = 0; k < mv; ++k) c[k] = 0.0;
  const int cnt = d.count[inst];
  const int newest = (d.head[inst] - 1 + mv) % mv;
  int use = cnt;
  while (use >= 2) {
    int slots[8];
    for (int k = 0; k < use; ++k) slots[k] = (newest - k + mv) % mv;
    const int m = use + 1;
    double A[9][10];
    double bmax = 0.0;
    for (int r = 0; r < use; ++r)
      for (int q = 0; q < use; ++q) {
        A[r][q] = B[slots[r] * mv + slots[q]];
        bmax = fmax(bmax, fabs(A[r][q]));
      }
    for (int r = 0; r < use; ++r) {
      A[r][use] = -1.0;
      A[use][r] = -1.0;
      A[r][m] = 0.0;
    }
    A[use][use] = 0.0;
    A[use][m] = -1.0;
    bool ok = true;
    for (int col = 0; col < m && ok; ++col) {
      int piv = col;
      for (int r = col + 1; r < m; ++r)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      const double pv = A[piv][col];
      if (!(fabs(pv) > 1e-14 * fmax(bmax, 1e-300))) { ok = false; break; }
      if (piv != col)
        for (int q = 0; q <= m; ++q) { const double t = A[col][q]; A[col][q] = A[piv][q]; A[piv][q] = t; }
      for (int r = 0; r < m; ++r) {
        if (r == col) continue;
        const double f = A[r][col] / pv;
        for (int q = col; q <= m; ++q) A[r][q] -= f * A[col][q];
      }
    }
    if (ok) {
      for (int k = 0; k < use; ++k) c[slots[k]] = A[k][m] / A[k][k];
      return;
    }
    --use;  // drop the oldest
  }
  c[newest] = 1.0;
}

__global__ void diis_combine_kernel(DiisArgs d, double* Fbar) {
  const int inst = blockIdx.y;
  if (!d.active[inst]) return;
  const int n = d.nbf[inst];
  const long long o = d.moff[inst], nn = (long long)n * n;
  const double* c = d.coef + (long long)inst * d.max_vec;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < d.max_vec; ++j)
      if (c[j] != 0.0) s += c[j] * d.Fhist[j * d.stride + o + k];
    Fbar[o + k] = s;
  }
}

__global__ void convergence_kernel(int ninst, const double* E, double* Eprev, const double* emax,
                                   double etol, double ctol, int iter, int* active,
                                   int* conv_iter, int* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst || !active[i]) return;
  const double e = E[i];
  if (!isfinite(e) || !isfinite(emax[i])) {
    active[i] = 0;
    status[i] |= 2;
    conv_iter[i] = iter + 1;
    return;
  }
  if (iter > 0 && fabs(e - Eprev[i]) < etol && emax[i] < ctol) {
    active[i] = 0;
    status[i] &= ~1;
    conv_iter[i] = iter + 1;
  }
  Eprev[i] = e;
}

__global__ void commit_kernel(BatchInfo b, const double* Pnew, double* P) {
  const int inst = blockIdx.y;
  if (!b.active[inst]) return;
  const int n = b.nbf[inst];
  const long long o = b.moff[inst], nn = (long long)n * n;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x)
    P[o + k] = Pnew[o + k];
}

__global__ void scale_copy_kernel(BatchInfo b, const double* src, double* dst, double alpha,
                                  int transpose) {
  const int inst = blockIdx.y;
  if (b.active && !b.active[inst]) return;
  const int n = b.nbf[inst];
  const long long o = b.moff[inst], nn = (long long)n * n;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nn;
       k += (long long)gridDim.x * blockDim.x) {
    const long long i = k / n, j = k % n;
    dst[o + k] = alpha * (transpose ? src[o + j * n + i] : src[o + k]);
  }
}

__global__ void nuclear_kernel(int ninst, const int* natoms, const int* atom_off,
                               const double* xyz, const double* Z, double* Enuc, double* grad,
                               int want_grad) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= ninst) return;
  const int n = natoms[inst], o = atom_off[inst];
  double e = 0.0;
  for (int i = 0; i < n; ++i) {
    double g[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = xyz[3 * (o + i)] - xyz[3 * (o + j)];
      const double dy = xyz[3 * (o + i) + 1] - xyz[3 * (o + j) + 1];
      const double dz = xyz[3 * (o + i) + 2] - xyz[3 * (o + j) + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double r = sqrt(r2);
      const double zz = Z[o + i] * Z[o + j];
      if (j < i) e += zz / r;
      const double f = zz / (r2 * r);
      g[0] -= f * dx;
      g[1] -= f * dy;
      g[2] -= f * dz;
    }
    if (want_grad)
      for (int d = 0; d < 3; ++d) grad[3 * (o + i) + d] += g[d];
  }
  Enuc[inst] = e;
}

}  // namespace

void launch_fill(double* p, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// rowE scratch lives after the energies: caller passes E with room for
// ninst + ninst*max_n doubles (first ninst are the energies).
void launch_fock_assemble(const BatchInfo& b, int max_n, const double* H, const double* J,
                          const double* K, const double* P, const double* Enuc, double* F,
                          double* E, hipStream_t s) {
  double* rowE = E + b.ninst;
  hipLaunchKernelGGL(fock_assemble_kernel, dim3(max_n, b.ninst), dim3(256), 0, s, b, H, J, K, P,
                     F, rowE);
  hipLaunchKernelGGL(energy_sum_kernel, dim3(b.ninst), dim3(256), 0, s, b.ninst, max_n, b.nbf,
                     b.active, rowE, Enuc, E);
}

void launch_antisym(const BatchInfo& b, int max_n, const double* A, double* out, double* emax,
                    hipStream_t s) {
  launch_fill(emax, b.ninst, 0.0, s);
  hipLaunchKernelGGL(antisym_kernel, dim3(max_n, b.ninst), dim3(256), 0, s, b, A, out, emax);
}

void launch_diis_store(const DiisArgs& d, int max_n, const double* F, const double* e,
                       hipStream_t s) {
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(diis_copy_kernel, dim3(gx, d.ninst), dim3(256), 0, s, d, F, e);
  hipLaunchKernelGGL(diis_dot_kernel, dim3(d.max_vec, d.ninst), dim3(256), 0, s, d);
  hipLaunchKernelGGL(diis_advance_kernel, dim3((d.ninst + 63) / 64), dim3(64), 0, s, d);
}

void launch_diis_extrapolate(const DiisArgs& d, int max_n, double* Fbar, hipStream_t s) {
  hipLaunchKernelGGL(diis_solve_kernel, dim3((d.ninst + 63) / 64), dim3(64), 0, s, d);
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(diis_combine_kernel, dim3(gx, d.ninst), dim3(256), 0, s, d, Fbar);
}

void launch_convergence(int ninst, const double* E, double* Eprev, const double* emax,
                        double etol, double ctol, int iter, int* active, int* conv_iter,
                        int* status, hipStream_t s) {
  hipLaunchKernelGGL(convergence_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, E,
                     Eprev, emax, etol, ctol, iter, active, conv_iter, status);
}

void launch_commit(const BatchInfo& b, int max_n, const double* Pnew, double* P, hipStream_t s) {
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(commit_kernel, dim3(gx, b.ninst), dim3(256), 0, s, b, Pnew, P);
}

void launch_scale_copy(const BatchInfo& b, int max_n, const double* src, double* dst,
                       double alpha, int transpose, hipStream_t s) {
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(scale_copy_kernel, dim3(gx, b.ninst), dim3(256), 0, s, b, src, dst, alpha,
                     transpose);
}

void launch_nuclear(int ninst, const int* natoms, const int* atom_off, const double* xyz,
                    const double* Z, double* Enuc, double* grad, int want_grad, hipStream_t s) {
  hipLaunchKernelGGL(nuclear_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, natoms,
                     atom_off, xyz, Z, Enuc, grad, want_grad);
}

// ---------------------------------------------------------------------------
// Host Boys table: F_m(T_k) = int_0^1 t^{2m} exp(-T_k t^2) dt by 160-point
// Gauss-Legendre quadrature on [0, 1] in long double; column 23 = exp(-T_k).
namespace {
void gauss_legendre(int n, long double* x, long double* w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-20L) break;
    }
    x[i] = z;
    w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}
}  // namespace

void boys_table_host(double* tab) {
  constexpr int NG = 160;
  static long double x[NG], w[NG];
  static bool init = false;
  if (!init) {
    gauss_legendre(NG, x, w);
    init = true;
  }
  for (int k = 0; k < kBoysRows; ++k) {
    const long double T = kBoysStep * k;
    for (int m = 0; m < kBoysExpCol; ++m) {
      long double s = 0.0L;
      for (int i = 0; i < NG; ++i) {
        const long double t = 0.5L * (x[i] + 1.0L);
        s += 0.5L * w[i] * powl(t, 2 * m) * expl(-T * t * t);
      }
      tab[k * kBoysCols + m] = (double)s;
    }
    tab[k * kBoysCols + kBoysExpCol] = (double)expl(-T);
  }
}

}  // namespace bscf
