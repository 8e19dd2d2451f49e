// Dense per-instance kernels of the SCF step: Fock assembly and energy,
// commutator error, Pulay DIIS, convergence flags, density commit, nuclear
// repulsion, and the host-side Boys table.
//
// Fock matrix and energy of closed-shell Hartree-Fock:
//   F = H + J - K/2,  E = Tr[P(H+F)]/2 + E_nuc  (Szabo and Ostlund, 3.4).
// The J and K accumulated by the class kernels are symmetrised here.
// Pulay DIIS (Pulay 1980/1982): B_ij = <e_i, e_j>, minimise |sum c_i e_i| with
// sum c_i = 1, Fbar = sum c_i F_i.
// Density from the orthonormal-basis Fock matrix F' by second-order spectral
// projection (SP2, the trace-correcting purification of Niklasson, Phys. Rev.
// B 66, 155115 (2002)): X_0 = (hi I - F') / (hi - lo) over Gershgorin bounds
// [lo, hi] maps the spectrum into [0, 1] with the lowest levels of F' on top;
// each step replaces X by X^2 or 2X - X^2, whichever brings Tr of the result
// closer to the number of occupied orbitals, which drives the occupied levels
// to 1 and the rest to 0 while keeping their order, so X converges to the
// projector on the occupied subspace that diagonalisation with aufbau
// occupation gives.
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
// F = H + J - (kx / 2) K (+ Vxc), symmetrised; row sums of the energy
// Tr[P (H + F')] / 2 with F' = F without Vxc, plus Exc on row 0 (kx = 1 and
// no Vxc: Hartree-Fock; kx = exact-exchange share with Vxc, Exc: hybrid DFT)
__global__ void fock_assemble_kernel(BatchInfo b, const double* H, const double* J,
                                     const double* K, const double* P, double* F, double* rowE,
                                     double kx, const double* Vxc, const double* Exc) {
  __shared__ double sh[8];
  const int inst = blockIdx.y, i = blockIdx.x;
  const int n = b.nbf[inst];
  // a converged (masked) instance keeps the F and E of its last build
  if (i >= n || (b.active && !b.active[inst])) return;
  const long long o = b.moff[inst];
  double e = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const long long ij = o + (long long)i * n + j, ji = o + (long long)j * n + i;
    const double f = H[ij] + 0.5 * (J[ij] + J[ji]) - 0.25 * kx * (K[ij] + K[ji]);
    F[ij] = Vxc ? f + Vxc[ij] : f;
    e += P[ij] * (H[ij] + f);
  }
  e = block_sum(e, sh);
  if (threadIdx.x == 0)
    rowE[(long long)inst * gridDim.x + i] = 0.5 * e + ((Exc && i == 0) ? Exc[inst] : 0.0);
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

constexpr int kTile = 32;
__host__ __device__ inline int ntiles_1d(int n) { return (n + kTile - 1) / kTile; }

// max that keeps a NaN (so a diverged replica is caught by the finiteness test)
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? NAN : fmax(a, b);
}

// out = A - A^T by 32 x 32 tiles staged in LDS (both reads coalesced); the
// largest |out| of each tile goes to tmax[inst][bi][bj] (tile grid of max_n)
__global__ void antisym_kernel(BatchInfo b, int max_n, const double* A, double* out,
                               double* tmax) {
  __shared__ double t1[kTile][kTile + 1], t2[kTile][kTile + 1];
  __shared__ double wm[4];
  const int inst = blockIdx.z;
  const int n = b.nbf[inst];
  const int nt = ntiles_1d(n), ntm = ntiles_1d(max_n);
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi >= nt || bj >= nt) return;
  const long long o = b.moff[inst];
  const int i0 = bi * kTile, j0 = bj * kTile, c = threadIdx.x;
  for (int r = threadIdx.y; r < kTile; r += blockDim.y) {
    t1[r][c] = (i0 + r < n && j0 + c < n) ? A[o + (long long)(i0 + r) * n + j0 + c] : 0.0;
    t2[r][c] = (j0 + r < n && i0 + c < n) ? A[o + (long long)(j0 + r) * n + i0 + c] : 0.0;
  }
  __syncthreads();
  double m = 0.0;
  for (int r = threadIdx.y; r < kTile; r += blockDim.y)
    if (i0 + r < n && j0 + c < n) {
      const double v = t1[r][c] - t2[c][r];   // A[i][j] - A[j][i]
      out[o + (long long)(i0 + r) * n + j0 + c] = v;
      m = nan_max(m, fabs(v));
    }
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  const int tid = threadIdx.y * kTile + threadIdx.x;
  if ((tid & 63) == 0) wm[tid >> 6] = m;
  __syncthreads();
  if (tid == 0)
    tmax[((long long)inst * ntm + bi) * ntm + bj] = nan_max(nan_max(wm[0], wm[1]), nan_max(wm[2], wm[3]));
}

// dP = P - Pprev per 32 x 32 tile, and the largest |dP| of each tile to
// tmax[inst][bi][bj] (tile grid of max_n), for the instances of b
__global__ void dp_kernel(BatchInfo b, int max_n, const double* P, const double* Pprev,
                          double* dP, double* tmax) {
  __shared__ double wm[4];
  const int inst = blockIdx.z;
  if (b.active && !b.active[inst]) return;
  const int n = b.nbf[inst];
  const int nt = ntiles_1d(n), ntm = ntiles_1d(max_n);
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi >= nt || bj >= nt) return;
  const long long o = b.moff[inst];
  double m = 0.0;
  for (int r = threadIdx.y; r < kTile; r += blockDim.y) {
    const int i = bi * kTile + r, j = bj * kTile + threadIdx.x;
    if (i < n && j < n) {
      const long long e = o + (long long)i * n + j;
      const double d = P[e] - Pprev[e];
      dP[e] = d;
      m = nan_max(m, fabs(d));
    }
  }
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  const int tid = threadIdx.y * kTile + threadIdx.x;
  if ((tid & 63) == 0) wm[tid >> 6] = m;
  __syncthreads();
  if (tid == 0)
    tmax[((long long)inst * ntm + bi) * ntm + bj] = nan_max(nan_max(wm[0], wm[1]), nan_max(wm[2], wm[3]));
}

// out[i] = the largest of instance i's tile maxima (one wavefront per instance)
__global__ __launch_bounds__(64) void tile_max_kernel(BatchInfo b, int max_n, const double* tmax,
                                                      double* out) {
  const int i = blockIdx.x;
  if (b.active && !b.active[i]) return;
  const int nt = ntiles_1d(b.nbf[i]), ntm = ntiles_1d(max_n);
  double m = 0.0;
  for (int t = threadIdx.x; t < nt * nt; t += 64)
    m = nan_max(m, tmax[((long long)i * ntm + t / nt) * ntm + t % nt]);
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
  if (threadIdx.x == 0) out[i] = m;
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
  // the slot's row and column of B are summed afresh by diis_dot_kernel
  if (blockIdx.x == 0 && threadIdx.x < d.max_vec) {
    double* B = d.B + (long long)inst * d.max_vec * d.max_vec;
    B[slot * d.max_vec + threadIdx.x] = 0.0;
    B[threadIdx.x * d.max_vec + slot] = 0.0;
  }
}

// B[inst][slot][j] = <e_slot, e_j> for stored j; grid (max_vec, ninst,
// kDotSplit): each block sums one slice of the elements into B (zeroed by
// diis_copy_kernel)
constexpr int kDotSplit = 8;
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
  const long long per = (nn + kDotSplit - 1) / kDotSplit;
  const long long k0 = blockIdx.z * per, k1 = min(nn, k0 + per);
  double s = 0.0;
  for (long long k = k0 + threadIdx.x; k < k1; k += blockDim.x)
    s += d.Ehist[slot * d.stride + o + k] * d.Ehist[j * d.stride + o + k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    double* B = d.B + (long long)inst * d.max_vec * d.max_vec;
    atomicAdd(&B[slot * d.max_vec + j], s);
    if (j != slot) atomicAdd(&B[j * d.max_vec + slot], s);
  }
}

__global__ void diis_advance_kernel(DiisArgs d) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= d.ninst || !d.active[inst]) return;
  d.count[inst] = min(d.count[inst] + 1, d.max_vec);
  d.head[inst] = (d.head[inst] + 1) % d.max_vec;
}

// Solve the DIIS system per instance; drop the oldest vector while the
// elimination meets a pivot below 1e-14 of the largest |B| entry.  One
// wavefront per instance: lane r holds row r of the bordered system
//   [B  -1] [c     ]   [ 0]
//   [-1  0] [lambda] = [-1]
// in registers (columns 0..8, right-hand side in column 9); Gauss-Jordan
// elimination with partial pivoting, rows exchanged by lane shuffles.
__global__ __launch_bounds__(64) void diis_solve_kernel(DiisArgs d) {
  constexpr int kMaxM = 9;   // max_vec + 1
  const int inst = blockIdx.x;
  if (!d.active[inst]) return;
  const int lane = threadIdx.x;
  const int mv = d.max_vec;
  const double* B = d.B + (long long)inst * mv * mv;
  double* cf = d.coef + (long long)inst * mv;
  const int cnt = d.count[inst];
  const int newest = (d.head[inst] - 1 + mv) % mv;
  for (int use = cnt; use >= 2; --use) {
    const int m = use + 1;
    double a[kMaxM + 1];
    double bmax = 0.0;
    const int sr = lane < mv ? (newest - lane + mv) % mv : 0;   // slot of this lane's row
#pragma unroll
    for (int q = 0; q <= kMaxM; ++q) a[q] = 0.0;
    if (lane < use) {
#pragma unroll
      for (int q = 0; q < kMaxM; ++q)
        if (q < use) {
          a[q] = B[sr * mv + (newest - q + mv) % mv];
          bmax = fmax(bmax, fabs(a[q]));
        }
#pragma unroll
      for (int q = 0; q < kMaxM; ++q)
        if (q == use) a[q] = -1.0;
    } else if (lane == use) {
#pragma unroll
      for (int q = 0; q < kMaxM; ++q)
        if (q < use) a[q] = -1.0;
      a[kMaxM] = -1.0;
    }
    for (int off = 32; off > 0; off >>= 1) bmax = fmax(bmax, __shfl_xor(bmax, off, 64));
    bool ok = true;
#pragma unroll
    for (int col = 0; col < kMaxM; ++col) {
      if (col >= m || !ok) continue;
      // pivot: the first row in [col, m) of largest |a[col]|
      const bool cand = lane >= col && lane < m;
      double v = cand ? fabs(a[col]) : -1.0;
      double vmax = v;
      for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off, 64));
      const unsigned long long hit = __ballot(cand && v == vmax);
      const int piv = __ffsll((long long)hit) - 1;
      const double pv = __shfl(a[col], piv, 64);
      if (!(fabs(pv) > 1e-14 * fmax(bmax, 1e-300))) { ok = false; continue; }
      const int partner = lane == col ? piv : (lane == piv ? col : lane);
#pragma unroll
      for (int q = 0; q <= kMaxM; ++q) a[q] = __shfl(a[q], partner, 64);
      double prow[kMaxM + 1];
#pragma unroll
      for (int q = 0; q <= kMaxM; ++q) prow[q] = __shfl(a[q], col, 64);
      if (lane != col && lane < m) {
        const double f = a[col] / pv;
#pragma unroll
        for (int q = 0; q <= kMaxM; ++q)
          if (q >= col) a[q] -= f * prow[q];
      }
    }
    if (ok) {
      double dg = 1.0;
#pragma unroll
      for (int q = 0; q < kMaxM; ++q)
        if (q == lane) dg = a[q];
      const double mine = a[kMaxM] / dg;   // coefficient of row lane's slot
      const int k = lane < mv ? (newest - lane + mv) % mv : 0;   // row holding slot `lane`
      const double v = __shfl(mine, k, 64);
      if (lane < mv) cf[lane] = k < use ? v : 0.0;
      return;
    }
  }
  if (lane < mv) cf[lane] = lane == newest ? 1.0 : 0.0;
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

// niter[i] counts the iterations instance i has taken (it stops when the
// instance leaves the active set, so it ends as the iteration count).
__global__ __launch_bounds__(64) void convergence_kernel(int ninst, int max_n, const int* nbf,
                                                        const double* E, double* Eprev,
                                                        const double* tmax, double* emax,
                                                        double etol, double ctol, int* active,
                                                        int* niter, int* status) {
  const int i = blockIdx.x;
  if (!active[i]) return;
  const int nt = ntiles_1d(nbf[i]), ntm = ntiles_1d(max_n);
  double em = 0.0;
  for (int t = threadIdx.x; t < nt * nt; t += 64)
    em = nan_max(em, tmax[((long long)i * ntm + t / nt) * ntm + t % nt]);
  for (int off = 32; off > 0; off >>= 1) em = nan_max(em, __shfl_xor(em, off, 64));
  if (threadIdx.x != 0) return;
  emax[i] = em;
  const int iter = niter[i];
  niter[i] = iter + 1;
  const double e = E[i];
  if (!isfinite(e) || !isfinite(em)) {
    active[i] = 0;
    status[i] |= 2;
    return;
  }
  if (iter > 0 && fabs(e - Eprev[i]) < etol && em < ctol) {
    active[i] = 0;
    status[i] &= ~1;
  }
  Eprev[i] = e;
}

// out[0, na) = a, out[na, na + nb) = b
__global__ void concat_ints_kernel(const int* a, int na, const int* b, int nb, int* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < na) out[t] = a[t];
  else if (t < na + nb) out[t] = b[t - na];
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

// Gershgorin intervals of the rows of each instance's symmetric F': one
// wavefront per row (read as its column, contiguous), rowb[inst][r] = (lo, hi)
__global__ void sp2_bounds_kernel(BatchInfo b, int max_n, const double* F, double* rowb) {
  const int inst = blockIdx.y;
  if (b.active && !b.active[inst]) return;
  const int n = b.nbf[inst];
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= n) return;   // whole wavefront; no barrier follows
  const long long o = b.moff[inst];
  double off = 0.0;
  for (int j = lane; j < n; j += 64)
    if (j != r) off += fabs(F[o + (long long)r * n + j]);
  for (int k = 32; k > 0; k >>= 1) off += __shfl_xor(off, k, 64);
  if (lane == 0) {
    const double d = F[o + (long long)r * n + r];
    rowb[((long long)inst * max_n + r) * 2] = d - off;
    rowb[((long long)inst * max_n + r) * 2 + 1] = d + off;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Per-instance tile grids launched one-dimensional over xcd_grid(ninst, T)
// blocks: block L runs on XCD L % kXcds, and instance i's T tiles all take
// blocks on XCD i % kXcds, so they share that XCD's L2.  False for the
// padding blocks past the last instance.
__device__ inline bool xcd_tile(int ninst, int T, int& inst, int& tile) {
  const int L = blockIdx.x, x = L % kXcds, j = L / kXcds;
  inst = x + kXcds * (j / T);
  tile = j % T;
  return inst < ninst;
}
inline unsigned xcd_grid(int ninst, int T) {
  return (unsigned)(kXcds * ((ninst + kXcds - 1) / kXcds) * T);
}

// sum of the per-tile partial (Tr, Tr^2) rows of one instance (a block-wide
// call; the result is valid in every thread)
__device__ void sp2_stats(const double* st, int nt2, double& tr, double& t2, double* sh) {
  double a = 0.0, q = 0.0;
  for (int t = threadIdx.x; t < nt2; t += blockDim.x) {
    a += st[2 * t];
    q += st[2 * t + 1];
  }
  for (int k = 32; k > 0; k >>= 1) {
    a += __shfl_xor(a, k, 64);
    q += __shfl_xor(q, k, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[2 * (threadIdx.x >> 6)] = a;
    sh[2 * (threadIdx.x >> 6) + 1] = q;
  }
  __syncthreads();
  tr = t2 = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    tr += sh[2 * w];
    t2 += sh[2 * w + 1];
  }
  __syncthreads();
}

// block-wide sum of (a, q) into st[0], st[1] by thread 0
__device__ void sp2_store_stats(double a, double q, double* st, double* sh) {
  for (int k = 32; k > 0; k >>= 1) {
    a += __shfl_xor(a, k, 64);
    q += __shfl_xor(q, k, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[2 * (threadIdx.x >> 6)] = a;
    sh[2 * (threadIdx.x >> 6) + 1] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tq = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ta += sh[2 * w];
      tq += sh[2 * w + 1];
    }
    st[0] = ta;
    st[1] = tq;
  }
}

// X_0 = (hi I - (F' + F'^T)/2) / (hi - lo) over the union of the rows'
// Gershgorin intervals; the symmetrised start keeps every later X exactly
// symmetric.  One block per (instance, 32 x 32 tile), placed by xcd_tile; each tile stores its
// (Tr, Tr^2) partial at st[inst][tile]; conv[inst] = -1 (not converged).
__global__ __launch_bounds__(256) void sp2_init_kernel(BatchInfo b, int max_n, const double* F,
                                                       const double* rowb, double* X, double* st,
                                                       int* conv) {
  __shared__ double sh[8];
  const int ntm = ntiles_1d(max_n);
  int inst, tile;
  if (!xcd_tile(b.ninst, ntm * ntm, inst, tile)) return;
  if (b.active && !b.active[inst]) return;
  const int n = b.nbf[inst], nt = ntiles_1d(n);
  if (tile >= nt * nt) return;
  if (tile == 0 && threadIdx.x == 0) conv[inst] = -1;
  const long long o = b.moff[inst];
  double lo = INFINITY, hi = -INFINITY;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    lo = fmin(lo, rowb[((long long)inst * max_n + r) * 2]);
    hi = fmax(hi, rowb[((long long)inst * max_n + r) * 2 + 1]);
  }
  for (int k = 32; k > 0; k >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, k, 64));
    hi = fmax(hi, __shfl_xor(hi, k, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sh[2 * (threadIdx.x >> 6)] = lo;
    sh[2 * (threadIdx.x >> 6) + 1] = hi;
  }
  __syncthreads();
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    lo = fmin(lo, sh[2 * w]);
    hi = fmax(hi, sh[2 * w + 1]);
  }
  __syncthreads();
  double wdt = hi - lo;
  if (!(wdt > 0.0)) wdt = 1.0;   // F' = c I: X_0 = 0, which the trace check rejects
  const int i0 = (tile / nt) * kTile, j0 = (tile % nt) * kTile;
  double ts = 0.0, fs = 0.0;
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int i = i0 + e / kTile, j = j0 + e % kTile;
    if (i >= n || j >= n) continue;
    const double f = 0.5 * (F[o + (long long)i * n + j] + F[o + (long long)j * n + i]);
    const double x = ((i == j ? hi : 0.0) - f) / wdt;
    X[o + (long long)i * n + j] = x;
    fs += x * x;
    if (i == j) ts += x;
  }
  sp2_store_stats(ts, fs, st + ((long long)inst * ntm * ntm + tile) * 2, sh);
}

// One projection step fused into the product: Y = X X (= X^T X, X symmetric)
// by FP64 MFMA (16x16x4), one 32 x 32 tile per block and a 16 x 16 quadrant
// per wavefront.  The operand panels X[k][i-range], X[k][j-range] (both
// coalesced by symmetry) pass through LDS in chunks of kSp2K rows of k, the
// next chunk loaded into registers while the current one is multiplied.  The
// epilogue writes Xn = Y or 2X - Y by the trace rule on the previous
// statistics and stores this tile's (Tr, Tr^2) partial of Xn.
//
// Stopping is decided here, per instance: conv_in[inst] is the first step
// whose X met Tr X - Tr X^2 < idem_tol and |Tr X - N| < trace_tol (-1 while
// none has); this step's X is tested when none has, and the result goes to
// conv_out[inst].  Two steps after that first step the instance is finished:
// Xn = X and its statistics are carried forward unchanged, so steps launched
// beyond the need are cheap copies.  conv_in and conv_out are different
// arrays (the caller alternates them), so no block reads what another block
// of the same launch writes.
constexpr int kSp2K = 96;
__global__ __launch_bounds__(256) void sp2_gemm_kernel(BatchInfo b, int max_n, const int* nocc,
                                                       const double* X, double* Xn,
                                                       const double* st_in, double* st_out,
                                                       int step, double idem_tol, double trace_tol,
                                                       const int* conv_in, int* conv_out) {
  constexpr int kPer = kSp2K * kTile / 256;   // panel elements per thread and chunk
  __shared__ double sh[8];
  __shared__ double As[kSp2K][kTile], Bs[kSp2K][kTile];
  const int ntm = ntiles_1d(max_n);
  int inst, tile;
  if (!xcd_tile(b.ninst, ntm * ntm, inst, tile)) return;
  if (b.active && !b.active[inst]) return;
  const int n = b.nbf[inst], nt = ntiles_1d(n);
  if (tile >= nt * nt) return;
  // X and X^2 are symmetric: the tiles above the diagonal are computed and
  // also written transposed; a tile below it only clears its statistics
  const int ti = tile / nt, tj = tile % nt;
  if (ti > tj) {
    if (threadIdx.x < 2) st_out[((long long)inst * ntm * ntm + tile) * 2 + threadIdx.x] = 0.0;
    return;
  }
  const bool mirror = ti != tj;
  const long long o = b.moff[inst];
  const int ti0 = ti * kTile, tj0 = tj * kTile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = ti0 + (wave >> 1) * 16, j0 = tj0 + (wave & 1) * 16;
  const int c = lane & 15, kq = lane >> 4;
  // FP64 16x16x4 output layout: register r of lane l holds row l / 16 + 4 r,
  // column l % 16 of the quadrant (unlike the FP32 16x16x4 instruction, whose
  // lane holds four consecutive rows)
  double xold[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + kq + 4 * r, j = j0 + c;
    xold[r] = (i < n && j < n) ? X[o + (long long)i * n + j] : 0.0;
  }
  double ra[kPer], rb[kPer];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + 256 * q, k = k0 + e / kTile, cc = e % kTile;
      ra[q] = (k < n && ti0 + cc < n) ? X[o + (long long)k * n + ti0 + cc] : 0.0;
      rb[q] = (k < n && tj0 + cc < n) ? X[o + (long long)k * n + tj0 + cc] : 0.0;
    }
  };
  fetch(0);
  double tr, t2;
  sp2_stats(st_in + (long long)inst * ntm * ntm * 2, nt * nt, tr, t2, sh);
  const double N = nocc[inst];
  int first = conv_in[inst];
  if (first < 0 && tr - t2 < idem_tol && fabs(tr - N) < trace_tol) first = step;
  if (tile == 0 && threadIdx.x == 0) conv_out[inst] = first;
  if (first >= 0 && step >= first + 2) {   // finished: carry X forward (block-uniform)
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
      const int i = ti0 + e / kTile, j = tj0 + e % kTile;
      if (i < n && j < n) {
        Xn[o + (long long)i * n + j] = X[o + (long long)i * n + j];
        if (mirror) Xn[o + (long long)j * n + i] = X[o + (long long)j * n + i];
      }
    }
    const long long so = ((long long)inst * ntm * ntm + tile) * 2;
    if (threadIdx.x < 2) st_out[so + threadIdx.x] = st_in[so + threadIdx.x];
    return;
  }
  const bool square = fabs(t2 - N) < fabs(2.0 * tr - t2 - N);
  v4d acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += kSp2K) {
    __syncthreads();   // the previous chunk has been read
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[e / kTile][e % kTile] = ra[q];
      Bs[e / kTile][e % kTile] = rb[q];
    }
    __syncthreads();
    if (k0 + kSp2K < n) fetch(k0 + kSp2K);
    const int kend = min(kSp2K, n - k0);
    // two accumulators halve the dependent MFMA chain
#pragma unroll
    for (int kk = 0; kk < kSp2K; kk += 8) {
      if (kk < kend) {
        // A[i][k] = X[k][i], B[k][j] = X[k][j]; rows past n were staged as zero
        const double a0 = As[kk + kq][i0 - ti0 + c], b0 = Bs[kk + kq][j0 - tj0 + c];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
      }
      if (kk + 4 < kend) {
        const double a1 = As[kk + 4 + kq][i0 - ti0 + c], b1 = Bs[kk + 4 + kq][j0 - tj0 + c];
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc2, 0, 0, 0);
      }
    }
  }
  acc += acc2;
  double ts = 0.0, fs = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + kq + 4 * r, j = j0 + c;
    if (i < n && j < n) {
      const double y = acc[r];
      const double x = square ? y : 2.0 * xold[r] - y;
      Xn[o + (long long)i * n + j] = x;
      if (mirror) Xn[o + (long long)j * n + i] = x;
      fs += x * x;
      if (i == j) ts += x;
    }
  }
  // an off-diagonal tile stands for its mirror too in sum X_ij^2
  sp2_store_stats(ts, mirror ? 2.0 * fs : fs, st_out + ((long long)inst * ntm * ntm + tile) * 2, sh);
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
                          double* E, hipStream_t s, double kx, const double* Vxc,
                          const double* Exc) {
  double* rowE = E + b.ninst;
  hipLaunchKernelGGL(fock_assemble_kernel, dim3(max_n, b.ninst), dim3(256), 0, s, b, H, J, K, P,
                     F, rowE, kx, Vxc, Exc);
  hipLaunchKernelGGL(energy_sum_kernel, dim3(b.ninst), dim3(256), 0, s, b.ninst, max_n, b.nbf,
                     b.active, rowE, Enuc, E);
}

void launch_antisym(const BatchInfo& b, int max_n, const double* A, double* out, double* emax,
                    hipStream_t s) {
  const int nt = ntiles_1d(max_n);
  hipLaunchKernelGGL(antisym_kernel, dim3(nt, nt, b.ninst), dim3(kTile, 8), 0, s, b, max_n, A, out,
                     emax + b.ninst);
}

void launch_density_change(const BatchInfo& b, int max_n, const double* P, const double* Pprev,
                           double* dP, double* dpmax, hipStream_t s) {
  const int nt = ntiles_1d(max_n);
  hipLaunchKernelGGL(dp_kernel, dim3(nt, nt, b.ninst), dim3(kTile, 8), 0, s, b, max_n, P, Pprev, dP,
                     dpmax + b.ninst);
  hipLaunchKernelGGL(tile_max_kernel, dim3(b.ninst), dim3(64), 0, s, b, max_n, dpmax + b.ninst,
                     dpmax);
}

void launch_diis_store(const DiisArgs& d, int max_n, const double* F, const double* e,
                       hipStream_t s) {
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(diis_copy_kernel, dim3(gx, d.ninst), dim3(256), 0, s, d, F, e);
  hipLaunchKernelGGL(diis_dot_kernel, dim3(d.max_vec, d.ninst, kDotSplit), dim3(256), 0, s, d);
  hipLaunchKernelGGL(diis_advance_kernel, dim3((d.ninst + 63) / 64), dim3(64), 0, s, d);
}

void launch_diis_extrapolate(const DiisArgs& d, int max_n, double* Fbar, hipStream_t s) {
  hipLaunchKernelGGL(diis_solve_kernel, dim3(d.ninst), dim3(64), 0, s, d);
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(diis_combine_kernel, dim3(gx, d.ninst), dim3(256), 0, s, d, Fbar);
}

void launch_convergence(int ninst, int max_n, const int* nbf, const double* E, double* Eprev,
                        double* emax, double etol, double ctol, int* active, int* niter,
                        int* status, hipStream_t s) {
  hipLaunchKernelGGL(convergence_kernel, dim3(ninst), dim3(64), 0, s, ninst, max_n, nbf, E, Eprev,
                     emax + ninst, emax, etol, ctol, active, niter, status);
}

void launch_concat_ints(const int* a, int na, const int* b, int nb, int* out, hipStream_t s) {
  const int n = na + nb;
  if (n <= 0) return;
  hipLaunchKernelGGL(concat_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, na, b, nb, out);
}

void launch_commit(const BatchInfo& b, int max_n, const double* Pnew, double* P, hipStream_t s) {
  const long long nn = (long long)max_n * max_n;
  const unsigned gx = (unsigned)std::min<long long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(commit_kernel, dim3(gx, b.ninst), dim3(256), 0, s, b, Pnew, P);
}

void launch_sp2_bounds(const BatchInfo& b, int max_n, const double* F, double* bounds,
                       hipStream_t s) {
  hipLaunchKernelGGL(sp2_bounds_kernel, dim3((max_n + 3) / 4, b.ninst), dim3(256), 0, s, b, max_n,
                     F, bounds);
}

void launch_sp2_init(const BatchInfo& b, int max_n, const double* F, const double* bounds,
                     double* X, double* st, int* conv, hipStream_t s) {
  const int nt = ntiles_1d(max_n);
  hipLaunchKernelGGL(sp2_init_kernel, dim3(xcd_grid(b.ninst, nt * nt)), dim3(256), 0, s, b, max_n,
                     F, bounds, X, st, conv);
}

void launch_sp2_step(const BatchInfo& b, int max_n, const int* nocc, const double* X, double* Xn,
                     const double* st_in, double* st_out, int step, double idem_tol,
                     double trace_tol, const int* conv_in, int* conv_out, hipStream_t s) {
  const int nt = ntiles_1d(max_n);
  hipLaunchKernelGGL(sp2_gemm_kernel, dim3(xcd_grid(b.ninst, nt * nt)), dim3(256), 0, s, b, max_n,
                     nocc, X, Xn, st_in, st_out, step, idem_tol, trace_tol, conv_in, conv_out);
}

int sp2_tiles(int max_n) { return ntiles_1d(max_n) * ntiles_1d(max_n); }

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
