// Per-class kernels of the direct-SCF Fock build.
//
// Every shell quartet (ab|cd) is digested into J and K as
//   J_mn += f_J (mn|ls) P_ls,   J_ls += f_J (mn|ls) P_mn,
//   K_ml += f_K (mn|ls) P_ns,   K_ms += f_K (mn|ls) P_nl,
//   K_nl += f_K (mn|ls) P_ms,   K_ns += f_K (mn|ls) P_ml,
// with f_J = g/2, f_K = g/4 and g the number of distinct permutations of the
// shell quartet (1, 2, 4 or 8); J and K are symmetrised afterwards.  Together
// this reproduces J_mn = sum (mn|ls) P_ls and K_ml = sum (mn|ls) P_ns over all
// ordered index quartets.  All K contributions land in the rows of the bra
// shells a and b.
//
// Lane kernels: one wavefront owns one FockUnit, a bra shell pair and up to a
// few hundred of its ket pairs (consecutive ket-list positions, possibly over
// several primitive-count rows).  Each lane evaluates one contracted quartet
// per pass (Obara-Saika VRR over the primitive quartets, contraction, HRR;
// generated per class).  FP64 atomics into global memory are issued per 64-byte
// segment, so scattered per-lane atomics run at about an eighth of the rate of
// row-contiguous ones; the digestion is therefore arranged so that no lane
// scatters into J or K:
//   * the K rows of shells a and b are accumulated in LDS (LDS atomics) for
//     the whole unit and flushed once with row-contiguous global atomics;
//   * the ket-side J block of each lane goes to Jk, indexed by ket-list
//     position and stored component-major (adjacent lanes write adjacent
//     doubles), and is folded into J after all classes (jk_finalize);
//   * the ket-side density P_cd is read from Pk, gathered the same way;
//   * the bra-side J block is reduced across the wavefront at the end.
#pragma once
#include "boys.h"
#include "common.h"

namespace bscf {

struct FockArgs {
  const WorkItem* items;   // 64-quartet items (cooperative kernels)
  int nitems;
  const WorkRow* rows;
  const WorkItem* units;   // per-bra units (lane kernels)
  int nunits;
  const WorkRow* urows;
  const ShellPair* pairs;
  const PrimPair* prims;
  const Shell* shells;
  const int* kets;
  const PrimPair* kprims;  // ket primitive pairs in ket-list order (see kpos)
  const int2* kpos;        // per ket position: first record in kprims, stride between primitives
  int max_prims;           // largest primitive count of a shell pair
  const long long* moff;   // matrix offset per instance
  const int* nbf;          // basis size per instance
  int nmax;                // largest basis size (row length of the LDS accumulators)
  int nk_total;            // number of ket-list positions (stride of Pk and Jk)
  const double* P;
  const double* Pk;        // Pk[e * nk_total + pos] = P_cd component e of the pair at pos
  double* J;
  double* Jk;              // ket-side J, same layout as Pk; cleared by jk_finalize
  double* K;
  const double* boys64;
  const float* boys32;
  const int* active;       // per instance: nonzero while its SCF runs
  // Incremental build (dpmax != nullptr): P is the density change since the
  // last full build and a quartet contributes only when
  // Q_ab Q_cd min(dpmax[inst], 1) >= tau; ukeep[r] is the number of kets of
  // unit row r that pass (the rows' kets run in descending Q, so they are a
  // prefix).  Full build: dpmax == nullptr, every listed quartet contributes.
  const int* ukeep;
  const double* Q;         // Schwarz bound per shell pair
  const double* dpmax;     // per instance max |dP|
  double tau;
  // With dPm (incremental builds): the largest |dP| of every shell-pair block
  // of every instance ([nsh][nsh] at pm_off); a quartet of the kept prefix is
  // also dropped when Q_ab Q_cd min(largest |dP| of its six blocks, 1) < tau,
  // and the class's kept counts of its instance (kept_q, kept_pq and, for the
  // mixed lane form, kept_32, filled from the prefixes) are lowered by what
  // the kernel drops.
  const double* dPm;
  const long long* pm_off;
  const int* shell_off;
  const int* nsh;
  double* kept_q;
  double* kept_pq;
  double* kept_32;
  // Deterministic build (Kfx != nullptr): J, K and Jk accumulate in the
  // fixed-point words of fx_add (two per element, same element order) instead
  // of FP64 atomics on J, K and Jk.
  unsigned long long* Jfx;
  unsigned long long* Kfx;
  unsigned long long* Jkfx;
  // threads of a lane-kernel unit: 64, 128 or 256 (one to four wavefronts
  // sharing the unit's LDS rows); 64 in deterministic builds
  int unit_threads;
};

struct SchwarzArgs {
  const int* pair_ids;     // pairs of one class
  int npairs;
  const ShellPair* pairs;
  const PrimPair* prims;
  const Shell* shells;
  const double* boys64;
  double* Q;               // per pair
};

struct TensorArgs {        // full ERI tensor of one instance (test path)
  const int* quartets;     // (bra, ket) pair indices, canonical
  int nquart;
  const ShellPair* pairs;
  const PrimPair* prims;
  const Shell* shells;
  const double* boys64;
  int n;
  double* out;             // n^4
};

// Contracted (ab|cd) block of class CL for one quartet, in type R.  Classes
// with total angular momentum >= 6 keep one out-of-line copy shared by all
// kernels of the class (bounded code size and compile time).
template <class CL, typename R, int BW = 12>
__device__ __forceinline__ void eri_block_body(const double* __restrict__ bp, int nb,
                                          const PrimPair* __restrict__ kp, int nk, int ks,
                                          const double AB[3], const double CD[3],
                                          const double* __restrict__ tab64,
                                          const float* __restrict__ tab32, R* out) {
  constexpr int L = CL::LA + CL::LB + CL::LC + CL::LD;
  R acc[CL::NACC];
#pragma unroll
  for (int k = 0; k < CL::NACC; ++k) acc[k] = R(0);
  // ket primitives (one set per lane) outermost: each is loaded once; the
  // bra primitives are shared by the lanes of a wavefront and stay cached
  for (int j = 0; j < nk; ++j) {
    const PrimPair Q = kp[j * ks];
    for (int i = 0; i < nb; ++i) {
      PrimPair B;
      if constexpr (BW == 12) {
        B = reinterpret_cast<const PrimPair*>(bp)[i];
      } else {   // the compact (ss|ss) records {p, Px, Py, Pz, C}
        static_assert(BW == 5 && L == 0, "compact bra records carry F_0 data only");
        const double* r = bp + BW * i;
        B = PrimPair{r[0], r[1], r[2], r[3], 0.0, 0.0, 0.0, r[4], 0.0, 0.0, 0.0, 0.0};
      }
      const double pq = B.p + Q.p;
      const double rpq = rsqrt(pq);
      const double oopq = rpq * rpq;
      const double rho = B.p * Q.p * oopq;
      const double PQx = B.Px - Q.Px, PQy = B.Py - Q.Py, PQz = B.Pz - Q.Pz;
      const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
      const double pref = B.C * Q.C * rpq;
      R F[L + 1];
      if constexpr (sizeof(R) == 8) {
        boys_f64<L>(T, pref, tab64, reinterpret_cast<double*>(F));
      } else {
        boys_f32<L>(T, pref, tab32, reinterpret_cast<float*>(F));
      }
      if constexpr (L == 0) {
        acc[0] += F[0];
      } else {
        const double qf = Q.p * oopq, pf = B.p * oopq;
        CL::template vrr<R>(F, R(B.PAx), R(B.PAy), R(B.PAz), R(-qf * PQx), R(-qf * PQy),
                            R(-qf * PQz), R(Q.PAx), R(Q.PAy), R(Q.PAz), R(pf * PQx),
                            R(pf * PQy), R(pf * PQz), R(B.oo2p), R(Q.oo2p), R(0.5 * oopq),
                            R(B.oo2p * qf), R(Q.oo2p * pf), R(1), acc);
      }
    }
  }
  CL::template hrr<R>(acc, R(AB[0]), R(AB[1]), R(AB[2]), R(CD[0]), R(CD[1]), R(CD[2]), out);
}

template <class CL, typename R>
__device__ __noinline__ void eri_block_outline(const PrimPair* __restrict__ bp, int nb,
                                               const PrimPair* __restrict__ kp, int nk, int ks,
                                               const double* AB, const double* CD,
                                               const double* __restrict__ tab64,
                                               const float* __restrict__ tab32, R* out) {
  eri_block_body<CL, R>(reinterpret_cast<const double*>(bp), nb, kp, nk, ks, AB, CD, tab64, tab32,
                        out);
}

// ket primitive j of the quartet is kp[j * ks]; the bra's primitives are
// PrimPair records, or with BW = 5 (class (ss|ss) only) the compact records
// {p, Px, Py, Pz, C} of 5 doubles each
template <class CL, typename R, int BW = 12>
__device__ __forceinline__ void eri_block(const PrimPair* __restrict__ bp, int nb,
                                          const PrimPair* __restrict__ kp, int nk, int ks,
                                          const double AB[3], const double CD[3],
                                          const double* __restrict__ tab64,
                                          const float* __restrict__ tab32, R* out) {
  if constexpr (CL::LA + CL::LB + CL::LC + CL::LD >= 6) {
    eri_block_outline<CL, R>(bp, nb, kp, nk, ks, AB, CD, tab64, tab32, out);
  } else {
    eri_block_body<CL, R, BW>(reinterpret_cast<const double*>(bp), nb, kp, nk, ks, AB, CD, tab64,
                              tab32, out);
  }
}

// Q_ab Q_cd min(largest |dP| over the quartet's six blocks, 1)
__device__ __forceinline__ double fock_block_bound(const FockArgs& a, int bid, int kid) {
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const int inst = a.shells[bra.a].inst;
  const int s0 = a.shell_off[inst], ns = a.nsh[inst];
  const double* M = a.dPm + a.pm_off[inst];
  const int i = bra.a - s0, j = bra.b - s0, k = ket.a - s0, l = ket.b - s0;
  const double m = fmax(fmax(fmax(M[i * ns + j], M[k * ns + l]), fmax(M[i * ns + k], M[j * ns + l])),
                        fmax(M[i * ns + l], M[j * ns + k]));
  return a.Q[bid] * a.Q[kid] * fmin(m, 1.0);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// LDS footprint of the unit kernel of a class: K accumulators and P rows of the
// bra shells, (NA + NB) rows of nmax doubles each, and the bra's primitive
// pairs (at most max_prims records of 12 doubles; of 5 for an (ss) bra, whose
// only class (ss|ss) needs p, P and C).  The footprint bounds the blocks per
// CU, so it is kept small.
__host__ __device__ constexpr int unit_lds_doubles(int la, int lb, int nmax, int max_prims) {
  return 2 * (ncart(la) + ncart(lb)) * nmax + (la + lb == 0 ? 5 : 12) * max_prims;
}

// Quartets of unit u selected by sel (0: the kept ones of every row;
// 1: those in each row's FP64 prefix, row.pad kets long; 2: the rest), with
// keep (incremental builds) bounding each row's kept prefix when given
__device__ __forceinline__ void unit_sel_range(const WorkRow& w, const int* keep, int rr, int sel,
                                               int& lo, int& hi) {
  hi = keep ? keep[rr] : w.nket;
  lo = 0;
  if (sel == 1) hi = min(hi, w.pad);
  else if (sel == 2) lo = w.pad;
}

__device__ __forceinline__ int unit_sel_count(const WorkItem& u, const WorkRow* __restrict__ rows,
                                              const int* keep, int sel) {
  int rem = u.count, rr = u.row, off = u.off, cnt = 0;
  while (rem > 0) {
    const WorkRow w = rows[rr];
    const int take = min(w.nket - off, rem);
    int lo, hi;
    unit_sel_range(w, keep, rr, sel, lo, hi);
    cnt += max(0, min(off + take, hi) - max(off, lo));
    rem -= take;
    ++rr;
    off = 0;
  }
  return cnt;
}

// Row rr and position k0 of selected quartet t (t < unit_sel_count) of unit u
__device__ __forceinline__ void unit_sel_quartet(const WorkItem& u,
                                                 const WorkRow* __restrict__ rows,
                                                 const int* keep, int sel, int t, int& rr,
                                                 int& k0) {
  int rem = u.count, off = u.off;
  rr = u.row;
  for (;;) {
    const WorkRow w = rows[rr];
    const int take = min(w.nket - off, rem);
    int lo, hi;
    unit_sel_range(w, keep, rr, sel, lo, hi);
    const int b = max(off, lo), c = max(0, min(off + take, hi) - b);
    if (t < c) {
      k0 = b + t;
      return;
    }
    t -= c;
    rem -= take;
    ++rr;
    off = 0;
  }
}

// MIX (with R = double): the mixed-precision form in one launch: the unit's
// quartets in its rows' FP64 prefixes first, with FP64 integrals, then the rest
// with FP32 integrals, over one set of LDS rows and one flush.
// A unit is one to four wavefronts (blockDim.x = a.unit_threads): they share
// the unit's LDS rows, so at large basis sizes, where those rows bound the
// workgroups per CU, more wavefronts per unit keep more of them resident.
template <class CL, typename R, bool MIX = false>
__global__ __launch_bounds__(256) void fock_unit_kernel(FockArgs a) {
  constexpr int NA = ncart(CL::LA), NB = ncart(CL::LB), NC = ncart(CL::LC), ND = ncart(CL::LD);
  constexpr int NR = NA + NB;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & (kWave - 1);
  const WorkItem u = a.units[blockIdx.x];
  const int bid = a.urows[u.row].bra;
  const ShellPair bra = a.pairs[bid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b];
  const int inst = sa.inst;
  if (!a.active[inst]) return;
  // incremental build: a unit whose quartets all fall below the bound does nothing
  const bool screen = a.dpmax != nullptr;
  const int* keep = screen ? a.ukeep : nullptr;
  if (screen && unit_sel_count(u, a.urows, keep, 0) == 0) return;
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const int m0 = sa.bf, n0 = sb.bf;
  double* Kacc = lds;           // row r: K row of bf m0 + r (r < NA) or n0 + r - NA
  double* Prow = lds + NR * n;  // the same rows of P
  // the bra's primitives: whole records, or for an (ss) bra {p, Px, Py, Pz, C}
  constexpr int BW = CL::LA + CL::LB == 0 ? 5 : 12;
  PrimPair* Bp = reinterpret_cast<PrimPair*>(lds + 2 * NR * a.nmax);
  for (int t = tid; t < NR * n; t += nt) {
    const int r = t / n, col = t - r * n;
    const int bf = r < NA ? m0 + r : n0 + (r - NA);
    Kacc[t] = 0.0;
    Prow[t] = a.P[mo + (long long)bf * n + col];
  }
  {
    const double* src = reinterpret_cast<const double*>(a.prims + bra.prim0);
    double* dst = reinterpret_cast<double*>(Bp);
    for (int t = tid; t < BW * bra.nprim; t += nt) {
      if constexpr (BW == 12) {
        dst[t] = src[t];
      } else {
        const int i = t / BW, f = t - i * BW;   // fields p, Px, Py, Pz, then C (field 7)
        dst[t] = src[12 * i + (f < 4 ? f : 7)];
      }
    }
  }
  __syncthreads();
  double Pab[NA][NB], jab[NA][NB];
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      Pab[i][j] = Prow[i * n + n0 + j];
      jab[i][j] = 0.0;
    }
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  double dropped[3] = {0.0, 0.0, 0.0};   // quartets, primitive quartets, FP32 quartets
  // one pass over the quartets of selection sel with integrals of precision RP
  auto pass = [&](auto prec, int sel) {
  using RP = decltype(prec);
  const int total = (screen || sel != 0) ? unit_sel_count(u, a.urows, keep, sel) : u.count;
  for (int c0 = 0; c0 < total; c0 += nt) {
    const int t = c0 + tid;
    const bool valid = t < total;
    int rr, k0;
    if (screen || sel != 0) {
      unit_sel_quartet(u, a.urows, keep, sel, valid ? t : 0, rr, k0);
    } else {
      rr = u.row;
      k0 = u.off + (valid ? t : 0);
      int nk = a.urows[rr].nket;
      while (k0 >= nk) {
        k0 -= nk;
        ++rr;
        nk = a.urows[rr].nket;
      }
    }
    const int pos = a.urows[rr].ket0 + k0;
    const int kid = a.kets[pos];
    const ShellPair ket = a.pairs[kid];
    if (valid && a.dPm && fock_block_bound(a, bid, kid) < a.tau) {
      dropped[0] += 1.0;
      dropped[1] += double(bra.nprim * ket.nprim);
      if (sel == 2) dropped[2] += 1.0;
      continue;   // the lanes of this pass that keep their quartet go on
    }
    const Shell sc = a.shells[ket.a], sd = a.shells[ket.b];
    const double CD[3] = {sc.x - sd.x, sc.y - sd.y, sc.z - sd.z};
    const int2 kp = a.kpos[pos];
    RP v[CL::NOUT];
    eri_block<CL, RP, BW>(Bp, bra.nprim, a.kprims + kp.x, ket.nprim, kp.y, AB, CD, a.boys64,
                          a.boys32, v);
    const double g = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                     ((kid == bid) ? 1.0 : 2.0);
    const double fj = valid ? 0.5 * g : 0.0;
    const double fk = 0.5 * fj;
    const int l0 = sc.bf, s0 = sd.bf;
    double Pcd[NC][ND];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < ND; ++l) Pcd[k][l] = a.Pk[(long long)(k * ND + l) * a.nk_total + pos];
    double jket[NC][ND], kac[NA][NC], kad[NA][ND], kbc[NB][NC], kbd[NB][ND];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int l = 0; l < ND; ++l) jket[k][l] = 0.0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
#pragma unroll
      for (int k = 0; k < NC; ++k) kac[i][k] = 0.0;
#pragma unroll
      for (int l = 0; l < ND; ++l) kad[i][l] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
#pragma unroll
      for (int k = 0; k < NC; ++k) kbc[j][k] = 0.0;
#pragma unroll
      for (int l = 0; l < ND; ++l) kbd[j][l] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double jb = 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
          for (int l = 0; l < ND; ++l) {
            const double x = double(v[((i * NB + j) * NC + k) * ND + l]);
            jb = fma(x, Pcd[k][l], jb);
            jket[k][l] = fma(x, Pab[i][j], jket[k][l]);
            kac[i][k] = fma(x, Prow[(NA + j) * n + s0 + l], kac[i][k]);
            kad[i][l] = fma(x, Prow[(NA + j) * n + l0 + k], kad[i][l]);
            kbc[j][k] = fma(x, Prow[i * n + s0 + l], kbc[j][k]);
            kbd[j][l] = fma(x, Prow[i * n + l0 + k], kbd[j][l]);
          }
        jab[i][j] = fma(fj, jb, jab[i][j]);
      }
    if (valid) {
#pragma unroll
      for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) {
          const long long e = (long long)(k * ND + l) * a.nk_total + pos;
          if (a.Jkfx) fx_add(&a.Jkfx[2 * e], fj * jket[k][l]);
          else atomicAdd(&a.Jk[e], fj * jket[k][l]);
        }
#pragma unroll
      for (int i = 0; i < NA; ++i) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomicAdd(&Kacc[i * n + l0 + k], fk * kac[i][k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomicAdd(&Kacc[i * n + s0 + l], fk * kad[i][l]);
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
#pragma unroll
        for (int k = 0; k < NC; ++k) atomicAdd(&Kacc[(NA + j) * n + l0 + k], fk * kbc[j][k]);
#pragma unroll
        for (int l = 0; l < ND; ++l) atomicAdd(&Kacc[(NA + j) * n + s0 + l], fk * kbd[j][l]);
      }
    }
  }
  };
  if constexpr (MIX) {
    pass(double(0), 1);
    pass(float(0), 2);
  } else {
    pass(R(0), 0);
  }
  if (a.dPm) {
#pragma unroll
    for (int k = 0; k < 3; ++k) dropped[k] = wave_sum(dropped[k]);
    if (lane == 0 && dropped[0] > 0.0) {
      atomicAdd(&a.kept_q[inst], -dropped[0]);
      atomicAdd(&a.kept_pq[inst], -dropped[1]);
      if (a.kept_32 && dropped[2] > 0.0) atomicAdd(&a.kept_32[inst], -dropped[2]);
    }
  }
  __syncthreads();
  for (int t = tid; t < NR * n; t += nt) {
    const double x = Kacc[t];
    if (x != 0.0) {
      const int r = t / n, col = t - r * n;
      const int bf = r < NA ? m0 + r : n0 + (r - NA);
      const long long e = mo + (long long)bf * n + col;
      if (a.Kfx) fx_add(&a.Kfx[2 * e], x);
      else atomicAdd(&a.K[e], x);
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double x = wave_sum(jab[i][j]);
      const long long e = mo + (long long)(m0 + i) * n + n0 + j;
      if (lane == 0) {
        if (a.Jfx) fx_add(&a.Jfx[2 * e], x);
        else atomicAdd(&a.J[e], x);
      }
    }
}

// Q for each pair of class (LA LB|LA LB): sqrt(max |(mn|mn)|).
template <class CL>
__global__ __launch_bounds__(256) void schwarz_kernel(SchwarzArgs a) {
  constexpr int NA = ncart(CL::LA), NB = ncart(CL::LB);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.npairs) return;
  const int pid = a.pair_ids[t];
  const ShellPair pr = a.pairs[pid];
  const Shell sa = a.shells[pr.a], sb = a.shells[pr.b];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  double v[CL::NOUT];
  eri_block<CL, double>(a.prims + pr.prim0, pr.nprim, a.prims + pr.prim0, pr.nprim, 1, AB, AB,
                        a.boys64, nullptr, v);
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) m = fmax(m, fabs(v[(i * NB + j) * NA * NB + i * NB + j]));
  a.Q[pid] = sqrt(m);
}

// Full tensor (test path): every canonical quartet writes its 8 permutations.
template <class CL>
__global__ __launch_bounds__(64) void tensor_kernel(TensorArgs a) {
  constexpr int NA = ncart(CL::LA), NB = ncart(CL::LB), NC = ncart(CL::LC), ND = ncart(CL::LD);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nquart) return;
  const ShellPair bra = a.pairs[a.quartets[2 * t]], ket = a.pairs[a.quartets[2 * t + 1]];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc = a.shells[ket.a],
              sd = a.shells[ket.b];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc.x - sd.x, sc.y - sd.y, sc.z - sd.z};
  double v[CL::NOUT];
  eri_block<CL, double>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, 1, AB, CD,
                        a.boys64, nullptr, v);
  const long long n = a.n;
  for (int i = 0; i < NA; ++i)
    for (int j = 0; j < NB; ++j)
      for (int k = 0; k < NC; ++k)
        for (int l = 0; l < ND; ++l) {
          const double x = v[((i * NB + j) * NC + k) * ND + l];
          const long long m = sa.bf + i, nn = sb.bf + j, la = sc.bf + k, s = sd.bf + l;
          const long long idx[8][4] = {{m, nn, la, s}, {nn, m, la, s}, {m, nn, s, la},
                                       {nn, m, s, la}, {la, s, m, nn}, {s, la, m, nn},
                                       {la, s, nn, m}, {s, la, nn, m}};
          for (int q = 0; q < 8; ++q)
            a.out[((idx[q][0] * n + idx[q][1]) * n + idx[q][2]) * n + idx[q][3]] = x;
        }
}

}  // namespace bscf
