// Two-electron part of the analytic RHF gradient over the screened work lists.
//
// For a canonical shell quartet with g distinct permutations, the gradient
// contribution of every function quartet is
//   (g/2) * [P_mn P_ls - (P_ml P_ns + P_ms P_nl)/4] * d(mn|ls)/dX
// (Pople, Krishnan, Schlegel and Binkley 1979; the bracket collects the
// Coulomb and exchange terms of the sum over the permutations).  Centre
// derivatives of the primitive Cartesian Gaussians,
//   d/dA_i g_a = 2 alpha g_{a+1_i} - a_i g_{a-1_i},
// turn every derivative integral into integrals of raised and lowered classes;
// the D-centre derivative follows from translational invariance,
// d/dD = -(d/dA + d/dB + d/dC).  One wavefront per work item as in the Fock
// build; bra-atom contributions are reduced across the wavefront.
#pragma once
#include "boys.h"
#include "common.h"
#include "grad.h"

namespace bscf {

// One centre's pass of a class whose six contracted sets do not fit a lane's
// registers at once: the primitive loop again, accumulating only the raised
// and lowered sets of centre X (0 = A, 1 = B, 2 = C), then their contraction.
// With CG::NSUB > 1 the pass is split further: sub-pass SUB keeps the SUB-th
// of NSUB contiguous ranges of the centre's sets (raised, then lowered) and
// drops the rest before the contraction, so the compiler removes their
// recurrence work and accumulators from this sub-pass; the contraction is
// linear in the sets, so the sub-passes' sums add up to the centre's.
template <class CG, int X, int SUB, class GF>
__device__ __forceinline__ void grad_centre_pass(const PrimPair* __restrict__ bp, int nb,
                                                 const PrimPair* __restrict__ kp, int nk, int ks,
                                                 const double* AB, const double* CD,
                                                 const double* __restrict__ tab64,
                                                 const GF& gfill, double* g9) {
  constexpr int L = CG::LA + CG::LB + CG::LC + CG::LD + 1;
  constexpr int N1 = X == 0 ? CG::NRA : (X == 1 ? CG::NRB : CG::NRC);
  constexpr int N2 = X == 0 ? CG::NLA : (X == 1 ? CG::NLB : CG::NLC);
  using R = double;
  R S1[N1], S2[N2];
#pragma unroll
  for (int k = 0; k < N1; ++k) S1[k] = 0;
#pragma unroll
  for (int k = 0; k < N2; ++k) S2[k] = 0;
  for (int j = 0; j < nk; ++j) {
    const PrimPair Q = kp[j * ks];
    for (int i = 0; i < nb; ++i) {
      const PrimPair B = bp[i];
      const double pq = B.p + Q.p;
      const double rpq = rsqrt(pq);
      const double oopq = rpq * rpq;
      const double rho = B.p * Q.p * oopq;
      const double PQx = B.Px - Q.Px, PQy = B.Py - Q.Py, PQz = B.Pz - Q.Pz;
      const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
      R F[L + 1];
      boys_f64<L>(T, B.C * Q.C * rpq, tab64, F);
      const double qf = Q.p * oopq, pf = B.p * oopq;
      CG::template vrrx<X, R>(F, B.PAx, B.PAy, B.PAz, -qf * PQx, -qf * PQy, -qf * PQz, Q.PAx,
                              Q.PAy, Q.PAz, pf * PQx, pf * PQy, pf * PQz, B.oo2p, Q.oo2p,
                              0.5 * oopq, B.oo2p * qf, Q.oo2p * pf, 2.0 * B.alpha, 2.0 * B.beta,
                              2.0 * Q.alpha, S1, S2);
    }
  }
  if constexpr (CG::NSUB > 1) {
    constexpr int lo = SUB * (N1 + N2) / CG::NSUB, hi = (SUB + 1) * (N1 + N2) / CG::NSUB;
#pragma unroll
    for (int k = 0; k < N1; ++k)
      if (k < lo || k >= hi) S1[k] = 0;
#pragma unroll
    for (int k = 0; k < N2; ++k)
      if (N1 + k < lo || N1 + k >= hi) S2[k] = 0;
  }
  double G[ncart(CG::LA) * ncart(CG::LB) * ncart(CG::LC) * ncart(CG::LD)];
  gfill(G);
  CG::template conx<X, R>(S1, S2, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], G, g9);
  // The force sums are needed here, in this pass.  Otherwise the compiler
  // sinks the contraction below the later passes' primitive loops (its
  // results are only used at the end), which keeps this pass's accumulators
  // live across those loops: several KB of scratch per lane for the classes
  // with d functions.
#pragma unroll
  for (int k = 0; k < 9; ++k) asm volatile("" : "+v"(g9[k]));
}

template <class CG, int X, int SUB, class GF>
__device__ __forceinline__ void grad_centre_subpasses(const PrimPair* __restrict__ bp, int nb,
                                                      const PrimPair* __restrict__ kp, int nk,
                                                      int ks, const double* AB, const double* CD,
                                                      const double* __restrict__ tab64,
                                                      const GF& gfill, double* g9) {
  grad_centre_pass<CG, X, SUB>(bp, nb, kp, nk, ks, AB, CD, tab64, gfill, g9);
  if constexpr (SUB + 1 < CG::NSUB)
    grad_centre_subpasses<CG, X, SUB + 1>(bp, nb, kp, nk, ks, AB, CD, tab64, gfill, g9);
}

// Contracted-set forms (lane kernels): gfill(G) writes the quartet's density
// factors, called right before each contraction so that they are not live
// across the primitive loop.
template <class CG, class GF>
__device__ __forceinline__ void grad_block_lane(const PrimPair* __restrict__ bp, int nb,
                                                const PrimPair* __restrict__ kp, int nk, int ks,
                                                const double* AB, const double* CD,
                                                const double* __restrict__ tab64,
                                                const GF& gfill, double* g9) {
  constexpr int L = CG::LA + CG::LB + CG::LC + CG::LD + 1;
  using R = double;
  static_assert(!CG::PRIM, "lane gradient classes contract their sets");
  if constexpr (CG::SPLIT) {
    grad_centre_subpasses<CG, 0, 0>(bp, nb, kp, nk, ks, AB, CD, tab64, gfill, g9);
    grad_centre_subpasses<CG, 1, 0>(bp, nb, kp, nk, ks, AB, CD, tab64, gfill, g9);
    grad_centre_subpasses<CG, 2, 0>(bp, nb, kp, nk, ks, AB, CD, tab64, gfill, g9);
  } else {
    R RA[CG::NRA], RB[CG::NRB], RC[CG::NRC], LA[CG::NLA], LB[CG::NLB], LC[CG::NLC];
#pragma unroll
    for (int k = 0; k < CG::NRA; ++k) RA[k] = 0;
#pragma unroll
    for (int k = 0; k < CG::NRB; ++k) RB[k] = 0;
#pragma unroll
    for (int k = 0; k < CG::NRC; ++k) RC[k] = 0;
#pragma unroll
    for (int k = 0; k < CG::NLA; ++k) LA[k] = 0;
#pragma unroll
    for (int k = 0; k < CG::NLB; ++k) LB[k] = 0;
#pragma unroll
    for (int k = 0; k < CG::NLC; ++k) LC[k] = 0;
    for (int j = 0; j < nk; ++j) {
      const PrimPair Q = kp[j * ks];
      for (int i = 0; i < nb; ++i) {
        const PrimPair B = bp[i];
        const double pq = B.p + Q.p;
        const double rpq = rsqrt(pq);
        const double oopq = rpq * rpq;
        const double rho = B.p * Q.p * oopq;
        const double PQx = B.Px - Q.Px, PQy = B.Py - Q.Py, PQz = B.Pz - Q.Pz;
        const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
        R F[L + 1];
        boys_f64<L>(T, B.C * Q.C * rpq, tab64, F);
        const double qf = Q.p * oopq, pf = B.p * oopq;
        CG::template vrr<R>(F, B.PAx, B.PAy, B.PAz, -qf * PQx, -qf * PQy, -qf * PQz, Q.PAx,
                            Q.PAy, Q.PAz, pf * PQx, pf * PQy, pf * PQz, B.oo2p, Q.oo2p,
                            0.5 * oopq, B.oo2p * qf, Q.oo2p * pf, 2.0 * B.alpha, 2.0 * B.beta,
                            2.0 * Q.alpha, RA, RB, RC, LA, LB, LC);
      }
    }
    double G[ncart(CG::LA) * ncart(CG::LB) * ncart(CG::LC) * ncart(CG::LD)];
    gfill(G);
    CG::template con<R>(RA, RB, RC, LA, LB, LC, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], G, g9);
  }
}

template <typename T>
__device__ __forceinline__ T gwave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// One to four wavefronts (blockDim.x = a.unit_threads) per unit of the Fock
// build (a bra pair and its kets; see fock_kernel.h), sharing the unit's LDS.
// The density factor of each quartet is built from the bra shells' P rows
// (LDS) and the ket block of Pk; dE/dR of the bra atoms is reduced across
// each wavefront once per unit, that of the ket atoms is accumulated per atom
// in LDS and flushed with contiguous atomics.
template <class CG>
__global__ __launch_bounds__(256) void grad_unit_kernel(GradArgs a) {
  constexpr int NA = ncart(CG::LA), NB = ncart(CG::LB), NC = ncart(CG::LC), ND = ncart(CG::LD);
  constexpr int NR = NA + NB;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & (kWave - 1);
  const WorkItem u = a.units[blockIdx.x];
  const int bid = a.urows[u.row].bra;
  const ShellPair bra = a.pairs[bid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b];
  const int inst = sa.inst;
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const int m0 = sa.bf, n0 = sb.bf;
  const int a0 = a.atom_off[inst];
  double* Prow = lds;                 // P rows of bf m0 + r (r < NA) and n0 + r - NA
  double* Gat = lds + NR * a.nmax;    // dE/dR per atom of the instance
  const int nat3 = 3 * a.max_atoms;
  PrimPair* Bp = reinterpret_cast<PrimPair*>(Gat + nat3);   // the bra's primitives
  {
    const double* src = reinterpret_cast<const double*>(a.prims + bra.prim0);
    double* dst = reinterpret_cast<double*>(Bp);
    for (int t = tid; t < 12 * bra.nprim; t += nt) dst[t] = src[t];
  }
  for (int t = tid; t < NR * n; t += nt) {
    const int r = t / n, col = t - r * n;
    const int bf = r < NA ? m0 + r : n0 + (r - NA);
    Prow[t] = a.P[mo + (long long)bf * n + col];
  }
  for (int t = tid; t < nat3; t += nt) Gat[t] = 0.0;
  __syncthreads();
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
  double nkeep = 0.0, nkeep_p = 0.0;   // evaluated quartets and primitive quartets
  for (int c0 = 0; c0 < u.count; c0 += nt) {
    const int t = c0 + tid;
    const bool valid = t < u.count;
    int rr = u.row, k0 = u.off + (valid ? t : 0);
    int nk = a.urows[rr].nket;
    while (k0 >= nk) {
      k0 -= nk;
      ++rr;
      nk = a.urows[rr].nket;
    }
    const int pos = a.urows[rr].ket0 + k0;
    const int kid = a.kets[pos];
    const ShellPair ket = a.pairs[kid];
    const Shell sc = a.shells[ket.a], sd = a.shells[ket.b];
    const double CD[3] = {sc.x - sd.x, sc.y - sd.y, sc.z - sd.z};
    const double deg = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                       ((kid == bid) ? 1.0 : 2.0);
    // density-weighted screening (GradArgs): a wavefront whose quartets are
    // all below the bound skips the integrals
    const bool keep = valid && !(a.tau > 0.0 && grad_quartet_bound(a, bid, kid) < a.tau);
    const double fac = keep ? 0.5 * deg : 0.0;
    const double qx = 0.25 * a.kx;
    const int l0 = sc.bf, s0 = sd.bf;
    // density factors of the quartet (Coulomb and exchange terms)
    auto gfill = [&](double* G) {
#pragma unroll
      for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) {
          const double pcd = a.Pk[(long long)(k * ND + l) * a.nk_total + pos];
#pragma unroll
          for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              const double pab = Prow[i * n + n0 + j];
              const double pac = Prow[i * n + l0 + k], pbd = Prow[(NA + j) * n + s0 + l];
              const double pad = Prow[i * n + s0 + l], pbc = Prow[(NA + j) * n + l0 + k];
              G[((i * NB + j) * NC + k) * ND + l] =
                  fac * (pab * pcd - qx * (pac * pbd + pad * pbc));
            }
        }
    };
    double g9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int2 kp = a.kpos[pos];
    if (keep) {
      grad_block_lane<CG>(Bp, bra.nprim, a.kprims + kp.x, ket.nprim, kp.y, AB, CD, a.boys64,
                          gfill, g9);
      nkeep += 1.0;
      nkeep_p += double(bra.nprim * ket.nprim);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gA[d] += g9[d];
      gB[d] += g9[3 + d];
    }
    if (keep) {
      const int ac = sc.atom - a0, ad = sd.atom - a0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        atomicAdd(&Gat[3 * ac + d], g9[6 + d]);
        atomicAdd(&Gat[3 * ad + d], -(g9[d] + g9[3 + d] + g9[6 + d]));
      }
    }
  }
  __syncthreads();
  double* grad = a.grad + 3LL * a0;
  for (int t = tid; t < nat3; t += nt) {
    const double x = Gat[t];
    if (x != 0.0) atomicAdd(&grad[t], x);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = gwave_sum(gA[d]), y = gwave_sum(gB[d]);
    if (lane == 0) {
      atomicAdd(&a.grad[3 * sa.atom + d], x);
      atomicAdd(&a.grad[3 * sb.atom + d], y);
    }
  }
  if (a.gstat) {
    const double q = gwave_sum(nkeep), pq = gwave_sum(nkeep_p);
    if (lane == 0 && q > 0.0) {
      atomicAdd(&a.gstat[0], q);
      atomicAdd(&a.gstat[1], pq);
    }
  }
}

}  // namespace bscf
