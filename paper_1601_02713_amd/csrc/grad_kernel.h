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

template <class CG>
__device__ __forceinline__ void grad_block_body(const PrimPair* __restrict__ bp, int nb,
                                                const PrimPair* __restrict__ kp, int nk,
                                                const double* AB, const double* CD,
                                                const double* __restrict__ tab64,
                                                const double* __restrict__ G, double* g9) {
  constexpr int L = CG::LA + CG::LB + CG::LC + CG::LD + 1;
  using R = double;
  if constexpr (!CG::PRIM) {
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
      const PrimPair Q = kp[j];
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
    CG::template con<R>(RA, RB, RC, LA, LB, LC, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], G, g9);
  } else {
    for (int j = 0; j < nk; ++j) {
      const PrimPair Q = kp[j];
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
        CG::template prim<R>(F, B.PAx, B.PAy, B.PAz, -qf * PQx, -qf * PQy, -qf * PQz, Q.PAx,
                             Q.PAy, Q.PAz, pf * PQx, pf * PQy, pf * PQz, B.oo2p, Q.oo2p,
                             0.5 * oopq, B.oo2p * qf, Q.oo2p * pf, 2.0 * B.alpha, 2.0 * B.beta,
                             2.0 * Q.alpha, AB[0], AB[1], AB[2], CD[0], CD[1], CD[2], G, g9);
      }
    }
  }
}

template <class CG>
__device__ __noinline__ void grad_block_outline(const PrimPair* __restrict__ bp, int nb,
                                                const PrimPair* __restrict__ kp, int nk,
                                                const double* AB, const double* CD,
                                                const double* __restrict__ tab64,
                                                const double* __restrict__ G, double* g9) {
  grad_block_body<CG>(bp, nb, kp, nk, AB, CD, tab64, G, g9);
}

template <typename T>
__device__ __forceinline__ T gwave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <class CG>
__global__ __launch_bounds__(256) void grad_kernel(GradArgs a) {
  constexpr int NA = ncart(CG::LA), NB = ncart(CG::LB), NC = ncart(CG::LC), ND = ncart(CG::LD);
  constexpr int NOUT = NA * NB * NC * ND;
  const int lane = threadIdx.x & (kWave - 1);
  const int item_id = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (item_id >= a.nitems) return;
  const WorkItem it = a.items[item_id];
  int bid, kid;
  bool single;
  const bool valid = lane_quartet(it, a.rows, a.kets, lane, bid, kid, single);
  const ShellPair bra = a.pairs[bid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b];
  const int inst = sa.inst;
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const double* __restrict__ P = a.P + mo;
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const int m0 = sa.bf, n0 = sb.bf;
  const ShellPair ket = a.pairs[kid];
  const Shell sc = a.shells[ket.a], sd = a.shells[ket.b];
  const double CD[3] = {sc.x - sd.x, sc.y - sd.y, sc.z - sd.z};
  const double deg = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                     ((kid == bid) ? 1.0 : 2.0);
  const double fac = valid ? 0.5 * deg : 0.0;
  const int l0 = sc.bf, s0 = sd.bf;
  double G[NOUT];
#pragma unroll
  for (int i = 0; i < NA; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double pab = P[(m0 + i) * n + n0 + j];
#pragma unroll
      for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < ND; ++l) {
          const double pcd = P[(l0 + k) * n + s0 + l];
          const double pac = P[(m0 + i) * n + l0 + k], pbd = P[(n0 + j) * n + s0 + l];
          const double pad = P[(m0 + i) * n + s0 + l], pbc = P[(n0 + j) * n + l0 + k];
          G[((i * NB + j) * NC + k) * ND + l] = fac * (pab * pcd - 0.25 * (pac * pbd + pad * pbc));
        }
    }
  double g9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if constexpr (CG::LA + CG::LB + CG::LC + CG::LD >= 5) {
    grad_block_outline<CG>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB,
                           CD, a.boys64, G, g9);
  } else {
    grad_block_body<CG>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                        a.boys64, G, g9);
  }
  if (valid) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * sc.atom + d], g9[6 + d]);
      atomicAdd(&a.grad[3 * sd.atom + d], -(g9[d] + g9[3 + d] + g9[6 + d]));
    }
  }
  if (single) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = gwave_sum(g9[d]), y = gwave_sum(g9[3 + d]);
      if (lane == 0) {
        atomicAdd(&a.grad[3 * sa.atom + d], x);
        atomicAdd(&a.grad[3 * sb.atom + d], y);
      }
    }
  } else if (valid) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * sa.atom + d], g9[d]);
      atomicAdd(&a.grad[3 * sb.atom + d], g9[3 + d]);
    }
  }
}

}  // namespace bscf
