// Cooperative kernels: one wavefront (a 64-thread block) per shell quartet.
//
// The recurrence graph of the quartet (Obara-Saika VRR per primitive quartet,
// accumulation into contracted targets, Head-Gordon-Pople HRR, and for the
// gradient the contraction with the density factor) is evaluated level by
// level out of LDS from generated node tables (gen_coop.py): every node is
// dst = sum_t mult_t * scalar[sel_t] * slot[src_t], and the nodes of a level
// are spread over the 64 lanes.  This keeps the state of high angular momentum
// classes in LDS instead of spilling it to scratch, and spreads one quartet's
// latency over a whole wavefront.
#pragma once
#include "boys.h"
#include "common.h"
#include "fock_kernel.h"
#include "grad.h"

namespace bscf {

// scalar slots, same order as gen_coop.SEL
enum : int {
  kSelOne = 0, kSelPA = 1, kSelWP = 4, kSelQC = 7, kSelWQ = 10, kSelOo2p = 13, kSelOo2q = 14,
  kSelOo2pq = 15, kSelRhoP2 = 16, kSelRhoQ2 = 17, kSelAB = 18, kSelCD = 21, kSelWa = 24,
  kSelWb = 25, kSelWc = 26, kNumSel = 27
};

// Evaluate one level range [n0, n1) of a node table.
__device__ __forceinline__ void coop_level(int n0, int n1, const unsigned short* __restrict__ dst,
                                           const int* __restrict__ t0,
                                           const unsigned short* __restrict__ src,
                                           const unsigned char* __restrict__ sel,
                                           const double* __restrict__ mult, const double* sc,
                                           double* slots) {
  for (int nd = n0 + (int)threadIdx.x; nd < n1; nd += kWave) {
    double v = 0.0;
    const int e = t0[nd + 1];
    for (int t = t0[nd]; t < e; ++t) v = fma(mult[t] * sc[sel[t]], slots[src[t]], v);
    slots[dst[nd]] = v;
  }
}

// Primitive loop of one quartet: F_m and scalars into LDS, VRR levels,
// accumulation of the (weighted) targets.  Leaves the contracted targets in
// the accumulator slots and AB, CD in sc.
template <class CP>
__device__ __forceinline__ void coop_primitives(const PrimPair* __restrict__ bp, int nb,
                                                const PrimPair* __restrict__ kp, int nk,
                                                const double AB[3], const double CD[3],
                                                const double* __restrict__ tab64, double* sc,
                                                double* slots) {
  constexpr int L = CP::L;
  const int tid = threadIdx.x;
  for (int t = tid; t < CP::NACC; t += kWave) slots[CP::acc_slot()[t]] = 0.0;
  if (tid == 0) {
    sc[kSelOne] = 1.0;
    sc[kSelAB] = AB[0];
    sc[kSelAB + 1] = AB[1];
    sc[kSelAB + 2] = AB[2];
    sc[kSelCD] = CD[0];
    sc[kSelCD + 1] = CD[1];
    sc[kSelCD + 2] = CD[2];
  }
  for (int j = 0; j < nk; ++j) {
    const PrimPair Q = kp[j];
    for (int i = 0; i < nb; ++i) {
      const PrimPair B = bp[i];
      __syncthreads();  // previous accumulation done before F and scalars change
      if (tid == 0) {
        const double pq = B.p + Q.p;
        const double rpq = rsqrt(pq);
        const double oopq = rpq * rpq;
        const double rho = B.p * Q.p * oopq;
        const double PQx = B.Px - Q.Px, PQy = B.Py - Q.Py, PQz = B.Pz - Q.Pz;
        const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
        double F[L + 1];
        boys_f64<L>(T, B.C * Q.C * rpq, tab64, F);
#pragma unroll
        for (int m = 0; m <= L; ++m) slots[CP::FSLOT + m] = F[m];
        const double qf = Q.p * oopq, pf = B.p * oopq;
        sc[kSelPA] = B.PAx;
        sc[kSelPA + 1] = B.PAy;
        sc[kSelPA + 2] = B.PAz;
        sc[kSelWP] = -qf * PQx;
        sc[kSelWP + 1] = -qf * PQy;
        sc[kSelWP + 2] = -qf * PQz;
        sc[kSelQC] = Q.PAx;
        sc[kSelQC + 1] = Q.PAy;
        sc[kSelQC + 2] = Q.PAz;
        sc[kSelWQ] = pf * PQx;
        sc[kSelWQ + 1] = pf * PQy;
        sc[kSelWQ + 2] = pf * PQz;
        sc[kSelOo2p] = B.oo2p;
        sc[kSelOo2q] = Q.oo2p;
        sc[kSelOo2pq] = 0.5 * oopq;
        sc[kSelRhoP2] = B.oo2p * qf;
        sc[kSelRhoQ2] = Q.oo2p * pf;
        sc[kSelWa] = 2.0 * B.alpha;
        sc[kSelWb] = 2.0 * B.beta;
        sc[kSelWc] = 2.0 * Q.alpha;
      }
      __syncthreads();
      const int* ls = CP::vrr_lstart();
      for (int lv = 0; lv < CP::NVLEV; ++lv) {
        coop_level(ls[lv], ls[lv + 1], CP::vrr_dst(), CP::vrr_t0(), CP::vrr_src(), CP::vrr_sel(),
                   CP::vrr_mult(), sc, slots);
        __syncthreads();
      }
      for (int t = tid; t < CP::NACC; t += kWave)
        slots[CP::acc_slot()[t]] = fma(sc[CP::tgt_w()[t]], slots[CP::tgt_slot()[t]],
                                       slots[CP::acc_slot()[t]]);
    }
  }
  __syncthreads();
}

// Row and column basis functions of element t of the six digestion blocks,
// listed as J_ab, J_cd, K_ac, K_ad, K_bc, K_bd (row-major each).
template <int NA, int NB, int NC, int ND>
__device__ __forceinline__ int2 block_rc(int t, int m0, int n0, int l0, int s0) {
  constexpr int OCD = NA * NB, OAC = OCD + NC * ND, OAD = OAC + NA * NC, OBC = OAD + NA * ND,
                OBD = OBC + NB * NC;
  if (t < OCD) return make_int2(m0 + t / NB, n0 + t % NB);
  if (t < OAC) { t -= OCD; return make_int2(l0 + t / ND, s0 + t % ND); }
  if (t < OAD) { t -= OAC; return make_int2(m0 + t / NC, l0 + t % NC); }
  if (t < OBC) { t -= OAD; return make_int2(m0 + t / ND, s0 + t % ND); }
  if (t < OBD) { t -= OBC; return make_int2(n0 + t / NC, l0 + t % NC); }
  t -= OBD;
  return make_int2(n0 + t / ND, s0 + t % ND);
}

// Quartet of block b of a cooperative launch (one quartet per block).
__device__ __forceinline__ bool coop_quartet(const WorkItem* items, const WorkRow* rows,
                                             const int* kets, int b, int& bid, int& kid) {
  const WorkItem it = items[b >> 6];
  bool single;
  return lane_quartet(it, rows, kets, b & (kWave - 1), bid, kid, single);
}

template <class CP>
__global__ __launch_bounds__(64) void coop_fock_kernel(FockArgs a) {
  __shared__ double slots[CP::NSLOT];
  __shared__ double sc[kNumSel];
  int bid, kid;
  if (!coop_quartet(a.items, a.rows, a.kets, blockIdx.x, bid, kid)) return;
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
              sd = a.shells[ket.b];
  const int inst = sa.inst;
  if (!a.active[inst]) return;
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc_.x - sd.x, sc_.y - sd.y, sc_.z - sd.z};
  coop_primitives<CP>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                      a.boys64, sc, slots);
  const int* hs = CP::hrr_lstart();
  for (int lv = 0; lv < CP::NHLEV; ++lv) {
    coop_level(hs[lv], hs[lv + 1], CP::hrr_dst(), CP::hrr_t0(), CP::hrr_src(), CP::hrr_sel(),
               CP::hrr_mult(), sc, slots);
    __syncthreads();
  }
  // digestion: the six density blocks go to LDS, then each lane contracts one
  // element of one of the six J/K blocks and adds it with one atomic; lanes
  // follow the column index, so an atomic instruction covers few segments
  constexpr int NA = ncart(CP::LA), NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  constexpr int OCD = NA * NB, OAC = OCD + NC * ND, OAD = OAC + NA * NC, OBC = OAD + NA * ND,
                OBD = OBC + NB * NC, NPB = OBD + NB * ND;
  __shared__ double pb[NPB];
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const double* __restrict__ P = a.P + mo;
  double* J = a.J + mo;
  double* K = a.K + mo;
  const int m0 = sa.bf, n0 = sb.bf, l0 = sc_.bf, s0 = sd.bf;
  for (int t = threadIdx.x; t < NPB; t += kWave) {
    const int2 rc = block_rc<NA, NB, NC, ND>(t, m0, n0, l0, s0);
    pb[t] = P[rc.x * n + rc.y];
  }
  for (int e = threadIdx.x; e < CP::NOUT; e += kWave) slots[CP::out_slot()[e]] *= CP::norm()[e];
  __syncthreads();
  const double g = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                   ((kid == bid) ? 1.0 : 2.0);
  const double fj = 0.5 * g, fk = 0.25 * g;
  const unsigned short* os = CP::out_slot();
  for (int t = threadIdx.x; t < NPB; t += kWave) {
    double acc = 0.0, f;
    if (t < OCD) {          // J_ab = sum_cd (ab|cd) P_cd
      const int i = t / NB, j = t % NB;
      #pragma unroll 1
      for (int k = 0; k < NC; ++k)
        #pragma unroll 1
        for (int l = 0; l < ND; ++l)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[OCD + k * ND + l], acc);
      f = fj;
    } else if (t < OAC) {   // J_cd = sum_ab (ab|cd) P_ab
      const int k = (t - OCD) / ND, l = (t - OCD) % ND;
      #pragma unroll 1
      for (int i = 0; i < NA; ++i)
        #pragma unroll 1
        for (int j = 0; j < NB; ++j)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[i * NB + j], acc);
      f = fj;
    } else if (t < OAD) {   // K_ac = sum_bd (ab|cd) P_bd
      const int i = (t - OAC) / NC, k = (t - OAC) % NC;
      #pragma unroll 1
      for (int j = 0; j < NB; ++j)
        #pragma unroll 1
        for (int l = 0; l < ND; ++l)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[OBD + j * ND + l], acc);
      f = fk;
    } else if (t < OBC) {   // K_ad = sum_bc (ab|cd) P_bc
      const int i = (t - OAD) / ND, l = (t - OAD) % ND;
      #pragma unroll 1
      for (int j = 0; j < NB; ++j)
        #pragma unroll 1
        for (int k = 0; k < NC; ++k)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[OBC + j * NC + k], acc);
      f = fk;
    } else if (t < OBD) {   // K_bc = sum_ad (ab|cd) P_ad
      const int j = (t - OBC) / NC, k = (t - OBC) % NC;
      #pragma unroll 1
      for (int i = 0; i < NA; ++i)
        #pragma unroll 1
        for (int l = 0; l < ND; ++l)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[OAD + i * ND + l], acc);
      f = fk;
    } else {                // K_bd = sum_ac (ab|cd) P_ac
      const int j = (t - OBD) / ND, l = (t - OBD) % ND;
      #pragma unroll 1
      for (int i = 0; i < NA; ++i)
        #pragma unroll 1
        for (int k = 0; k < NC; ++k)
          acc = fma(slots[os[((i * NB + j) * NC + k) * ND + l]], pb[OAC + i * NC + k], acc);
      f = fk;
    }
    const int2 rc = block_rc<NA, NB, NC, ND>(t, m0, n0, l0, s0);
    atomicAdd(t < OAC ? &J[rc.x * n + rc.y] : &K[rc.x * n + rc.y], f * acc);
  }
}

template <class CP>
__global__ __launch_bounds__(64) void coop_grad_kernel(GradArgs a) {
  constexpr int NA = ncart(CP::LA), NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  constexpr int NOUT = NA * NB * NC * ND;
  __shared__ double slots[CP::NSLOT];
  __shared__ double G[NOUT];
  __shared__ double sc[kNumSel];
  int bid, kid;
  if (!coop_quartet(a.items, a.rows, a.kets, blockIdx.x, bid, kid)) return;
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
              sd = a.shells[ket.b];
  const int inst = sa.inst;
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const double* __restrict__ P = a.P + mo;
  const double deg = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                     ((kid == bid) ? 1.0 : 2.0);
  for (int e = threadIdx.x; e < NOUT; e += kWave) {
    const int l = e % ND, k = (e / ND) % NC, j = (e / (ND * NC)) % NB, i = e / (ND * NC * NB);
    const int mu = sa.bf + i, nu = sb.bf + j, la = sc_.bf + k, si = sd.bf + l;
    G[e] = 0.5 * deg *
           (P[mu * n + nu] * P[la * n + si] -
            0.25 * (P[mu * n + la] * P[nu * n + si] + P[mu * n + si] * P[nu * n + la]));
  }
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc_.x - sd.x, sc_.y - sd.y, sc_.z - sd.z};
  coop_primitives<CP>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                      a.boys64, sc, slots);
  double g[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = 0.0;
  const int* hs = CP::hrr_lstart();
  const int* cs = CP::con_lstart();
  constexpr int NLOOP = CP::NHLEV + 1 > CP::NCLEV ? CP::NHLEV + 1 : CP::NCLEV;
  for (int lv = 0; lv < NLOOP; ++lv) {
    if (lv > 0 && lv <= CP::NHLEV) {
      coop_level(hs[lv - 1], hs[lv], CP::hrr_dst(), CP::hrr_t0(), CP::hrr_src(), CP::hrr_sel(),
                 CP::hrr_mult(), sc, slots);
      __syncthreads();
    }
    if (lv < CP::NCLEV)
      for (int c = cs[lv] + (int)threadIdx.x; c < cs[lv + 1]; c += kWave) {
      const double v = CP::con_c()[c] * G[CP::con_G()[c]] * slots[CP::con_slot()[c]];
      const int gk = CP::con_g()[c];
#pragma unroll
      for (int k = 0; k < 9; ++k) g[k] += (gk == k) ? v : 0.0;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    for (int o = 32; o > 0; o >>= 1) g[k] += __shfl_xor(g[k], o, kWave);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * sa.atom + d], g[d]);
      atomicAdd(&a.grad[3 * sb.atom + d], g[3 + d]);
      atomicAdd(&a.grad[3 * sc_.atom + d], g[6 + d]);
      atomicAdd(&a.grad[3 * sd.atom + d], -(g[d] + g[3 + d] + g[6 + d]));
    }
  }
}

}  // namespace bscf

namespace bscf {

// Schwarz bound of one pair per block: sqrt(max |(mn|mn)|) over the pair.
template <class CP>
__global__ __launch_bounds__(64) void coop_schwarz_kernel(SchwarzArgs a) {
  __shared__ double slots[CP::NSLOT];
  __shared__ double sc[kNumSel];
  const int pid = a.pair_ids[blockIdx.x];
  const ShellPair pr = a.pairs[pid];
  const Shell sa = a.shells[pr.a], sb = a.shells[pr.b];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  coop_primitives<CP>(a.prims + pr.prim0, pr.nprim, a.prims + pr.prim0, pr.nprim, AB, AB,
                      a.boys64, sc, slots);
  const int* hs = CP::hrr_lstart();
  for (int lv = 0; lv < CP::NHLEV; ++lv) {
    coop_level(hs[lv], hs[lv + 1], CP::hrr_dst(), CP::hrr_t0(), CP::hrr_src(), CP::hrr_sel(),
               CP::hrr_mult(), sc, slots);
    __syncthreads();
  }
  constexpr int NAB = ncart(CP::LA) * ncart(CP::LB);
  double m = 0.0;
  for (int d = threadIdx.x; d < NAB; d += kWave) {
    const int e = d * NAB + d;
    m = fmax(m, fabs(slots[CP::out_slot()[e]] * CP::norm()[e]));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
  if (threadIdx.x == 0) a.Q[pid] = sqrt(m);
}

// Full tensor of one instance (test path): every canonical quartet writes its
// eight index permutations.
template <class CP>
__global__ __launch_bounds__(64) void coop_tensor_kernel(TensorArgs a) {
  __shared__ double slots[CP::NSLOT];
  __shared__ double sc[kNumSel];
  const ShellPair bra = a.pairs[a.quartets[2 * blockIdx.x]];
  const ShellPair ket = a.pairs[a.quartets[2 * blockIdx.x + 1]];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
              sd = a.shells[ket.b];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc_.x - sd.x, sc_.y - sd.y, sc_.z - sd.z};
  coop_primitives<CP>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                      a.boys64, sc, slots);
  const int* hs = CP::hrr_lstart();
  for (int lv = 0; lv < CP::NHLEV; ++lv) {
    coop_level(hs[lv], hs[lv + 1], CP::hrr_dst(), CP::hrr_t0(), CP::hrr_src(), CP::hrr_sel(),
               CP::hrr_mult(), sc, slots);
    __syncthreads();
  }
  constexpr int NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  const long long n = a.n;
  for (int e = threadIdx.x; e < CP::NOUT; e += kWave) {
    const int l = e % ND, k = (e / ND) % NC, j = (e / (ND * NC)) % NB, i = e / (ND * NC * NB);
    const double x = slots[CP::out_slot()[e]] * CP::norm()[e];
    const long long m = sa.bf + i, nn = sb.bf + j, la = sc_.bf + k, s = sd.bf + l;
    const long long idx[8][4] = {{m, nn, la, s}, {nn, m, la, s}, {m, nn, s, la}, {nn, m, s, la},
                                 {la, s, m, nn}, {s, la, m, nn}, {la, s, nn, m}, {s, la, nn, m}};
    for (int q = 0; q < 8; ++q)
      a.out[((idx[q][0] * n + idx[q][1]) * n + idx[q][2]) * n + idx[q][3]] = x;
  }
}

}  // namespace bscf
