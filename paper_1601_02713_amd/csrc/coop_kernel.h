// Cooperative kernels: one block of CP::NT threads (one to eight wavefronts)
// per shell quartet.
//
// The recurrence graph of the quartet (Obara-Saika VRR per primitive quartet,
// accumulation into contracted targets, Head-Gordon-Pople HRR, and for the
// gradient the contraction with the density factor) is evaluated level by
// level out of LDS from generated node tables (gen_coop.py): every node is
// dst = sum_t mult_t * scalar[sel_t] * slot[src_t], and the nodes of a level
// are spread over the threads of the block.  A node is one 64-bit word (first
// term, destination slot, term count) and a term one 32-bit word (source slot,
// scalar selector, integer multiplier + 8), so each term costs one table load.
// This keeps the state of high angular momentum classes in LDS instead of
// spilling it to scratch; classes whose LDS footprint admits few blocks per CU
// get more threads per quartet.
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

// Evaluate one level range [n0, n1) of a packed node table (nodes of at most
// MAXT terms).  The kernels are bound by the latency of the table loads, so a
// thread takes two nodes at a time and issues every term load of both before
// it uses any of them.
template <int NT, int MAXT>
__device__ __forceinline__ void coop_level(int n0, int n1,
                                           const unsigned long long* __restrict__ node,
                                           const unsigned int* __restrict__ term,
                                           const double* sc, double* slots) {
  for (int nd = n0 + (int)threadIdx.x; nd < n1; nd += 2 * NT) {
    const bool two = nd + NT < n1;
    const unsigned long long w0 = node[nd];
    const unsigned long long w1 = two ? node[nd + NT] : 0ull;   // no terms
    const int a0 = (int)(w0 & 0xFFFFFFFFull), c0 = (int)((w0 >> 48) & 0xFFull);
    const int a1 = (int)(w1 & 0xFFFFFFFFull), c1 = (int)((w1 >> 48) & 0xFFull);
    unsigned int u0[MAXT], u1[MAXT];
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      u0[k] = k < c0 ? term[a0 + k] : 0u;
      u1[k] = k < c1 ? term[a1 + k] : 0u;
    }
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      if (k < c0)
        v0 = fma((double)((int)(u0[k] >> 24) - 8) * sc[(u0[k] >> 16) & 0xFFu], slots[u0[k] & 0xFFFFu], v0);
      if (k < c1)
        v1 = fma((double)((int)(u1[k] >> 24) - 8) * sc[(u1[k] >> 16) & 0xFFu], slots[u1[k] & 0xFFFFu], v1);
    }
    slots[(int)((w0 >> 32) & 0xFFFFull)] = v0;
    if (two) slots[(int)((w1 >> 32) & 0xFFFFull)] = v1;
  }
}

// Terms per node: a VRR node has at most five (gen_coop.vrr_graph), an HRR
// node two.
constexpr int kVrrTerms = 5, kHrrTerms = 2;

// Primitive loop of one quartet: F_m and scalars into LDS, VRR levels,
// accumulation of the (weighted) targets.  Leaves the contracted targets in
// the accumulator slots and AB, CD in sc.
template <class CP>
__device__ __forceinline__ void coop_primitives(const PrimPair* __restrict__ bp, int nb,
                                                const PrimPair* __restrict__ kp, int nk,
                                                const double AB[3], const double CD[3],
                                                const double* __restrict__ tab64, double* sc,
                                                double* slots) {
  constexpr int L = CP::L, NT = CP::NT;
  const int tid = threadIdx.x;
  for (int t = tid; t < CP::NACC; t += NT) slots[t] = 0.0;   // accumulator k is slot k
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
        coop_level<NT, kVrrTerms>(ls[lv], ls[lv + 1], CP::vrr_node(), CP::vrr_term(), sc, slots);
        __syncthreads();
      }
      // accumulator k is slot k (gen_coop places them first); two at a time,
      // table loads first
      const unsigned short* ts = CP::tgt_slot();
      const unsigned char* tw = CP::tgt_w();
      for (int t = tid; t < CP::NACC; t += 2 * NT) {
        const bool two = t + NT < CP::NACC;
        const int s0 = ts[t], w0 = tw[t];
        const int s1 = two ? ts[t + NT] : 0, w1 = two ? tw[t + NT] : 0;
        slots[t] = fma(sc[w0], slots[s0], slots[t]);
        if (two) slots[t + NT] = fma(sc[w1], slots[s1], slots[t + NT]);
      }
    }
  }
  __syncthreads();
}

// HRR levels of a quartet (Fock, Schwarz and tensor kernels).
template <class CP>
__device__ __forceinline__ void coop_hrr(const double* sc, double* slots) {
  const int* hs = CP::hrr_lstart();
  for (int lv = 0; lv < CP::NHLEV; ++lv) {
    coop_level<CP::NT, kHrrTerms>(hs[lv], hs[lv + 1], CP::hrr_node(), CP::hrr_term(), sc, slots);
    __syncthreads();
  }
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

// Quartet of block b of a cooperative launch (one quartet per block, over
// coop_blocks(nitems) blocks).  Block b runs on XCD b % kXcds; that XCD's
// blocks take the items at positions congruent to it modulo kXcds in order,
// 64 blocks (one per quartet) per item.  False for blocks past the items
// and for lanes past an item's quartets.
__device__ __forceinline__ bool coop_quartet(const WorkItem* items, int nitems,
                                             const WorkRow* rows, const int* kets, int b,
                                             int& bid, int& kid) {
  const int x = b % kXcds, j = b / kXcds;
  const int pos = x + kXcds * (j >> 6);
  if (pos >= nitems) return false;
  const WorkItem it = items[pos];
  bool single;
  return lane_quartet(it, rows, kets, j & (kWave - 1), bid, kid, single);
}
__host__ __device__ inline unsigned coop_blocks(int nitems) {
  return (unsigned)(kXcds * ((nitems + kXcds - 1) / kXcds) * kWave);
}

template <class CP>
__global__ __launch_bounds__(CP::NT) void coop_fock_kernel(FockArgs a) {
  constexpr int NT = CP::NT;
  __shared__ double slots[CP::NSLOT];
  __shared__ double sc[kNumSel];
  int bid, kid;
  if (!coop_quartet(a.items, a.nitems, a.rows, a.kets, blockIdx.x, bid, kid)) return;
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
              sd = a.shells[ket.b];
  const int inst = sa.inst;
  if (!a.active[inst]) return;
  // incremental build: quartets below the density-weighted bound do nothing
  if (a.dpmax && a.Q[bid] * a.Q[kid] * fmin(a.dpmax[inst], 1.0) < a.tau) return;
  // and those that the bound of their own density-change blocks drops (the
  // kept counts, taken from the instance bound, lose them)
  if (a.dPm && fock_block_bound(a, bid, kid) < a.tau) {
    if (threadIdx.x == 0) {
      atomicAdd(&a.kept_q[inst], -1.0);
      atomicAdd(&a.kept_pq[inst], -double(bra.nprim * ket.nprim));
    }
    return;
  }
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc_.x - sd.x, sc_.y - sd.y, sc_.z - sd.z};
  coop_primitives<CP>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                      a.boys64, sc, slots);
  coop_hrr<CP>(sc, slots);
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
  for (int t = threadIdx.x; t < NPB; t += NT) {
    const int2 rc = block_rc<NA, NB, NC, ND>(t, m0, n0, l0, s0);
    pb[t] = P[rc.x * n + rc.y];
  }
  for (int e = threadIdx.x; e < CP::NOUT; e += NT) slots[CP::out_slot()[e]] *= CP::norm()[e];
  __syncthreads();
  const double g = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                   ((kid == bid) ? 1.0 : 2.0);
  const double fj = 0.5 * g, fk = 0.25 * g;
  const unsigned short* os = CP::out_slot();
  for (int t = threadIdx.x; t < NPB; t += NT) {
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
    if (a.Kfx) {
      const long long e = mo + (long long)rc.x * n + rc.y;
      fx_add(t < OAC ? &a.Jfx[2 * e] : &a.Kfx[2 * e], f * acc);
    } else {
      atomicAdd(t < OAC ? &J[rc.x * n + rc.y] : &K[rc.x * n + rc.y], f * acc);
    }
  }
}

// Quartet q of block b of a launch with QB quartets per block (QB divides
// 64): block b runs on XCD b % kXcds, and its quartets are lanes
// (b / kXcds) QB + q of the items at positions congruent to that XCD, 64 per
// item, so all QB belong to one item.
__device__ __forceinline__ bool coop_quartet_q(const WorkItem* items, int nitems,
                                               const WorkRow* rows, const int* kets, int b, int q,
                                               int QB, int& bid, int& kid) {
  const int x = b % kXcds, j = (b / kXcds) * QB + q;
  const int pos = x + kXcds * (j >> 6);
  if (pos >= nitems) return false;
  const WorkItem it = items[pos];
  bool single;
  return lane_quartet(it, rows, kets, j & (kWave - 1), bid, kid, single);
}
__host__ __device__ inline unsigned coop_blocks_q(int nitems, int qb) {
  return (unsigned)(kXcds * ((nitems + kXcds - 1) / kXcds) * (kWave / qb));
}

// One level range of a node table for QB quartets at once: each node's words
// are loaded once and applied to every quartet's slots.
template <int NT, int MAXT, int QB, int NSLOT>
__device__ __forceinline__ void coop_level_q(int n0, int n1,
                                             const unsigned long long* __restrict__ node,
                                             const unsigned int* __restrict__ term,
                                             const double (*sc)[kNumSel], double (*slots)[NSLOT]) {
  if constexpr (QB == 1) {
    coop_level<NT, MAXT>(n0, n1, node, term, sc[0], slots[0]);
  } else {
    for (int nd = n0 + (int)threadIdx.x; nd < n1; nd += NT) {
      const unsigned long long w = node[nd];
      const int a0 = (int)(w & 0xFFFFFFFFull), c = (int)((w >> 48) & 0xFFull);
      const int dst = (int)((w >> 32) & 0xFFFFull);
      unsigned int u[MAXT];
#pragma unroll
      for (int k = 0; k < MAXT; ++k) u[k] = k < c ? term[a0 + k] : 0u;
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < MAXT; ++k)
          if (k < c)
            v = fma((double)((int)(u[k] >> 24) - 8) * sc[q][(u[k] >> 16) & 0xFFu],
                    slots[q][u[k] & 0xFFFFu], v);
        slots[q][dst] = v;
      }
    }
  }
}

// Gradient: CP::QB quartets per block of CP::NTQ threads.  Per quartet the
// density factors G, the primitive loop (threads 0..QB-1 set up one quartet's
// primitive each, a quartet without that primitive gets F = 0), the HRR of
// every set and its contraction with G into the nine components of the A, B
// and C centres; thread t contracts for quartet t % QB.
template <class CP>
__global__ __launch_bounds__(CP::NTQ) void coop_grad_kernel(GradArgs a) {
  constexpr int NT = CP::NTQ, NW = NT / kWave, QB = CP::QB, L = CP::L;
  constexpr int NA = ncart(CP::LA), NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  constexpr int NOUT = NA * NB * NC * ND;
  static_assert(NT % QB == 0 && kWave % QB == 0, "quartets per block");
  __shared__ double slots[QB][CP::NSLOT];
  __shared__ double G[QB][NOUT];
  __shared__ double sc[QB][kNumSel];
  __shared__ double ctab[CP::NCTAB];
  __shared__ double red[NW][QB][9];
  __shared__ int qv[QB], qbid[QB], qkid[QB], qnp[QB];
  const int tid = threadIdx.x;
  if (tid < QB) {
    int bid = 0, kid = 0;
    const bool ok =
        coop_quartet_q(a.items, a.nitems, a.rows, a.kets, blockIdx.x, tid, QB, bid, kid) &&
        !(a.tau > 0.0 && grad_quartet_bound(a, bid, kid) < a.tau);
    qv[tid] = ok ? 1 : 0;
    qbid[tid] = bid;
    qkid[tid] = kid;
    qnp[tid] = ok ? a.pairs[bid].nprim * a.pairs[kid].nprim : 0;
    if (ok) {
      const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
      const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
                  sd = a.shells[ket.b];
      sc[tid][kSelOne] = 1.0;
      sc[tid][kSelAB] = sa.x - sb.x;
      sc[tid][kSelAB + 1] = sa.y - sb.y;
      sc[tid][kSelAB + 2] = sa.z - sb.z;
      sc[tid][kSelCD] = sc_.x - sd.x;
      sc[tid][kSelCD + 1] = sc_.y - sd.y;
      sc[tid][kSelCD + 2] = sc_.z - sd.z;
    } else {
      for (int k = 0; k < kNumSel; ++k) sc[tid][k] = 0.0;
    }
  }
  for (int t = tid; t < CP::NCTAB; t += NT) ctab[t] = CP::con_ctab()[t];
  __syncthreads();
  int np = 0, any = 0;
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    np = max(np, qnp[q]);
    any |= qv[q];
  }
  if (a.gstat && tid == 0 && any) {
    double nq = 0.0, npq = 0.0;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      nq += qv[q];
      npq += qnp[q];
    }
    atomicAdd(&a.gstat[0], nq);
    atomicAdd(&a.gstat[1], npq);
  }
  if (!any) return;
  // density factors of every quartet (zero for an empty one)
  for (int e = tid; e < QB * NOUT; e += NT) {
    const int q = e / NOUT, r = e - q * NOUT;
    double v = 0.0;
    if (qv[q]) {
      const ShellPair bra = a.pairs[qbid[q]], ket = a.pairs[qkid[q]];
      const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
                  sd = a.shells[ket.b];
      const long long mo = a.moff[sa.inst];
      const int n = a.nbf[sa.inst];
      const double* __restrict__ P = a.P + mo;
      const double deg = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                         ((qkid[q] == qbid[q]) ? 1.0 : 2.0);
      const int l = r % ND, k = (r / ND) % NC, j = (r / (ND * NC)) % NB, i = r / (ND * NC * NB);
      const int mu = sa.bf + i, nu = sb.bf + j, la = sc_.bf + k, si = sd.bf + l;
      v = 0.5 * deg *
          (P[mu * n + nu] * P[la * n + si] -
           0.25 * a.kx * (P[mu * n + la] * P[nu * n + si] + P[mu * n + si] * P[nu * n + la]));
    }
    G[q][r] = v;
  }
  for (int t = tid; t < QB * CP::NACC; t += NT) slots[t % QB][t / QB] = 0.0;   // accumulator k is slot k
  // primitive loop
  for (int p = 0; p < np; ++p) {
    __syncthreads();   // the previous accumulation is done before F and scalars change
    if (tid < QB) {
      const int q = tid;
      double* S = slots[q];
      double* X = sc[q];
      if (p < qnp[q]) {
        const ShellPair bra = a.pairs[qbid[q]], ket = a.pairs[qkid[q]];
        const int nb = bra.nprim, jj = p / nb, ii = p - jj * nb;
        const PrimPair B = a.prims[bra.prim0 + ii], Q = a.prims[ket.prim0 + jj];
        const double pq = B.p + Q.p;
        const double rpq = rsqrt(pq);
        const double oopq = rpq * rpq;
        const double rho = B.p * Q.p * oopq;
        const double PQx = B.Px - Q.Px, PQy = B.Py - Q.Py, PQz = B.Pz - Q.Pz;
        const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
        double F[L + 1];
        boys_f64<L>(T, B.C * Q.C * rpq, a.boys64, F);
#pragma unroll
        for (int m = 0; m <= L; ++m) S[CP::FSLOT + m] = F[m];
        const double qf = Q.p * oopq, pf = B.p * oopq;
        X[kSelPA] = B.PAx;
        X[kSelPA + 1] = B.PAy;
        X[kSelPA + 2] = B.PAz;
        X[kSelWP] = -qf * PQx;
        X[kSelWP + 1] = -qf * PQy;
        X[kSelWP + 2] = -qf * PQz;
        X[kSelQC] = Q.PAx;
        X[kSelQC + 1] = Q.PAy;
        X[kSelQC + 2] = Q.PAz;
        X[kSelWQ] = pf * PQx;
        X[kSelWQ + 1] = pf * PQy;
        X[kSelWQ + 2] = pf * PQz;
        X[kSelOo2p] = B.oo2p;
        X[kSelOo2q] = Q.oo2p;
        X[kSelOo2pq] = 0.5 * oopq;
        X[kSelRhoP2] = B.oo2p * qf;
        X[kSelRhoQ2] = Q.oo2p * pf;
        X[kSelWa] = 2.0 * B.alpha;
        X[kSelWb] = 2.0 * B.beta;
        X[kSelWc] = 2.0 * Q.alpha;
      } else {   // no such primitive: every recurrence value and weight is zero
#pragma unroll
        for (int m = 0; m <= L; ++m) S[CP::FSLOT + m] = 0.0;
        for (int k = kSelPA; k < kSelAB; ++k) X[k] = 0.0;
        X[kSelWa] = X[kSelWb] = X[kSelWc] = 0.0;
      }
    }
    __syncthreads();
    const int* ls = CP::vrr_lstart();
    for (int lv = 0; lv < CP::NVLEV; ++lv) {
      coop_level_q<NT, kVrrTerms, QB, CP::NSLOT>(ls[lv], ls[lv + 1], CP::vrr_node(),
                                                 CP::vrr_term(), sc, slots);
      __syncthreads();
    }
    const unsigned short* ts = CP::tgt_slot();
    const unsigned char* tw = CP::tgt_w();
    for (int t = tid; t < QB * CP::NACC; t += NT) {
      const int q = t % QB, k = t / QB;
      slots[q][k] = fma(sc[q][tw[k]], slots[q][ts[k]], slots[q][k]);
    }
  }
  __syncthreads();
  // HRR of every set, each value contracted right after the level that made it
  double g[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = 0.0;
  const int myq = tid % QB;
  const int* hs = CP::hrr_lstart();
  const int* cs = CP::con_lstart();
  const unsigned long long* cw = CP::con_word();
  constexpr int NLOOP = CP::NHLEV + 1 > CP::NCLEV ? CP::NHLEV + 1 : CP::NCLEV;
  for (int lv = 0; lv < NLOOP; ++lv) {
    if (lv > 0 && lv <= CP::NHLEV) {
      coop_level_q<NT, kHrrTerms, QB, CP::NSLOT>(hs[lv - 1], hs[lv], CP::hrr_node(),
                                                 CP::hrr_term(), sc, slots);
      __syncthreads();
    }
    if (lv < CP::NCLEV)
      for (int c = cs[lv] + tid / QB; c < cs[lv + 1]; c += NT / QB) {
        const unsigned long long w = cw[c];
        const double v = ctab[(w >> 40) & 0xFFull] * G[myq][(w >> 16) & 0xFFFFull] *
                         slots[myq][w & 0xFFFFull];
        const int gk = (int)((w >> 32) & 0xFFull);
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] += (gk == k) ? v : 0.0;
      }
    __syncthreads();
  }
  // per quartet: across the lanes that share it, then across wavefronts
  const int lane = tid & (kWave - 1), wv = tid / kWave;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    for (int o = kWave / 2; o >= QB; o >>= 1) g[k] += __shfl_xor(g[k], o, kWave);
    if (lane < QB) red[wv][lane][k] = g[k];
  }
  __syncthreads();
  if (tid < QB && qv[tid]) {
    double t9[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      t9[k] = 0.0;
      for (int w = 0; w < NW; ++w) t9[k] += red[w][tid][k];
    }
    const ShellPair bra = a.pairs[qbid[tid]], ket = a.pairs[qkid[tid]];
    const int A = a.shells[bra.a].atom, B = a.shells[bra.b].atom, C = a.shells[ket.a].atom,
              D = a.shells[ket.b].atom;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * A + d], t9[d]);
      atomicAdd(&a.grad[3 * B + d], t9[3 + d]);
      atomicAdd(&a.grad[3 * C + d], t9[6 + d]);
      atomicAdd(&a.grad[3 * D + d], -(t9[d] + t9[3 + d] + t9[6 + d]));
    }
  }
}

}  // namespace bscf

namespace bscf {

// Schwarz bound of one pair per block: sqrt(max |(mn|mn)|) over the pair.
template <class CP>
__global__ __launch_bounds__(CP::NT) void coop_schwarz_kernel(SchwarzArgs a) {
  constexpr int NT = CP::NT, NW = NT / kWave;
  __shared__ double slots[CP::NSLOT];
  __shared__ double sc[kNumSel];
  __shared__ double red[NW];
  const int pid = a.pair_ids[blockIdx.x];
  const ShellPair pr = a.pairs[pid];
  const Shell sa = a.shells[pr.a], sb = a.shells[pr.b];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  coop_primitives<CP>(a.prims + pr.prim0, pr.nprim, a.prims + pr.prim0, pr.nprim, AB, AB,
                      a.boys64, sc, slots);
  coop_hrr<CP>(sc, slots);
  constexpr int NAB = ncart(CP::LA) * ncart(CP::LB);
  double m = 0.0;
  for (int d = threadIdx.x; d < NAB; d += NT) {
    const int e = d * NAB + d;
    m = fmax(m, fabs(slots[CP::out_slot()[e]] * CP::norm()[e]));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NW; ++w) m = fmax(m, red[w]);
    a.Q[pid] = sqrt(m);
  }
}

// Full tensor of one instance (test path): every canonical quartet writes its
// eight index permutations.
template <class CP>
__global__ __launch_bounds__(CP::NT) void coop_tensor_kernel(TensorArgs a) {
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
  coop_hrr<CP>(sc, slots);
  constexpr int NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  const long long n = a.n;
  for (int e = threadIdx.x; e < CP::NOUT; e += CP::NT) {
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
