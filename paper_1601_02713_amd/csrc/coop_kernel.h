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

// Evaluate one level range [n0, n1) of a packed node table.
template <int NT>
__device__ __forceinline__ void coop_level(int n0, int n1,
                                           const unsigned long long* __restrict__ node,
                                           const unsigned int* __restrict__ term,
                                           const double* sc, double* slots) {
  for (int nd = n0 + (int)threadIdx.x; nd < n1; nd += NT) {
    const unsigned long long w = node[nd];
    const int t0 = (int)(w & 0xFFFFFFFFull);
    const int dst = (int)((w >> 32) & 0xFFFFull);
    const int t1 = t0 + (int)((w >> 48) & 0xFFull);
    double v = 0.0;
    for (int t = t0; t < t1; ++t) {
      const unsigned int u = term[t];
      const double m = (double)((int)(u >> 24) - 8);
      v = fma(m * sc[(u >> 16) & 0xFFu], slots[u & 0xFFFFu], v);
    }
    slots[dst] = v;
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
  constexpr int L = CP::L, NT = CP::NT;
  const int tid = threadIdx.x;
  for (int t = tid; t < CP::NACC; t += NT) slots[CP::acc_slot()[t]] = 0.0;
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
        coop_level<NT>(ls[lv], ls[lv + 1], CP::vrr_node(), CP::vrr_term(), sc, slots);
        __syncthreads();
      }
      for (int t = tid; t < CP::NACC; t += NT)
        slots[CP::acc_slot()[t]] = fma(sc[CP::tgt_w()[t]], slots[CP::tgt_slot()[t]],
                                       slots[CP::acc_slot()[t]]);
    }
  }
  __syncthreads();
}

// HRR levels of a quartet (Fock, Schwarz and tensor kernels).
template <class CP>
__device__ __forceinline__ void coop_hrr(const double* sc, double* slots) {
  const int* hs = CP::hrr_lstart();
  for (int lv = 0; lv < CP::NHLEV; ++lv) {
    coop_level<CP::NT>(hs[lv], hs[lv + 1], CP::hrr_node(), CP::hrr_term(), sc, slots);
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

template <class CP>
__global__ __launch_bounds__(CP::NT) void coop_grad_kernel(GradArgs a) {
  constexpr int NT = CP::NT, NW = NT / kWave;
  constexpr int NA = ncart(CP::LA), NB = ncart(CP::LB), NC = ncart(CP::LC), ND = ncart(CP::LD);
  constexpr int NOUT = NA * NB * NC * ND;
  __shared__ double slots[CP::NSLOT];
  __shared__ double G[NOUT];
  __shared__ double sc[kNumSel];
  __shared__ double ctab[CP::NCTAB];
  __shared__ double red[NW][9];
  int bid, kid;
  if (!coop_quartet(a.items, a.nitems, a.rows, a.kets, blockIdx.x, bid, kid)) return;
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const Shell sa = a.shells[bra.a], sb = a.shells[bra.b], sc_ = a.shells[ket.a],
              sd = a.shells[ket.b];
  const int inst = sa.inst;
  const long long mo = a.moff[inst];
  const int n = a.nbf[inst];
  const double* __restrict__ P = a.P + mo;
  const double deg = ((bra.a == bra.b) ? 1.0 : 2.0) * ((ket.a == ket.b) ? 1.0 : 2.0) *
                     ((kid == bid) ? 1.0 : 2.0);
  for (int e = threadIdx.x; e < NOUT; e += NT) {
    const int l = e % ND, k = (e / ND) % NC, j = (e / (ND * NC)) % NB, i = e / (ND * NC * NB);
    const int mu = sa.bf + i, nu = sb.bf + j, la = sc_.bf + k, si = sd.bf + l;
    G[e] = 0.5 * deg *
           (P[mu * n + nu] * P[la * n + si] -
            0.25 * (P[mu * n + la] * P[nu * n + si] + P[mu * n + si] * P[nu * n + la]));
  }
  for (int t = threadIdx.x; t < CP::NCTAB; t += NT) ctab[t] = CP::con_ctab()[t];
  const double AB[3] = {sa.x - sb.x, sa.y - sb.y, sa.z - sb.z};
  const double CD[3] = {sc_.x - sd.x, sc_.y - sd.y, sc_.z - sd.z};
  coop_primitives<CP>(a.prims + bra.prim0, bra.nprim, a.prims + ket.prim0, ket.nprim, AB, CD,
                      a.boys64, sc, slots);
  double g[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) g[k] = 0.0;
  const int* hs = CP::hrr_lstart();
  const int* cs = CP::con_lstart();
  const unsigned long long* cw = CP::con_word();
  constexpr int NLOOP = CP::NHLEV + 1 > CP::NCLEV ? CP::NHLEV + 1 : CP::NCLEV;
  for (int lv = 0; lv < NLOOP; ++lv) {
    if (lv > 0 && lv <= CP::NHLEV) {
      coop_level<NT>(hs[lv - 1], hs[lv], CP::hrr_node(), CP::hrr_term(), sc, slots);
      __syncthreads();
    }
    if (lv < CP::NCLEV)
      for (int c = cs[lv] + (int)threadIdx.x; c < cs[lv + 1]; c += NT) {
        const unsigned long long w = cw[c];
        const double v = ctab[(w >> 40) & 0xFFull] * G[(w >> 16) & 0xFFFFull] *
                         slots[w & 0xFFFFull];
        const int gk = (int)((w >> 32) & 0xFFull);
#pragma unroll
        for (int k = 0; k < 9; ++k) g[k] += (gk == k) ? v : 0.0;
      }
    __syncthreads();
  }
  // block reduction: across the wavefront, then across wavefronts
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    for (int o = 32; o > 0; o >>= 1) g[k] += __shfl_xor(g[k], o, kWave);
    if (lane == 0) red[wv][k] = g[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      t[k] = 0.0;
      for (int w = 0; w < NW; ++w) t[k] += red[w][k];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * sa.atom + d], t[d]);
      atomicAdd(&a.grad[3 * sb.atom + d], t[3 + d]);
      atomicAdd(&a.grad[3 * sc_.atom + d], t[6 + d]);
      atomicAdd(&a.grad[3 * sd.atom + d], -(t[d] + t[3 + d] + t[6 + d]));
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
