// One-electron integrals (S, T, V) and their nuclear derivatives, plus the
// per-geometry primitive-pair setup.
//
// Overlap: one-dimensional Obara-Saika recurrences
//   S_{i+1,j} = X_PA S_ij + (i S_{i-1,j} + j S_{i,j-1}) / (2p),
//   S_{i,j+1} = X_PB S_ij + (i S_{i-1,j} + j S_{i,j-1}) / (2p),
//   S_00 = sqrt(pi/p) exp(-mu X_AB^2).
// Kinetic: -1/2 <a|d^2/dx^2|b> per direction from overlaps with the ket power
// shifted by -2, 0, +2.  Nuclear attraction: Obara-Saika two-index
// recurrence on [a|b]^(m) with [0|0]^(m) = 2 pi/p K_AB F_m(p |PC|^2).
// Centre derivatives: d/dA_i g_a = 2 alpha g_{a+1_i} - a_i g_{a-1_i}; the
// operator-centre derivative of V follows from translational invariance,
// d/dC = -(d/dA + d/dB).
#include "boys.h"
#include "common.h"
#include "kernels.h"

namespace bscf {

namespace {

__device__ __forceinline__ void comp(int l, int c, int& lx, int& ly, int& lz) {
  int n = 0;
  for (int x = l; x >= 0; --x)
    for (int y = l - x; y >= 0; --y) {
      if (n == c) { lx = x; ly = y; lz = l - x - y; return; }
      ++n;
    }
}

// index of tuple t among all tuples with |t| <= its shell, ordered by |t| then
// lexicographically
__device__ __forceinline__ int tidx(int lx, int ly, int lz) {
  const int l = lx + ly + lz;
  const int u = l - lx;
  return l * (l + 1) * (l + 2) / 6 + u * (u + 1) / 2 + (u - ly);
}

__device__ __forceinline__ double comp_factor(int lx, int ly, int lz) {
  // 1 / sqrt((2lx-1)!! (2ly-1)!! (2lz-1)!!)
  double d = 1.0;
  for (int k = 2 * lx - 1; k > 1; k -= 2) d *= k;
  for (int k = 2 * ly - 1; k > 1; k -= 2) d *= k;
  for (int k = 2 * lz - 1; k > 1; k -= 2) d *= k;
  return 1.0 / sqrt(d);
}

constexpr int kMaxL1 = 3;           // shell l after one raise
constexpr int kS1 = kMaxL1 + 4;     // 1-D overlap index range
constexpr int kTeam = 64;           // threads per block (one wavefront)

// A block handles one shell pair and all nuclei.  Its wavefront splits into
// NS sub-teams of TS = kTeam / NS threads; sub-team s takes nuclei s, s + NS,
// s + 2 NS, ... and fills its own nuclear-attraction table.  Larger tables
// (total angular momentum L of the recursion) get larger sub-teams.
__host__ __device__ constexpr int sub_teams(int L) { return L <= 2 ? 32 : (L == 3 ? 16 : (L <= 5 ? 4 : 2)); }

// 1-D overlap tables S[d][i][j], one direction per thread (threads 0..2).
__device__ void overlap_1d_dir(double a, double b, double Ad, double Bd, int imax, int jmax,
                               double (*S)[kS1]) {
  const double p = a + b, oo2p = 0.5 / p, mu = a * b / p;
  const double P = (a * Ad + b * Bd) / p;
  const double XPA = P - Ad, XPB = P - Bd, XAB = Ad - Bd;
  S[0][0] = sqrt(M_PI / p) * exp(-mu * XAB * XAB);
  for (int i = 0; i <= imax; ++i) {
    if (i > 0) S[i][0] = XPA * S[i - 1][0] + (i > 1 ? (i - 1) * oo2p * S[i - 2][0] : 0.0);
    for (int j = 1; j <= jmax; ++j)
      S[i][j] = XPB * S[i][j - 1] + oo2p * ((i > 0 ? i * S[i - 1][j - 1] : 0.0) +
                                            (j > 1 ? (j - 1) * S[i][j - 2] : 0.0));
  }
}

__device__ __forceinline__ double ov3(const double (*S)[kS1][kS1], const int* ta, const int* tb) {
  for (int d = 0; d < 3; ++d)
    if (ta[d] < 0 || tb[d] < 0) return 0.0;
  return S[0][ta[0]][tb[0]] * S[1][ta[1]][tb[1]] * S[2][ta[2]][tb[2]];
}

__device__ double kin3(const double (*S)[kS1][kS1], const int* ta, const int* tb, double b) {
  if (ta[0] < 0 || ta[1] < 0 || ta[2] < 0 || tb[0] < 0 || tb[1] < 0 || tb[2] < 0) return 0.0;
  double t = 0.0;
  for (int d = 0; d < 3; ++d) {
    const int j = tb[d];
    int tp[3] = {tb[0], tb[1], tb[2]}, tm[3] = {tb[0], tb[1], tb[2]};
    tp[d] += 2;
    tm[d] -= 2;
    t += 4.0 * b * b * ov3(S, ta, tp) - 2.0 * b * (2 * j + 1) * ov3(S, ta, tb) +
         (j > 1 ? j * (j - 1) * ov3(S, ta, tm) : 0.0);
  }
  return -0.5 * t;
}

__host__ __device__ constexpr int ntup(int l) { return (l + 1) * (l + 2) * (l + 3) / 6; }

// [a|1/r_C|b]^(m) for all tuples |a| <= TA, |b| <= TB (primitive, positive
// sign), in LDS: v[m][tidx(a)][tidx(b)].
template <int TA, int TB>
struct NucTab {
  double v[TA + TB + 1][ntup(TA)][ntup(TB)];
  double PA[3], PB[3], PC[3], oo2p;
};

// Entry k of recursion level tot (na + nb = tot, m <= L - tot), ordered by na,
// then the a and b components, then m.
template <int TA, int TB>
__device__ __forceinline__ bool nuc_entry(int tot, int k, int& na, int& nb, int& ca, int& cb,
                                          int& m) {
  constexpr int L = TA + TB;
  const int nm = L - tot + 1;
  for (na = (tot > TB ? tot - TB : 0); na <= (tot < TA ? tot : TA); ++na) {
    nb = tot - na;
    const int cnt = ncart(na) * ncart(nb) * nm;
    if (k < cnt) {
      m = k % nm;
      k /= nm;
      cb = k % ncart(nb);
      ca = k / ncart(nb);
      return true;
    }
    k -= cnt;
  }
  return false;
}

// The recursion steps of a table, decoded once per block.  Level tot (na + nb
// = tot) holds nuc_count(tot) entries; entry k of the table is one step
//   v[dst] = X_i v[s0] - PC_i v[s0 + S] + c1/(2p) (v[s1] - v[s1 + S])
//                                       + c2/(2p) (v[s2] - v[s2 + S]),
// X = PB (b raised, b > 0) or PA (a raised, b = 0), S the stride from m to
// m + 1, offsets flat in v[m][tidx(a)][tidx(b)].  Packed as two words:
// w0 = dst | s0 << 12 | i << 24 | (X = PB) << 26 | c1 << 27 | c2 << 29,
// w1 = s1 | s2 << 12.
template <int TA, int TB>
__host__ __device__ constexpr int nuc_count(int tot) {
  int c = 0;
  for (int na = (tot > TB ? tot - TB : 0); na <= (tot < TA ? tot : TA); ++na)
    c += ncart(na) * ncart(tot - na) * (TA + TB - tot + 1);
  return c;
}
template <int TA, int TB>
__host__ __device__ constexpr int nuc_start(int tot) {   // first entry of level tot >= 1
  int c = 0;
  for (int t = 1; t < tot; ++t) c += nuc_count<TA, TB>(t);
  return c;
}
template <int TA, int TB>
struct NucPlan {
  static constexpr int L = TA + TB;
  static constexpr int S = ntup(TA) * ntup(TB);
  static constexpr int total = nuc_start<TA, TB>(L + 1);
  static constexpr int slots = total > 0 ? total : 1;
};

template <int TA, int TB>
__device__ void nuc_plan(uint2* desc) {
  using Pl = NucPlan<TA, TB>;
  constexpr int NB = ntup(TB);
  for (int e = threadIdx.x; e < Pl::total; e += blockDim.x) {
    int tot = 1;
    while (e >= nuc_start<TA, TB>(tot + 1)) ++tot;
    int na, nb, ca, cb, m;
    nuc_entry<TA, TB>(tot, e - nuc_start<TA, TB>(tot), na, nb, ca, cb, m);
    int ta[3], tb[3];
    comp(na, ca, ta[0], ta[1], ta[2]);
    comp(nb, cb, tb[0], tb[1], tb[2]);
    const int ia = tidx(ta[0], ta[1], ta[2]), ib = tidx(tb[0], tb[1], tb[2]);
    auto flat = [&](int x, int y) { return (unsigned)(m * Pl::S + x * NB + y); };
    unsigned dst = flat(ia, ib), s0, s1 = 0, s2 = 0, c1 = 0, c2 = 0, i, bside;
    if (nb > 0) {
      bside = 1;
      i = tb[0] > 0 ? 0 : (tb[1] > 0 ? 1 : 2);
      int b1[3] = {tb[0], tb[1], tb[2]};
      b1[i] -= 1;
      const int j1 = tidx(b1[0], b1[1], b1[2]);
      s0 = flat(ia, j1);
      if (ta[i] > 0) {
        int a1[3] = {ta[0], ta[1], ta[2]};
        a1[i] -= 1;
        s1 = flat(tidx(a1[0], a1[1], a1[2]), j1);
        c1 = ta[i];
      }
      if (b1[i] > 0) {
        int b2[3] = {b1[0], b1[1], b1[2]};
        b2[i] -= 1;
        s2 = flat(ia, tidx(b2[0], b2[1], b2[2]));
        c2 = b1[i];
      }
    } else {
      bside = 0;
      i = ta[0] > 0 ? 0 : (ta[1] > 0 ? 1 : 2);
      int a1[3] = {ta[0], ta[1], ta[2]};
      a1[i] -= 1;
      s0 = flat(tidx(a1[0], a1[1], a1[2]), ib);
      if (a1[i] > 0) {
        int a2[3] = {a1[0], a1[1], a1[2]};
        a2[i] -= 1;
        s2 = flat(tidx(a2[0], a2[1], a2[2]), ib);
        c2 = a1[i];
      }
    }
    desc[e] = make_uint2(dst | s0 << 12 | i << 24 | bside << 26 | c1 << 27 | c2 << 29, s1 | s2 << 12);
  }
  __syncthreads();
}

// Fill one sub-team's table (lt: thread index within the sub-team of TS):
// its first thread sets the Boys values and scalars, then each level of total
// angular momentum is spread over the sub-team by the decoded steps.  Every
// thread of the block calls this together (the level barriers are block-wide).
template <int TA, int TB, int TS>
__device__ void nuc_table(double a, double b, const double* A, const double* B, const double* C,
                          const double* boys64, int lt, const uint2* desc, NucTab<TA, TB>& t) {
  using Pl = NucPlan<TA, TB>;
  constexpr int L = TA + TB;
  if (lt == 0) {
    const double p = a + b, mu = a * b / p;
    double AB2 = 0.0, PC2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double P = (a * A[d] + b * B[d]) / p;
      t.PA[d] = P - A[d];
      t.PB[d] = P - B[d];
      t.PC[d] = P - C[d];
      AB2 += (A[d] - B[d]) * (A[d] - B[d]);
      PC2 += t.PC[d] * t.PC[d];
    }
    t.oo2p = 0.5 / p;
    double F[L + 1];
    boys_f64<L>(p * PC2, 2.0 * M_PI / p * exp(-mu * AB2), boys64, F);
    for (int m = 0; m <= L; ++m) t.v[m][0][0] = F[m];
  }
  __syncthreads();
  const double oo2p = t.oo2p;
  double* v = &t.v[0][0][0];
#pragma unroll
  for (int tot = 1; tot <= L; ++tot) {
    const int first = nuc_start<TA, TB>(tot), cnt = nuc_count<TA, TB>(tot);
    for (int k = lt; k < cnt; k += TS) {
      const uint2 d = desc[first + k];
      const unsigned dst = d.x & 4095u, s0 = (d.x >> 12) & 4095u, i = (d.x >> 24) & 3u;
      const unsigned c1 = (d.x >> 27) & 3u, c2 = (d.x >> 29) & 3u;
      const double X = (d.x >> 26) & 1u ? t.PB[i] : t.PA[i];
      double r = X * v[s0] - t.PC[i] * v[s0 + Pl::S];
      if (c1) {
        const unsigned s1 = d.y & 4095u;
        r += c1 * oo2p * (v[s1] - v[s1 + Pl::S]);
      }
      if (c2) {
        const unsigned s2 = (d.y >> 12) & 4095u;
        r += c2 * oo2p * (v[s2] - v[s2 + Pl::S]);
      }
      v[dst] = r;
    }
    __syncthreads();
  }
}

template <int TA, int TB>
__device__ __forceinline__ double nuc_get(const NucTab<TA, TB>& t, const int* ta, const int* tb) {
  for (int d = 0; d < 3; ++d)
    if (ta[d] < 0 || tb[d] < 0) return 0.0;
  if (ta[0] + ta[1] + ta[2] > TA || tb[0] + tb[1] + tb[2] > TB) return 0.0;
  return t.v[0][tidx(ta[0], ta[1], ta[2])][tidx(tb[0], tb[1], tb[2])];
}

}  // namespace

// ---------------------------------------------------------------------------
// Primitive-pair data: one thread per primitive pair.
__global__ void prim_pair_kernel(PrimPairSetupArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nprim) return;
  const int pid = a.prim_pair_owner[t];
  const ShellPair sp = a.pairs[pid];
  const int k = t - sp.prim0;
  const Shell sa = a.shells[sp.a], sb = a.shells[sp.b];
  const int ka = k / sb.nprim, kb = k % sb.nprim;
  const double al = a.sh_exp[sa.prim0 + ka], be = a.sh_exp[sb.prim0 + kb];
  const double ca = a.sh_coef[sa.prim0 + ka], cb = a.sh_coef[sb.prim0 + kb];
  const double p = al + be;
  const double Px = (al * sa.x + be * sb.x) / p, Py = (al * sa.y + be * sb.y) / p,
               Pz = (al * sa.z + be * sb.z) / p;
  const double dx = sa.x - sb.x, dy = sa.y - sb.y, dz = sa.z - sb.z;
  const double K = exp(-al * be / p * (dx * dx + dy * dy + dz * dz));
  PrimPair o;
  o.p = p;
  o.Px = Px; o.Py = Py; o.Pz = Pz;
  o.PAx = Px - sa.x; o.PAy = Py - sa.y; o.PAz = Pz - sa.z;
  // sqrt(2) * pi^(5/4)
  o.C = 5.9149671727956128778 * ca * cb * K / p;
  o.oo2p = 0.5 / p;
  o.alpha = al;
  o.beta = be;
  o.pad = 0.0;
  a.prims[t] = o;
}

// ---------------------------------------------------------------------------
// S, T, V: one 64-thread block per shell pair a >= b of one instance.  The
// nuclei are taken in groups of NS, one per sub-team; within a sub-team the
// threads own component pairs of the shell block (strided by TS).  S and T
// (no nucleus) come from thread e = component pair e in the first group; the
// sub-teams' V partial sums meet in LDS at the end, so every element is
// written once, without atomics.  Output is the normalised-component basis.
template <int LA, int LB>
__global__ __launch_bounds__(kTeam) void onee_kernel(OneEArgs a) {
  constexpr int NS = sub_teams(LA + LB), TS = kTeam / NS;
  constexpr int NA = ncart(LA), NB = ncart(LB), NE = (NA * NB + TS - 1) / TS;
  __shared__ NucTab<LA, LB> nt[NS];
  __shared__ uint2 desc[NucPlan<LA, LB>::slots];
  __shared__ double S1[3][kS1][kS1];
  __shared__ double red[NS][NA * NB];
  const int sh_a = a.task_a[blockIdx.x], sh_b = a.task_b[blockIdx.x];
  const Shell sa = a.shells[sh_a], sb = a.shells[sh_b];
  const int inst = sa.inst;
  const int n = a.nbf[inst], natoms = a.natoms[inst];
  const long long mo = a.moff[inst];
  const double A[3] = {sa.x, sa.y, sa.z}, B[3] = {sb.x, sb.y, sb.z};
  const int s = threadIdx.x / TS, lt = threadIdx.x % TS;
  nuc_plan<LA, LB>(desc);
  int ta[NE][3], tb[NE][3];
  bool own[NE];
  double Vv[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = lt + q * TS;
    own[q] = e < NA * NB;
    ta[q][0] = ta[q][1] = ta[q][2] = tb[q][0] = tb[q][1] = tb[q][2] = 0;
    if (own[q]) {
      comp(LA, e / NB, ta[q][0], ta[q][1], ta[q][2]);
      comp(LB, e % NB, tb[q][0], tb[q][1], tb[q][2]);
    }
    Vv[q] = 0.0;
  }
  // component pair of this thread for S and T
  const int es = threadIdx.x;
  const bool own_st = es < NA * NB;
  int xa[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
  if (own_st) {
    comp(LA, es / NB, xa[0], xa[1], xa[2]);
    comp(LB, es % NB, xb[0], xb[1], xb[2]);
  }
  double Sv = 0.0, Tv = 0.0;
  for (int c0 = 0; c0 < natoms; c0 += NS) {
    const int cidx = c0 + s;
    const bool live = cidx < natoms;   // idle sub-teams run the barriers with Z = 0
    const int atom = a.atom_off[inst] + (live ? cidx : 0);
    const double Cc[3] = {a.atom_xyz[3 * atom], a.atom_xyz[3 * atom + 1], a.atom_xyz[3 * atom + 2]};
    const double Zc = live ? a.atom_Z[atom] : 0.0;
    for (int ka = 0; ka < sa.nprim; ++ka)
      for (int kb = 0; kb < sb.nprim; ++kb) {
        const double al = a.sh_exp[sa.prim0 + ka], be = a.sh_exp[sb.prim0 + kb];
        const double cc = a.sh_coef[sa.prim0 + ka] * a.sh_coef[sb.prim0 + kb];
        __syncthreads();   // previous primitive's tables read
        if (c0 == 0 && threadIdx.x < 3)
          overlap_1d_dir(al, be, A[threadIdx.x], B[threadIdx.x], LA, LB + 2, S1[threadIdx.x]);
        nuc_table<LA, LB, TS>(al, be, A, B, Cc, a.boys64, lt, desc, nt[s]);   // ends with a barrier
#pragma unroll
        for (int q = 0; q < NE; ++q)
          if (own[q]) Vv[q] -= Zc * cc * nuc_get(nt[s], ta[q], tb[q]);
        if (c0 == 0 && own_st) {
          Sv += cc * ov3(S1, xa, xb);
          Tv += cc * kin3(S1, xa, xb, be);
        }
      }
  }
#pragma unroll
  for (int q = 0; q < NE; ++q)
    if (own[q]) red[s][lt + q * TS] = Vv[q];
  __syncthreads();
  if (own_st) {
    double v = 0.0;
    for (int k = 0; k < NS; ++k) v += red[k][es];
    const double f = comp_factor(xa[0], xa[1], xa[2]) * comp_factor(xb[0], xb[1], xb[2]);
    const long long ij = mo + (long long)(sa.bf + es / NB) * n + sb.bf + es % NB;
    const long long ji = mo + (long long)(sb.bf + es % NB) * n + sa.bf + es / NB;
    a.V[ij] = f * v;
    a.S[ij] = f * Sv;
    a.T[ij] = f * Tv;
    if (sh_a != sh_b) {   // a diagonal block's elements each have their own thread
      a.V[ji] = f * v;
      a.S[ji] = f * Sv;
      a.T[ji] = f * Tv;
    }
  }
}

// ---------------------------------------------------------------------------
// One-electron gradient: sum P dH/dX - sum W dS/dX per atom; one 64-thread
// block per shell pair a >= b (off-diagonal pairs counted twice) with the
// nuclei in sub-team groups as above.  A sub-team reduces its operator-centre
// terms over its threads after each nucleus; the overlap and kinetic terms
// come from thread e = component pair e in the first group; the basis-centre
// terms are reduced over the wavefront once at the end.
template <int LA, int LB>
__global__ __launch_bounds__(kTeam) void grad1e_kernel(Grad1EArgs a) {
  constexpr int NS = sub_teams(LA + LB + 2), TS = kTeam / NS;
  constexpr int NA = ncart(LA), NB = ncart(LB), NE = (NA * NB + TS - 1) / TS;
  __shared__ NucTab<LA + 1, LB + 1> nt[NS];
  __shared__ uint2 desc[NucPlan<LA + 1, LB + 1>::slots];
  __shared__ double S1[3][kS1][kS1];
  const int sh_a = a.task_a[blockIdx.x], sh_b = a.task_b[blockIdx.x];
  const Shell sa = a.shells[sh_a], sb = a.shells[sh_b];
  const int inst = sa.inst;
  if (!a.active[inst]) return;
  const int n = a.nbf[inst], natoms = a.natoms[inst];
  const long long mo = a.moff[inst];
  const double A[3] = {sa.x, sa.y, sa.z}, B[3] = {sb.x, sb.y, sb.z};
  const double sym = (sh_a == sh_b) ? 1.0 : 2.0;
  const int s = threadIdx.x / TS, lt = threadIdx.x % TS;
  nuc_plan<LA + 1, LB + 1>(desc);
  auto load_pw = [&](int e, int* xa, int* xb, double& pe, double& we) {
    comp(LA, e / NB, xa[0], xa[1], xa[2]);
    comp(LB, e % NB, xb[0], xb[1], xb[2]);
    const double f = comp_factor(xa[0], xa[1], xa[2]) * comp_factor(xb[0], xb[1], xb[2]);
    const long long ij = mo + (long long)(sa.bf + e / NB) * n + sb.bf + e % NB;
    pe = sym * f * a.P[ij];
    we = sym * f * a.W[ij];
  };
  int ta[NE][3], tb[NE][3];
  bool own[NE];
  double pij[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = lt + q * TS;
    own[q] = e < NA * NB;
    ta[q][0] = ta[q][1] = ta[q][2] = tb[q][0] = tb[q][1] = tb[q][2] = 0;
    pij[q] = 0.0;
    double w_unused;
    if (own[q]) load_pw(e, ta[q], tb[q], pij[q], w_unused);
  }
  // component pair of this thread for the overlap and kinetic terms
  const bool own_st = threadIdx.x < NA * NB;
  int xa[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
  double pst = 0.0, wst = 0.0;
  if (own_st) load_pw(threadIdx.x, xa, xb, pst, wst);
  double gab[6] = {0, 0, 0, 0, 0, 0};   // A, B
  for (int c0 = 0; c0 < natoms; c0 += NS) {
    const int cidx = c0 + s;
    const bool live = cidx < natoms;   // idle sub-teams run the barriers with Z = 0
    const int atom = a.atom_off[inst] + (live ? cidx : 0);
    const double Cc[3] = {a.atom_xyz[3 * atom], a.atom_xyz[3 * atom + 1], a.atom_xyz[3 * atom + 2]};
    const double Zc = live ? a.atom_Z[atom] : 0.0;
    double gc[3] = {0, 0, 0};
    for (int ka = 0; ka < sa.nprim; ++ka)
      for (int kb = 0; kb < sb.nprim; ++kb) {
        const double al = a.sh_exp[sa.prim0 + ka], be = a.sh_exp[sb.prim0 + kb];
        const double cc = a.sh_coef[sa.prim0 + ka] * a.sh_coef[sb.prim0 + kb];
        __syncthreads();
        if (c0 == 0 && threadIdx.x < 3)
          overlap_1d_dir(al, be, A[threadIdx.x], B[threadIdx.x], LA + 1, LB + 3, S1[threadIdx.x]);
        nuc_table<LA + 1, LB + 1, TS>(al, be, A, B, Cc, a.boys64, lt, desc, nt[s]);
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          if (!own[q]) continue;
          for (int d = 0; d < 3; ++d) {
            int up[3] = {ta[q][0], ta[q][1], ta[q][2]}, dn[3] = {ta[q][0], ta[q][1], ta[q][2]};
            up[d] += 1;
            dn[d] -= 1;
            int upb[3] = {tb[q][0], tb[q][1], tb[q][2]}, dnb[3] = {tb[q][0], tb[q][1], tb[q][2]};
            upb[d] += 1;
            dnb[d] -= 1;
            // nuclear attraction of this nucleus, basis-centre derivatives
            const double vA = -Zc * (2 * al * nuc_get(nt[s], up, tb[q]) - ta[q][d] * nuc_get(nt[s], dn, tb[q]));
            const double vB = -Zc * (2 * be * nuc_get(nt[s], ta[q], upb) - tb[q][d] * nuc_get(nt[s], ta[q], dnb));
            gab[d] += cc * pij[q] * vA;
            gab[3 + d] += cc * pij[q] * vB;
            gc[d] -= cc * pij[q] * (vA + vB);
          }
        }
        if (c0 == 0 && own_st)
          for (int d = 0; d < 3; ++d) {
            int up[3] = {xa[0], xa[1], xa[2]}, dn[3] = {xa[0], xa[1], xa[2]};
            up[d] += 1;
            dn[d] -= 1;
            int upb[3] = {xb[0], xb[1], xb[2]}, dnb[3] = {xb[0], xb[1], xb[2]};
            upb[d] += 1;
            dnb[d] -= 1;
            const double sA = 2 * al * ov3(S1, up, xb) - xa[d] * ov3(S1, dn, xb);
            const double sB = 2 * be * ov3(S1, xa, upb) - xb[d] * ov3(S1, xa, dnb);
            const double kA = 2 * al * kin3(S1, up, xb, be) - xa[d] * kin3(S1, dn, xb, be);
            const double kB = 2 * be * kin3(S1, xa, upb, be) - xb[d] * kin3(S1, xa, dnb, be);
            gab[d] += cc * (pst * kA - wst * sA);
            gab[3 + d] += cc * (pst * kB - wst * sB);
          }
      }
    // operator-centre terms of this sub-team's nucleus (lanes of a sub-team
    // are contiguous and aligned, so the xor butterfly stays inside it)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      for (int o = TS / 2; o > 0; o >>= 1) gc[d] += __shfl_xor(gc[d], o, kTeam);
    if (live && lt == 0)
      for (int d = 0; d < 3; ++d) atomicAdd(&a.grad[3 * atom + d], gc[d]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int o = 32; o > 0; o >>= 1) gab[k] += __shfl_xor(gab[k], o, kTeam);
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) {
      atomicAdd(&a.grad[3 * sa.atom + d], gab[d]);
      atomicAdd(&a.grad[3 * sb.atom + d], gab[3 + d]);
    }
}

void launch_onee(int la, int lb, const OneEArgs& a, hipStream_t s) {
  if (a.ntasks == 0) return;
  const dim3 g(a.ntasks), b(kTeam);
#define BSCF_ONEE(X, Y) \
  if (la == X && lb == Y) { hipLaunchKernelGGL((onee_kernel<X, Y>), g, b, 0, s, a); return; }
  BSCF_ONEE(0, 0) BSCF_ONEE(1, 0) BSCF_ONEE(1, 1) BSCF_ONEE(2, 0) BSCF_ONEE(2, 1) BSCF_ONEE(2, 2)
#undef BSCF_ONEE
}

void launch_grad1e(int la, int lb, const Grad1EArgs& a, hipStream_t s) {
  if (a.ntasks == 0) return;
  const dim3 g(a.ntasks), b(kTeam);
#define BSCF_G1(X, Y) \
  if (la == X && lb == Y) { hipLaunchKernelGGL((grad1e_kernel<X, Y>), g, b, 0, s, a); return; }
  BSCF_G1(0, 0) BSCF_G1(1, 0) BSCF_G1(1, 1) BSCF_G1(2, 0) BSCF_G1(2, 1) BSCF_G1(2, 2)
#undef BSCF_G1
}

namespace {
template <int M>
__device__ void boys_eval_one(double T, int fp32, const double* t64, const float* t32, double* o) {
  if (fp32) {
    float F[M + 1];
    boys_f32<M>(T, 1.0, t32, F);
    for (int m = 0; m <= M; ++m) o[m] = F[m];
  } else {
    double F[M + 1];
    boys_f64<M>(T, 1.0, t64, F);
    for (int m = 0; m <= M; ++m) o[m] = F[m];
  }
}
__global__ void boys_eval_kernel(int m_max, int n, const double* T, double* out, int fp32,
                                 const double* t64, const float* t32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* o = out + (long long)i * (m_max + 1);
  switch (m_max) {
    case 0: boys_eval_one<0>(T[i], fp32, t64, t32, o); break;
    case 1: boys_eval_one<1>(T[i], fp32, t64, t32, o); break;
    case 2: boys_eval_one<2>(T[i], fp32, t64, t32, o); break;
    case 3: boys_eval_one<3>(T[i], fp32, t64, t32, o); break;
    case 4: boys_eval_one<4>(T[i], fp32, t64, t32, o); break;
    case 5: boys_eval_one<5>(T[i], fp32, t64, t32, o); break;
    case 6: boys_eval_one<6>(T[i], fp32, t64, t32, o); break;
    case 7: boys_eval_one<7>(T[i], fp32, t64, t32, o); break;
    case 8: boys_eval_one<8>(T[i], fp32, t64, t32, o); break;
    case 9: boys_eval_one<9>(T[i], fp32, t64, t32, o); break;
    case 10: boys_eval_one<10>(T[i], fp32, t64, t32, o); break;
    case 11: boys_eval_one<11>(T[i], fp32, t64, t32, o); break;
    default: boys_eval_one<12>(T[i], fp32, t64, t32, o); break;
  }
}
}  // namespace

void launch_boys_eval(int m_max, int n, const double* T, double* out, int fp32,
                      const double* tab64, const float* tab32, hipStream_t s) {
  hipLaunchKernelGGL(boys_eval_kernel, dim3((n + 127) / 128), dim3(128), 0, s, m_max, n, T, out,
                     fp32, tab64, tab32);
}

void launch_prim_pairs(const PrimPairSetupArgs& a, hipStream_t s) {
  if (a.nprim == 0) return;
  hipLaunchKernelGGL(prim_pair_kernel, dim3((a.nprim + 255) / 256), dim3(256), 0, s, a);
}

}  // namespace bscf
