// Two-electron gradient kernels over the screened work lists (grad_*.hip).
#pragma once
#include "common.h"

namespace bscf {

struct GradArgs {
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
  const PrimPair* kprims;  // ket primitive pairs in ket-list order (see FockArgs)
  const int2* kpos;
  int max_prims;
  const long long* moff;
  const int* nbf;
  const int* atom_off;     // first global atom of each instance
  int nmax;                // largest basis size
  int max_atoms;           // largest atom count of an instance
  int nk_total;            // stride of Pk
  const double* P;
  const double* Pk;        // P gathered by ket-list position (see FockArgs)
  double* grad;            // [total atoms][3], dE/dR accumulated
  const double* boys64;
  int unit_threads;        // threads of a lane-kernel unit: 64, 128 or 256
  // density-weighted screening of the cooperative kernels: a quartet is
  // skipped when Q_ab Q_cd (Pm_ab Pm_cd + (Pm_ac Pm_bd + Pm_ad Pm_bc) / 4) <
  // tau, with Pm the largest |P| of each shell-pair block (tau <= 0: none)
  const double* Q;         // Schwarz bound per shell pair
  const double* Pm;        // per instance [nsh][nsh] at pm_off
  const long long* pm_off;
  const int* shell_off;    // first global shell of each instance
  const int* nsh;          // shells per instance
  double tau;
  // share of exact exchange in the density factor: 1 for Hartree-Fock, 0.2
  // for B3LYP (the bound above stays an upper bound for kx <= 1)
  double kx;
  // with gstat: the class's evaluated (not skipped) quartets and primitive
  // quartets are added into gstat[0] and gstat[1]
  double* gstat;
};

// Density-weighted bound of quartet (bid|kid) (see GradArgs).
__device__ __forceinline__ double grad_quartet_bound(const GradArgs& a, int bid, int kid) {
  const ShellPair bra = a.pairs[bid], ket = a.pairs[kid];
  const int inst = a.shells[bra.a].inst;
  const int s0 = a.shell_off[inst], ns = a.nsh[inst];
  const double* M = a.Pm + a.pm_off[inst];
  const int i = bra.a - s0, j = bra.b - s0, k = ket.a - s0, l = ket.b - s0;
  const double g = M[i * ns + j] * M[k * ns + l] +
                   0.25 * (M[i * ns + k] * M[j * ns + l] + M[i * ns + l] * M[j * ns + k]);
  return a.Q[bid] * a.Q[kid] * g;
}

// LDS footprint of the gradient unit kernel: P rows of the bra shells, one
// dE/dR accumulator triple per atom of the instance and the bra's primitive
// pairs.
__host__ __device__ constexpr int grad_unit_lds_doubles(int la, int lb, int nmax, int max_atoms,
                                                        int max_prims) {
  return (ncart(la) + ncart(lb)) * nmax + 3 * max_atoms + 12 * max_prims;
}

using GradLauncher = void (*)(const GradArgs&, hipStream_t);
// grad_launcher(q) is defined in the generated classes.h

}  // namespace bscf
