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
};

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
