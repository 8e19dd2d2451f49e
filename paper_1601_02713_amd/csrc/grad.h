// Two-electron gradient kernels over the screened work lists (grad_*.hip).
#pragma once
#include "common.h"

namespace bscf {

struct GradArgs {
  const WorkItem* items;
  int nitems;
  const WorkRow* rows;
  const ShellPair* pairs;
  const PrimPair* prims;
  const Shell* shells;
  const int* kets;
  const long long* moff;
  const int* nbf;
  const double* P;
  double* grad;            // [total atoms][3], dE/dR accumulated
  const double* boys64;
};

using GradLauncher = void (*)(const GradArgs&, hipStream_t);
// grad_launcher(q) is defined in the generated classes.h

}  // namespace bscf
