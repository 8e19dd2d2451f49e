// Two-electron gradient launchers (placeholder: reports unsupported).
#include <stdexcept>

#include "grad.h"

namespace bscf {
static void grad_missing(const GradArgs&, hipStream_t) {
  throw std::runtime_error("two-electron gradient kernels are not built");
}
GradLauncher grad_launcher(int) { return grad_missing; }
}  // namespace bscf
