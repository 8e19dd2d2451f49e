// Ring-polymer (path-integral) integrator on the device: the position and
// momentum update of every replica between force calls (the serial replica
// update of the paper's PIMD layer, Section 2), in normal-mode coordinates
// with the PILE-L Langevin thermostat (Ceriotti, Parrinello, Markland and
// Manolopoulos 2010).
//
// Convention: P beads with physical masses, each feeling V/P, cyclic springs
// of frequency w_P = sqrt(P) k_B T / hbar, sampled at T (atomic units).  A
// step of length dt is O B A B O:
//   O  p~_k <- c1_k p~_k + sqrt(m k_B T) c2_k xi   (normal modes k; c1 =
//      exp(-gamma_k dt/2), c2 = sqrt(1 - c1^2), gamma_0 = 1/tau_0, gamma_k =
//      2 lambda w_k, w_k = 2 w_P sin(k pi / P)); skipped without thermostat;
//   B  p_j <- p_j + (dt/2) F_j / P  (F_j = -dV/dq_j of bead j);
//   A  exact free ring-polymer motion of every normal mode over dt.
// The Gaussian deviates xi come from Philox4x32-10 (Salmon et al. 2011) and
// the Box-Muller transform: deviate i = k * 3N + 3 * atom + xyz of half-step
// h (2 * step before the force call, 2 * step + 1 after) takes counter
// (i / 2, h mod 2^32, h / 2^32, 0x50494d44) and key (seed mod 2^32,
// seed / 2^32); words (w0, w1) and (w2, w3) give two 53-bit uniforms
// u = ((w_hi << 32 | w_lo) >> 11) 2^-53 + 2^-54, then r = sqrt(-2 ln u1),
// xi_even = r cos(2 pi u2), xi_odd = r sin(2 pi u2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bscf {

constexpr int kPimdMaxBeads = 64;   // one thread per bead / mode in a 64-lane block

struct PimdArgs {
  int P;                  // beads
  int ncol;               // 3 N (atom-major, xyz fastest)
  double dt;
  double* x;              // [P][ncol] positions (bohr)
  double* p;              // [P][ncol] momenta (m_e bohr / atomic time)
  const double* C;        // [P][P] normal-mode matrix C[j][k]
  const double* w;        // [P] mode frequencies
  const double* c1;       // [P] O-step decay per mode
  const double* c2;       // [P]
  const double* mass;     // [N] (m_e)
  const double* sig;      // [N] sqrt(m k_B T)
  uint64_t seed;
};

// O (if thermostat) then B on every column: forces F [P][ncol] with sign
// fsign (+1: forces, -1: a gradient dE/dq), half-step index h.  order 0: O
// then B (before the force call); order 1: B then O (after it).
void launch_pimd_ob(const PimdArgs& a, const double* F, double fsign, int thermostat, uint64_t h,
                    int order, hipStream_t s);
// A: exact free ring-polymer propagation over dt.
void launch_pimd_a(const PimdArgs& a, hipStream_t s);

}  // namespace bscf
