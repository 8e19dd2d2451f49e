"""Ring-polymer (path-integral) molecular dynamics: the propagation the paper's
PIMD layer performs between force calls (Section 2: the replica layer updates
every replica's position and velocity from its BO force, then hands the new
configurations back to the electronic-structure layer).

TEST INFRASTRUCTURE (see the package docstring).  Plain NumPy, written from
the published definitions cited below; it shares no code with the HIP path.

The paper names its integrator only by citation (Shiga et al. 2001, unified
PIMD); the reading used here is normal-mode PIMD with the path-integral
Langevin equation thermostat, PILE-L (Ceriotti, Parrinello, Markland and
Manolopoulos, J. Chem. Phys. 133, 124104 (2010)):

* Ring polymer of P beads with physical masses m, each bead feeling V/P, and
  harmonic springs between neighbouring beads (cyclic),
      H = sum_j [ |p_j|^2 / 2m + V(q_j) / P + m w_P^2 |q_j - q_{j+1}|^2 / 2 ],
  w_P = sqrt(P) k_B T / hbar, sampled at temperature T (atomic units,
  hbar = 1).  The force on bead j is F_j / P, F_j = -grad V(q_j).
* Normal modes of the free ring polymer: the orthogonal matrix C
  (C[j, 0] = 1/sqrt(P); C[j, k] = sqrt(2/P) cos(2 pi j k / P) for
  1 <= k < P/2; C[j, P/2] = (-1)^j / sqrt(P) for even P;
  C[j, k] = sqrt(2/P) sin(2 pi j k / P) for P/2 < k < P), frequencies
  w_k = 2 w_P sin(k pi / P).
* One step of length dt, symmetric splitting O B A B O:
    O: in normal modes p~_k <- c1_k p~_k + sqrt(m k_B T) c2_k xi,
       c1 = exp(-gamma_k dt / 2), c2 = sqrt(1 - c1^2),
       gamma_0 = 1 / tau_0 (centroid), gamma_k = 2 lambda w_k (k > 0);
    B: p_j <- p_j + (dt / 2) F_j / P;
    A: exact free ring-polymer motion for dt in normal modes (rotation of
       (p~_k, m w_k q~_k) by w_k dt; the centroid drifts freely);
    forces at the new positions, then B and O again.
  Without the thermostat the O steps are skipped (NVE).
* Gaussian deviates xi come from the counter-based generator Philox4x32-10
  (Salmon, Moraes, Dror and Shaw, SC'11, "Parallel random numbers: as easy as
  1, 2, 3") and the Box-Muller transform (Box and Muller 1958).  Deviate
  number i of half-step h (h = 2 * step + 0 before the force, + 1 after) of a
  run with seed s uses counter (i // 2, h mod 2^32, h >> 32, 0x50494d44) and
  key (s mod 2^32, s >> 32); the 128-bit output gives two 53-bit uniforms
  u = ((w0 << 32 | w1) >> 11 + 0.5) 2^-53 and (w2, w3) likewise, and
  xi_{2m} = sqrt(-2 ln u1) cos(2 pi u2), xi_{2m+1} = sqrt(-2 ln u1) sin(2 pi u2).
  The deviates are laid out [mode k][atom][xyz].
"""

from __future__ import annotations

import math

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
COUNTER_TAG = 0x50494D44
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds: 4 x 32-bit counter, 2 x 32-bit key."""
    c = [int(v) & MASK32 for v in ctr]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for r in range(10):
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
    return c


def gaussians(seed: int, half_step: int, n: int) -> np.ndarray:
    """n standard normal deviates of one half-step (layout of the module doc)."""
    key = (seed & MASK32, (seed >> 32) & MASK32)
    out = np.empty(n + (n & 1))
    for m in range((n + 1) // 2):
        w = philox4x32_10((m, half_step & MASK32, (half_step >> 32) & MASK32, COUNTER_TAG), key)
        u1 = (((w[0] << 32) | w[1]) >> 11) * 2.0 ** -53 + 2.0 ** -54
        u2 = (((w[2] << 32) | w[3]) >> 11) * 2.0 ** -53 + 2.0 ** -54
        r = math.sqrt(-2.0 * math.log(u1))
        out[2 * m] = r * math.cos(2.0 * math.pi * u2)
        out[2 * m + 1] = r * math.sin(2.0 * math.pi * u2)
    return out[:n]


def normal_mode_matrix(P: int) -> np.ndarray:
    """C[j, k], orthogonal; q~ = C^T q (beads j, modes k)."""
    C = np.empty((P, P))
    for j in range(P):
        for k in range(P):
            if k == 0:
                C[j, k] = 1.0 / math.sqrt(P)
            elif 2 * k < P:
                C[j, k] = math.sqrt(2.0 / P) * math.cos(2.0 * math.pi * j * k / P)
            elif 2 * k == P:
                C[j, k] = (-1.0) ** j / math.sqrt(P)
            else:
                C[j, k] = math.sqrt(2.0 / P) * math.sin(2.0 * math.pi * j * k / P)
    return C


def omega_p(P: int, temperature: float, kb: float) -> float:
    return math.sqrt(P) * kb * temperature


def mode_frequencies(P: int, wp: float) -> np.ndarray:
    return np.array([2.0 * wp * math.sin(k * math.pi / P) for k in range(P)])


class PileL:
    """State (x, p [P, N, 3]) and the O B A B O step of the module doc."""

    def __init__(self, masses, x, p, temperature, dt, kb, thermostat=True, tau0=0.0,
                 lam=1.0, seed=0):
        self.m = np.asarray(masses, float)
        self.x = np.array(x, float)
        self.p = np.array(p, float)
        self.T, self.dt, self.kb = float(temperature), float(dt), float(kb)
        self.P = self.x.shape[0]
        self.C = normal_mode_matrix(self.P)
        self.wp = omega_p(self.P, self.T, self.kb)
        self.w = mode_frequencies(self.P, self.wp)
        self.thermostat = thermostat
        gam = 2.0 * lam * self.w
        gam[0] = 1.0 / tau0 if tau0 > 0 else 0.0
        self.c1 = np.exp(-gam * self.dt / 2.0)
        self.c2 = np.sqrt(1.0 - self.c1 ** 2)
        self.seed = int(seed)
        self.step_index = 0

    # bead <-> normal-mode coordinates, per atom and direction
    def to_modes(self, a):
        return np.einsum("jk,jad->kad", self.C, a)

    def to_beads(self, a):
        return np.einsum("jk,kad->jad", self.C, a)

    def O(self, half):
        if not self.thermostat:
            return
        pt = self.to_modes(self.p)
        xi = gaussians(self.seed, 2 * self.step_index + half, pt.size).reshape(pt.shape)
        sig = np.sqrt(self.m * self.kb * self.T)[None, :, None]
        pt = self.c1[:, None, None] * pt + sig * self.c2[:, None, None] * xi
        self.p = self.to_beads(pt)

    def B(self, forces):
        self.p = self.p + 0.5 * self.dt * np.asarray(forces, float) / self.P

    def A(self):
        qt, pt = self.to_modes(self.x), self.to_modes(self.p)
        m = self.m[None, :, None]
        for k in range(self.P):
            if k == 0 or self.w[k] == 0.0:
                qt[k] = qt[k] + self.dt * pt[k] / m[0]
                continue
            c, s, mw = math.cos(self.w[k] * self.dt), math.sin(self.w[k] * self.dt), m[0] * self.w[k]
            q0, p0 = qt[k].copy(), pt[k].copy()
            pt[k] = c * p0 - mw * s * q0
            qt[k] = c * q0 + s * p0 / mw
        self.x, self.p = self.to_beads(qt), self.to_beads(pt)

    def begin(self, forces):
        """O, B, A: the part of a step before the force call."""
        self.O(0)
        self.B(forces)
        self.A()

    def end(self, forces):
        """B, O at the forces of the new positions."""
        self.B(forces)
        self.O(1)
        self.step_index += 1

    # observables
    def kinetic(self):
        return float(np.sum(self.p ** 2 / (2.0 * self.m[None, :, None])))

    def spring(self):
        d = self.x - np.roll(self.x, -1, axis=0)
        return float(0.5 * self.wp ** 2 * np.sum(self.m[None, :, None] * d * d))

    def hamiltonian(self, potentials):
        """H of the module doc, with potentials V(q_j) of the current beads."""
        return self.kinetic() + self.spring() + float(np.sum(potentials)) / self.P
