"""Ring-polymer molecular dynamics driver around the batched energy/force
engine: the primitive path-integral propagation the paper's PIMD layer runs
between force calls (Section 2), with the SCF guess chosen per step.

Hamiltonian of P beads with physical masses m (atomic units):
  H = sum_k [ p_k^2 / 2m + m w_P^2 |x_k - x_(k+1)|^2 / 2 + V(x_k) / P ],
  w_P = sqrt(P) k_B T / hbar, beads cyclic;
integrated with velocity Verlet in the NVE ensemble.  The force evaluation
(every bead's SCF and analytic gradient) is the engine's; the integrator
itself is a few vector operations on the host.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import beadscf

KB = 3.166811563e-6            # Eh / K
AMU = 1822.888486209           # electron masses per unified atomic mass unit
FS = 41.341373336              # atomic time units per femtosecond
MASS_AMU = {1: 1.008, 6: 12.011, 7: 14.007, 8: 15.999}


@dataclass
class StepRecord:
    step: int
    energies: np.ndarray
    iterations: np.ndarray
    status: np.ndarray
    scf_ms: float
    force_ms: float
    train_ms: float = 0.0
    train_loss: float | None = None


@dataclass
class RingPolymer:
    """P beads of one system: positions and velocities [P, atoms, 3] (bohr,
    bohr per atomic time unit)."""
    Z: np.ndarray
    x: np.ndarray
    v: np.ndarray
    temperature: float
    masses: np.ndarray = field(init=False)

    def __post_init__(self):
        self.masses = np.array([MASS_AMU[int(z)] for z in self.Z]) * AMU

    @property
    def n_beads(self):
        return self.x.shape[0]

    def spring_forces(self):
        P = self.n_beads
        if P == 1:
            return np.zeros_like(self.x)
        wp = np.sqrt(P) * KB * self.temperature
        lap = 2.0 * self.x - np.roll(self.x, 1, axis=0) - np.roll(self.x, -1, axis=0)
        return -(self.masses[None, :, None] * wp * wp) * lap


def run(engine: beadscf.Engine, poly: RingPolymer, n_steps: int, dt_fs: float, guess: str = "previous",
        train_from: int = 1, train_steps: int = 5, predict_from: int = 3, opts=None,
        geometries=None, basis=None, log=None):
    """Propagate n_steps; returns the per-step records and the geometries.

    guess: "core" (every step from the core Hamiltonian), "previous" (the
    previous step's orbitals, re-orthonormalised; the paper's reuse) or
    "learned" (previous-step guess corrected by the in-run network, trained
    after every step from step train_from on and applied from step
    predict_from on).  With geometries given the positions are replayed
    instead of integrated (same trajectory for guess comparisons).  basis (a
    basis-set dict) is loaded first when given."""
    dt = dt_fs * FS
    if basis is not None:
        engine.load_basis(basis)
    P = poly.n_beads
    Zs = [poly.Z] * P
    engine.set_instances(Zs)
    mode = {"core": beadscf.GUESS_CORE, "previous": beadscf.GUESS_PREVIOUS,
            "learned": beadscf.GUESS_LEARNED}[guess]
    base = opts or beadscf.default_opts()
    records, traj = [], []
    for step in range(n_steps):
        if geometries is not None:
            poly.x = np.array(geometries[step])
        traj.append(poly.x.copy())
        engine.set_geometries(list(poly.x))
        g = mode
        if step == 0 or (mode == beadscf.GUESS_LEARNED and step < predict_from):
            g = beadscf.GUESS_CORE if step == 0 else beadscf.GUESS_PREVIOUS
        o = beadscf.default_opts()
        for name, _ in beadscf.ScfOpts._fields_:
            setattr(o, name, getattr(base, name))
        o.guess = g
        t0 = time.perf_counter()
        E, it, st = engine.run_scf(o)
        t1 = time.perf_counter()
        forces = np.array(engine.forces())        # -dE/dR per bead [P, atoms, 3]
        t2 = time.perf_counter()
        rec = StepRecord(step, E, it, st, (t1 - t0) * 1e3, (t2 - t1) * 1e3)
        if mode == beadscf.GUESS_LEARNED and step >= train_from:
            t3 = time.perf_counter()
            rec.train_loss = engine.guess_train(train_steps)
            rec.train_ms = (time.perf_counter() - t3) * 1e3
        records.append(rec)
        if log is not None:
            log(rec)
        if geometries is not None:
            continue
        # velocity Verlet: finish the previous step's kick with the new
        # acceleration, then kick and drift to the next positions
        acc = (forces / P + poly.spring_forces()) / poly.masses[None, :, None]
        if step > 0:
            poly.v = poly.v + 0.5 * dt * acc
        if step + 1 < n_steps:
            poly.v = poly.v + 0.5 * dt * acc
            poly.x = poly.x + dt * poly.v
    return records, traj
