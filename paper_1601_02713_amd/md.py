"""Ring-polymer molecular dynamics driver around the batched energy/force
engine: the path-integral propagation the paper's PIMD layer runs between
force calls (Section 2), with the SCF guess chosen per step.

The integrator runs on the device (bscf_pimd_*: normal-mode PIMD with the
PILE-L thermostat, or NVE): every step moves all beads, sets the engine's
geometry from the new positions, runs the SCF of every bead and computes the
forces for the next step, without the ring polymer's state leaving the GPU
except for the positions the work lists need.  Convention: physical masses,
bead potential V/P, w_P = sqrt(P) k_B T / hbar, sampling at T.
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
    step_ms: float                 # integrator + geometry + SCF + forces of this step
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


def _with_guess(base, guess):
    o = beadscf.default_opts()
    for name, _ in beadscf.ScfOpts._fields_:
        setattr(o, name, getattr(base, name))
    o.guess = guess
    return o


def run(engine: beadscf.Engine, poly: RingPolymer, n_steps: int, dt_fs: float, guess: str = "previous",
        train_from: int = 1, train_steps: int = 5, predict_from: int = 3, opts=None,
        geometries=None, basis=None, log=None, thermostat: bool = True, tau_centroid_fs: float = 100.0,
        seed: int = 0):
    """Propagate n_steps (step 0 is the starting configuration); returns the
    per-step records and the geometries.

    guess: "core" (every step from the core Hamiltonian), "previous" (the
    previous step's orbitals, re-orthonormalised; the paper's reuse) or
    "learned" (previous-step guess corrected by the in-run network, trained
    after every step from step train_from on and applied from step
    predict_from on).  With geometries given the positions are replayed
    instead of integrated (same trajectory for guess or precision
    comparisons).  basis (a basis-set dict) is loaded first when given."""
    if basis is not None:
        engine.load_basis(basis)
    P = poly.n_beads
    engine.set_instances([poly.Z] * P)
    mode = {"core": beadscf.GUESS_CORE, "previous": beadscf.GUESS_PREVIOUS,
            "learned": beadscf.GUESS_LEARNED}[guess]
    base = opts or beadscf.default_opts()
    integrate = geometries is None
    engine.set_geometries(list(poly.x if integrate else geometries[0]))
    if integrate:
        engine.pimd_init(poly.masses, poly.v * poly.masses[None, :, None],
                         beadscf.pimd_default_opts(dt=dt_fs * FS, temperature=poly.temperature,
                                                   thermostat=1 if thermostat else 0,
                                                   tau_centroid=tau_centroid_fs * FS, seed=seed))
    records, traj = [], []
    for step in range(n_steps):
        g = mode
        if step == 0 or (mode == beadscf.GUESS_LEARNED and step < predict_from):
            g = beadscf.GUESS_CORE if step == 0 else beadscf.GUESS_PREVIOUS
        o = _with_guess(base, g)
        t0 = time.perf_counter()
        if step == 0:
            E, it, st = engine.run_scf(o)
            engine.forces()
        elif integrate:
            E, it, st = engine.pimd_step(o)
        else:
            engine.set_geometries(list(geometries[step]))
            E, it, st = engine.run_scf(o)
            engine.forces()
        rec = StepRecord(step, E, it, st, (time.perf_counter() - t0) * 1e3)
        traj.append(engine.pimd_state()[0] if integrate else np.array(geometries[step]))
        if mode == beadscf.GUESS_LEARNED and step >= train_from:
            t3 = time.perf_counter()
            rec.train_loss = engine.guess_train(train_steps)
            rec.train_ms = (time.perf_counter() - t3) * 1e3
        records.append(rec)
        if log is not None:
            log(rec)
    if integrate:
        poly.x = traj[-1].copy()
        poly.v = engine.pimd_state()[1] / poly.masses[None, :, None]
    return records, traj
