"""The device ring-polymer integrator (bscf_pimd_*) against the NumPy oracle
of oracle/pimd.py, which follows the same published scheme (normal-mode
PIMD with the PILE-L thermostat, Philox4x32-10 and Box-Muller deviates) in
code of its own.

* With caller forces of a harmonic well, 60 thermostatted steps of the
  device and of the oracle from the same state, seed and forces agree to
  rounding: the deviates, the normal-mode transforms, the O, B and A steps
  and the step counters all match.
* With this library's SCF forces (one water, 4 beads), three steps agree with
  the oracle integrator driven by the oracle's own SCF and gradient per bead.
* NVE with SCF forces conserves the ring-polymer Hamiltonian.
* The thermostat samples the exact kinetic energy of a harmonic ring polymer.
* Refusals: more than 64 beads, beads of different systems, a half-step
  without forces.
"""

import numpy as np
import pytest

import inputs
import oracle
from oracle import pimd as opimd

pytestmark = pytest.mark.gpu

KB = 3.166811563e-6
FS = 41.341373336
AMU = 1822.888486209
MASS = {1: 1.008 * AMU, 8: 15.999 * AMU}


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


def _water_beads(P, seed):
    z, x = inputs.workload("h2o_sto3g")["instances"][0]
    return z, inputs.beads(z, x, P, seed)


def test_harmonic_steps_match_oracle(beadscf, sto3g):
    P, T, dt = 6, 300.0, 0.5 * FS
    z, xb = _water_beads(P, 3)
    m = np.array([MASS[int(v)] for v in z])
    k = m * 0.02 ** 2
    x0c = xb.mean(axis=0)
    force = lambda x: -k[None, :, None] * (x - x0c[None])
    p0 = np.random.default_rng(4).standard_normal(xb.shape) * np.sqrt(m * KB * T)[None, :, None]
    e = beadscf.Engine(0)
    try:
        e.load_basis(sto3g)
        e.set_instances([z] * P)
        e.set_geometries(list(xb))
        opts = beadscf.pimd_default_opts(dt=dt, temperature=T, thermostat=1, tau_centroid=50 * FS,
                                         friction_scale=0.5, seed=0x1234567890AB)
        e.pimd_init(m, p0, opts)
        ref = opimd.PileL(m, xb, p0, T, dt, KB, thermostat=True, tau0=50 * FS, lam=0.5,
                          seed=0x1234567890AB)
        for s in range(60):
            xg = e.pimd_state()[0]
            e.pimd_begin(force(xg))
            ref.begin(force(ref.x))
            xg = e.pimd_state()[0]
            e.pimd_end(force(xg))
            ref.end(force(ref.x))
        x, p, ke, sp, steps = e.pimd_state()
        assert steps == 60
        assert np.abs(x - ref.x).max() < 1e-11 * np.abs(ref.x).max()
        assert np.abs(p - ref.p).max() < 1e-11 * np.abs(ref.p).max()
        assert abs(ke - ref.kinetic()) < 1e-11 * ref.kinetic()
        assert abs(sp - ref.spring()) < 1e-10 * ref.spring()
        # the context's own geometry is untouched by caller-force steps
        S, _ = e.one_electron(0)
        assert S.shape == (7, 7)
    finally:
        e.close()


def test_scf_driven_steps_match_oracle_integrator(beadscf, sto3g):
    """Water, STO-3G, 4 beads, 3 thermostatted steps of 0.5 fs: the device
    step (SCF of every bead, forces, integrator) against the oracle
    integrator whose forces come from the oracle's SCF and gradient."""
    P, T, dt = 4, 300.0, 0.5 * FS
    z, xb = _water_beads(P, 5)
    m = np.array([MASS[int(v)] for v in z])
    p0 = inputs.maxwell_boltzmann(z, P, T, 5) * m[None, :, None]
    e = beadscf.Engine(0)
    try:
        e.load_basis(sto3g)
        e.set_instances([z] * P)
        e.set_geometries(list(xb))
        opts = beadscf.pimd_default_opts(dt=dt, temperature=T, seed=99)
        e.pimd_init(m, p0, opts)
        so = beadscf.default_opts(e_tol=1e-12, comm_tol=1e-10, guess=beadscf.GUESS_PREVIOUS)
        Es = [e.pimd_step(so)[0] for _ in range(3)]
        x, p, _, _, steps = e.pimd_state()
    finally:
        e.close()
    assert steps == 3

    def forces(xx):
        out, en = [], []
        for j in range(P):
            b = oracle.build_basis(sto3g, z, xx[j])
            r = oracle.scf(b, 1e-12, 1e-10)
            out.append(-oracle.gradient(b, r["P"], r["F"]))
            en.append(r["E"])
        return np.array(out), np.array(en)

    ref = opimd.PileL(m, xb, p0, T, dt, KB, thermostat=True, tau0=opts.tau_centroid, lam=1.0, seed=99)
    F, _ = forces(ref.x)
    for s in range(3):
        ref.begin(F)
        F, En = forces(ref.x)
        ref.end(F)
        assert np.abs(Es[s] - En).max() < 1e-9, s
    assert np.abs(x - ref.x).max() < 1e-9
    assert np.abs(p - ref.p).max() < 1e-8 * np.abs(ref.p).max()


def test_nve_conserves_the_ring_polymer_hamiltonian(beadscf, sto3g):
    """NVE, water, STO-3G, 4 beads, 16 steps of 0.25 fs with SCF forces: the
    ring-polymer Hamiltonian (kinetic + spring + sum E_j / P) fluctuates by
    about 1e-3 of the kinetic energy scale (second order in dt; the oracle
    integrator with the oracle's forces gives the same sequence, compared
    step by step) and does not drift."""
    P, T, dt, n = 4, 300.0, 0.25 * FS, 16
    z, xb = _water_beads(P, 7)
    m = np.array([MASS[int(v)] for v in z])
    p0 = inputs.maxwell_boltzmann(z, P, T, 7) * m[None, :, None]
    e = beadscf.Engine(0)
    try:
        e.load_basis(sto3g)
        e.set_instances([z] * P)
        e.set_geometries(list(xb))
        e.pimd_init(m, p0, beadscf.pimd_default_opts(dt=dt, temperature=T, thermostat=0))
        so = beadscf.default_opts(e_tol=1e-12, comm_tol=1e-10, guess=beadscf.GUESS_PREVIOUS)
        H = []
        for _ in range(n):
            E, _, st = e.pimd_step(so)
            assert (st == 0).all()
            _, _, ke, sp, _ = e.pimd_state()
            H.append(ke + sp + E.sum() / P)
    finally:
        e.close()
    H = np.array(H)

    def forces(xx):
        out, en = [], []
        for j in range(P):
            b = oracle.build_basis(sto3g, z, xx[j])
            r = oracle.scf(b, 1e-12, 1e-10)
            out.append(-oracle.gradient(b, r["P"], r["F"]))
            en.append(r["E"])
        return np.array(out), np.array(en)

    ref = opimd.PileL(m, xb, p0, T, dt, KB, thermostat=False)
    F, _ = forces(ref.x)
    Hr = []
    for _ in range(n):
        ref.begin(F)
        F, En = forces(ref.x)
        ref.end(F)
        Hr.append(ref.hamiltonian(En))
    ke0 = 1.5 * P * len(z) * KB * T
    print("H fluctuation", np.ptp(H), "oracle", np.ptp(Hr), "kinetic scale", ke0)
    assert np.abs(H - np.array(Hr)).max() < 1e-9
    assert np.ptp(H) < 2.5e-3 * ke0
    assert abs(H[-4:].mean() - H[:4].mean()) < 2.5e-3 * ke0


def test_thermostat_kinetic_energy(beadscf, sto3g):
    P, T, dt = 8, 300.0, 0.5 * FS
    z, xb = _water_beads(P, 9)
    m = np.array([MASS[int(v)] for v in z])
    k = m * 0.01 ** 2
    x0 = xb.copy()
    e = beadscf.Engine(0)
    try:
        e.load_basis(sto3g)
        e.set_instances([z] * P)
        e.set_geometries(list(xb))
        e.pimd_init(m, None, beadscf.pimd_default_opts(dt=dt, temperature=T, tau_centroid=20 * FS, seed=5))
        ke = []
        x = x0
        for s in range(3000):
            e.pimd_begin(-k[None, :, None] * (x - x0))
            x = e.pimd_state()[0]
            e.pimd_end(-k[None, :, None] * (x - x0))
            if s >= 300:
                ke.append(e.pimd_state()[2])
        ratio = np.mean(ke) / (1.5 * P * len(z) * KB * T)
        print("kinetic energy / exact", ratio)
        assert abs(ratio - 1) < 0.05
    finally:
        e.close()


def test_refusals(beadscf, sto3g):
    e = beadscf.Engine(0)
    try:
        e.load_basis(sto3g)
        z, x = inputs.h2_molecule()
        e.set_instances([z] * 65)
        e.set_geometries([x] * 65)
        with pytest.raises(beadscf.BscfError) as ei:
            e.pimd_init(np.array([1837.0, 1837.0]))
        assert ei.value.code == -2
        zw, xw = inputs.workload("h2o_sto3g")["instances"][0]
        e.set_instances([zw, z])
        e.set_geometries([xw, x])
        with pytest.raises(beadscf.BscfError) as ei:
            e.pimd_init(np.array([1.0, 1.0, 1.0]))
        assert ei.value.code == -1
        e.set_instances([z, z])
        e.set_geometries([x, x])
        with pytest.raises(beadscf.BscfError) as ei:
            e.pimd_begin()
        assert ei.value.code == -4     # no ring polymer yet
        e.pimd_init(np.array([1837.0, 1837.0]))
        with pytest.raises(beadscf.BscfError) as ei:
            e.pimd_end()
        assert ei.value.code == -4     # no forces of the context at these positions
        e.pimd_begin(np.zeros((2, 2, 3)))
        e.pimd_end(np.zeros((2, 2, 3)))
        assert e.pimd_state()[4] == 1
    finally:
        e.close()
