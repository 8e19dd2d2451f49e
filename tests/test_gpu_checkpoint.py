"""Checkpoint and resume between MD steps (bscf_checkpoint_save / _load): a
new context that loads the file written after step k takes step k + 1 as the
uninterrupted run does.  The carried orbitals (the previous-step and
extrapolated guesses, the reuse of orbitals of Section 2), the ring
polymer's positions, momenta and step counter (the thermostat's counters),
the gradient at the current positions and the guess network all come back.
FP64 path with deterministic J/K; the forces' own accumulation is atomic, so
the comparison allows rounding."""

import os

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

FS = 41.341373336
AMU = 1822.888486209
MASS = {1: 1.008 * AMU, 8: 15.999 * AMU}


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


def _setup(beadscf, basis, z, xb):
    e = beadscf.Engine(0)
    e.load_basis(basis)
    e.set_instances([z] * len(xb))
    e.set_geometries(list(xb))
    return e


def test_resumed_step_repeats_the_uninterrupted_one(beadscf, b631gs, tmp_path):
    P, T = 4, 300.0
    z, x = inputs.water_cluster(2, 21)
    xb = inputs.beads(z, x, P, 21)
    m = np.array([MASS[int(v)] for v in z])
    p0 = inputs.maxwell_boltzmann(z, P, T, 21) * m[None, :, None]
    so = beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8, guess=beadscf.GUESS_EXTRAPOLATED,
                              deterministic=1)
    path = str(tmp_path / "run.ckpt")
    e = _setup(beadscf, b631gs, z, xb)
    try:
        e.pimd_init(m, p0, beadscf.pimd_default_opts(dt=0.5 * FS, temperature=T, seed=7))
        for _ in range(3):
            e.pimd_step(so)
        x3, p3, _, _, k3 = e.pimd_state()
        e.guess_configure(24, 8, seed=11)
        theta = e.guess_params()
        e.checkpoint_save(path)
        E4, it4, st4, F4 = e.pimd_step(so, return_forces=True)
        x4, p4, _, _, k4 = e.pimd_state()
    finally:
        e.close()
    assert k3 == 3 and k4 == 4 and (st4 == 0).all()

    # a fresh context of the same batch, at an unrelated geometry
    r = _setup(beadscf, b631gs, z, inputs.beads(z, x, P, 99))
    try:
        r.checkpoint_load(path)
        y3, q3, _, _, j3 = r.pimd_state()
        assert j3 == 3
        assert np.array_equal(y3, x3) and np.array_equal(q3, p3)
        assert np.array_equal(r.guess_params(), theta)
        E, it, st, F = r.pimd_step(so, return_forces=True)
        y4, q4, _, _, j4 = r.pimd_state()
    finally:
        r.close()
    assert j4 == 4 and (st == 0).all()
    # the saved gradient is used: no SCF at the saved positions, the same
    # iterations from the carried orbitals
    assert np.array_equal(it, it4)
    assert np.abs(E - E4).max() < 1e-10
    for a, b in zip(F, F4):
        assert np.abs(a - b).max() < 1e-9
    assert np.abs(y4 - x4).max() < 1e-12
    assert np.abs(q4 - p4).max() < 1e-9 * np.abs(p4).max()


def test_step_counter_sets_the_thermostat_draws(beadscf, b631gs, tmp_path):
    """Restarting the integrator at the saved positions and momenta with a
    new bscf_pimd_init (step 0) draws other thermostat deviates: the
    checkpoint's step counter is what makes the resumed step repeat."""
    P, T = 4, 300.0
    z, x = inputs.water_cluster(2, 22)
    xb = inputs.beads(z, x, P, 22)
    m = np.array([MASS[int(v)] for v in z])
    opts = beadscf.pimd_default_opts(dt=0.5 * FS, temperature=T, seed=3)
    F = [np.zeros((len(z), 3))] * P
    path = str(tmp_path / "h.ckpt")
    e = _setup(beadscf, b631gs, z, xb)
    try:
        e.pimd_init(m, None, opts)
        for _ in range(2):
            e.pimd_begin(F)
            e.pimd_end(F)
        x2, p2, _, _, _ = e.pimd_state()
        e.checkpoint_save(path)
        e.pimd_begin(F)
        e.pimd_end(F)
        xa, pa, _, _, _ = e.pimd_state()
        e.checkpoint_load(path)
        e.pimd_begin(F)
        e.pimd_end(F)
        xb2, pb, _, _, k = e.pimd_state()
        e.set_geometries(list(x2))
        e.pimd_init(m, p2, opts)
        e.pimd_begin(F)
        e.pimd_end(F)
        xc, pc, _, _, _ = e.pimd_state()
    finally:
        e.close()
    assert k == 3
    assert np.array_equal(xb2, xa) and np.array_equal(pb, pa)
    assert np.abs(pc - pa).max() > 1e-3 * np.abs(pa).max()


def test_rejected_files_leave_the_context_unchanged(beadscf, b631gs, tmp_path):
    z, x = inputs.water_cluster(2, 23)
    xb = inputs.beads(z, x, 3, 23)
    path = str(tmp_path / "a.ckpt")
    e = _setup(beadscf, b631gs, z, xb)
    try:
        E0, _, _ = e.run_scf(e_tol=1e-10, comm_tol=1e-8)
        e.checkpoint_save(path)
        raw = open(path, "rb").read()
        short = str(tmp_path / "short.ckpt")
        with open(short, "wb") as f:
            f.write(raw[: len(raw) // 2])
        junk = str(tmp_path / "junk.ckpt")
        with open(junk, "wb") as f:
            f.write(os.urandom(64))
        for bad in (short, junk, str(tmp_path / "missing.ckpt")):
            with pytest.raises(beadscf.BscfError):
                e.checkpoint_load(bad)
        # the geometry and density are those of before the rejected loads
        F = e.forces()
        assert all(np.isfinite(f).all() for f in F)
        E1, it1, _ = e.run_scf(e_tol=1e-10, comm_tol=1e-8, guess=beadscf.GUESS_PREVIOUS)
        assert np.abs(E1 - E0).max() < 1e-9 and (it1 <= 3).all()
    finally:
        e.close()
    # a batch of another size refuses the file
    o = _setup(beadscf, b631gs, z, inputs.beads(z, x, 2, 23))
    try:
        with pytest.raises(beadscf.BscfError):
            o.checkpoint_load(path)
    finally:
        o.close()


def test_resume_with_the_learned_guess(beadscf, b631gs, tmp_path):
    """The headline's guess: the network, its Adam moments, its last
    residual and its replay buffer come back, so the resumed step predicts
    from the same model and needs the same iterations, and training after it
    continues from the same buffer."""
    P, T = 4, 300.0
    z, x = inputs.water_cluster(2, 24)
    xb = inputs.beads(z, x, P, 24)
    m = np.array([MASS[int(v)] for v in z])
    so = beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8, guess=beadscf.GUESS_LEARNED)
    path = str(tmp_path / "learned.ckpt")
    e = _setup(beadscf, b631gs, z, xb)
    try:
        e.pimd_init(m, None, beadscf.pimd_default_opts(dt=0.5 * FS, temperature=T, seed=8))
        for _ in range(4):
            e.pimd_step(so)
            e.guess_train(30)
        theta = e.guess_params()
        e.checkpoint_save(path)
        E5, it5, st5 = e.pimd_step(so)
        l5 = e.guess_train(30)
        theta5 = e.guess_params()
    finally:
        e.close()
    assert ((st5 & 1) == 0).all() and not (st5 & 4).any()   # converged, the network was used

    r = _setup(beadscf, b631gs, z, xb)
    try:
        r.checkpoint_load(path)
        assert np.array_equal(r.guess_params(), theta)
        E, it, st = r.pimd_step(so)
        l = r.guess_train(30)
        th = r.guess_params()
    finally:
        r.close()
    assert not (st & 4).any()
    assert np.array_equal(it, it5)
    assert np.abs(E - E5).max() < 1e-10
    assert abs(l - l5) <= 1e-4 * abs(l5)
    assert np.abs(th - theta5).max() <= 1e-4 * np.abs(theta5).max()
