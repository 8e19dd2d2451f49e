"""Learned SCF guess on the GPU.

The network kernels (MFMA GEMMs, loss gradient, ReLU masks, bias sums, Adam)
against the NumPy FP64 oracle of oracle/mlp.py on the same FP32-rounded
parameters and rows; then the in-run use on a ring-polymer trajectory: the
converged energies are those of the previous-step guess (the converged SCF
decides) while the learned guess needs fewer SCF iterations, and sabotaged
weights are caught by the fallback.
"""

import numpy as np
import pytest

import inputs
from oracle import mlp

pytestmark = pytest.mark.gpu

H = 256


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


@pytest.fixture(scope="module")
def eng(beadscf):
    e = beadscf.Engine(0)
    yield e
    e.close()


def _rows(rng, rows, din, dout):
    X = rng.standard_normal((rows, din)).astype(np.float32)
    T = rng.standard_normal((rows, dout)).astype(np.float32)
    M = (rng.random((rows, dout)) < 0.8).astype(np.float32)
    return X, T, M


def _theta(rng, din, dout):
    th = mlp.init(din, H, dout, rng)
    W1, b1, W2, b2, W3, b3 = mlp.unflatten(th, din, H, dout)
    # a last layer of ordinary size so the gradients of every block are visible
    W3 = rng.standard_normal(W3.shape) * np.sqrt(2.0 / H)
    b1 = rng.standard_normal(b1.shape) * 0.1
    b2 = rng.standard_normal(b2.shape) * 0.1
    b3 = rng.standard_normal(b3.shape) * 0.1
    return mlp.flatten([W1, b1, W2, b2, W3, b3]).astype(np.float32)


@pytest.mark.parametrize("rows,din,dout", [(150, 37, 9), (64, 64, 64), (1, 70, 5), (3000, 40, 12)])
def test_network_forward_and_gradient_against_oracle(eng, rows, din, dout):
    """Ragged and exact tile shapes, and a long reduction (weight gradients
    over 3000 rows take the split-K path): outputs, loss and every parameter
    gradient within 1e-4 of the FP64 oracle (relative to each block's size)."""
    rng = np.random.default_rng([2000, rows, din])
    eng.guess_configure(din, dout)
    th = _theta(rng, din, dout)
    eng.guess_set_params(th)
    X, T, M = _rows(rng, rows, din, dout)
    Y, g, L = eng.guess_eval(X, T, M)
    th64, X64 = th.astype(np.float64), X.astype(np.float64)
    y_ref, _, _ = mlp.forward(th64, X64, din, H, dout)
    L_ref, g_ref = mlp.gradient(th64, X64, T.astype(np.float64), M.astype(np.float64), din, H, dout)
    assert np.abs(Y - y_ref).max() <= 1e-4 * np.abs(y_ref).max()
    assert abs(L - L_ref) <= 1e-4 * L_ref
    k = 0
    for shape in mlp.shapes(din, H, dout):
        n = int(np.prod(shape))
        blk, ref = g[k:k + n], g_ref[k:k + n]
        assert np.abs(blk - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-30), shape
        k += n


def test_adam_training_against_oracle(eng):
    """Five full-batch Adam steps on the GPU against the oracle's: the loss
    sequence and the parameter updates of well-conditioned entries agree."""
    rng = np.random.default_rng([2000, 7])
    din, dout, rows, steps, lr = 40, 12, 90, 5, 1e-3
    eng.guess_configure(din, dout)
    th = _theta(rng, din, dout)
    eng.guess_set_params(th)
    X, T, M = _rows(rng, rows, din, dout)
    L_last = eng.guess_fit(X, T, M, steps, lr)
    th_gpu = eng.guess_params().astype(np.float64)
    th_ref, losses = mlp.train(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                               M.astype(np.float64), din, H, dout, steps, lr)
    assert abs(L_last - losses[-1]) <= 1e-4 * losses[-1]
    # entries whose gradient stays well away from zero follow the same updates
    _, g0 = mlp.gradient(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                         M.astype(np.float64), din, H, dout)
    sel = np.abs(g0) > 1e-2 * np.abs(g0).max()
    d_gpu, d_ref = th_gpu - th, th_ref - th
    assert np.abs(d_gpu[sel] - d_ref[sel]).max() <= 0.05 * steps * lr


def _trajectory(beadscf, eng, n_steps, seed):
    from paper_1601_02713_amd import md
    z, x = inputs.water_cluster(2, seed)
    P = 2
    xb = inputs.beads(z, x, P, seed)
    v = inputs.maxwell_boltzmann(z, P, 300.0, seed)
    poly = md.RingPolymer(z, xb, v, 300.0)
    opts = beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8)
    return md, poly, opts


BASIS = inputs.load_basis("6-31g*")


def test_learned_guess_gains_over_previous_step_reuse(beadscf, eng):
    """(H2O)2, 2 beads, 12 steps of 0.25 fs: the previous-step guess run
    integrates the trajectory; the learned-guess run replays it, trains after
    every step from step 1 and predicts from step 3.  Same converged energies;
    fewer SCF iterations over the predicted steps."""
    from paper_1601_02713_amd import md
    n_steps = 12
    _, poly, opts = _trajectory(beadscf, eng, n_steps, 31)
    ref, traj = md.run(eng, poly, n_steps, 0.25, guess="previous", opts=opts, basis=BASIS)
    e2 = beadscf.Engine(0)
    try:
        learned, _ = md.run(e2, poly, n_steps, 0.25, guess="learned", opts=opts, geometries=traj,
                            train_from=1, train_steps=40, predict_from=3, basis=BASIS)
    finally:
        e2.close()
    it_ref = np.array([r.iterations for r in ref])
    it_l = np.array([r.iterations for r in learned])
    print("iterations per step, previous-step guess:", it_ref.sum(axis=1).tolist())
    print("iterations per step, learned guess:      ", it_l.sum(axis=1).tolist())
    print("training loss:", [r.train_loss for r in learned])
    for a, b in zip(ref, learned):
        assert np.abs(a.energies - b.energies).max() < 1e-8
        assert ((b.status & ~beadscf.STATUS_FALLBACK) == 0).all()
    # the predicted steps used the network (no fallback) ...
    assert all((r.status & beadscf.STATUS_FALLBACK == 0).all() for r in learned[3:])
    # ... and saved SCF iterations
    assert it_l[3:].sum() < it_ref[3:].sum()


def test_sabotaged_network_falls_back(beadscf, eng):
    """Huge weights make the prediction implausible: the guess falls back to
    the previous-step density, flags it, and the converged energies stand."""
    from paper_1601_02713_amd import md
    n_steps = 5
    _, poly, opts = _trajectory(beadscf, eng, n_steps, 41)
    ref, traj = md.run(eng, poly, n_steps, 0.25, guess="previous", opts=opts, basis=BASIS)
    e2 = beadscf.Engine(0)
    try:
        # train briefly so a model exists, then sabotage it before prediction
        recs, _ = md.run(e2, poly, 3, 0.25, guess="learned", opts=opts, geometries=traj[:3],
                         train_from=1, train_steps=5, predict_from=99, basis=BASIS)
        din, dout, _ = e2.guess_dims()
        rng = np.random.default_rng(5)
        X, T, M = _rows(rng, 16, din, dout)
        e2.guess_fit(X, 1e4 * T, M, 3, 100.0)   # a wild learning rate ruins the weights
        o = beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8, guess=beadscf.GUESS_LEARNED)
        e2.set_geometries(list(traj[3]))
        E, it, st = e2.run_scf(o)
    finally:
        e2.close()
    assert (st & beadscf.STATUS_FALLBACK).all()
    assert np.abs(E - ref[3].energies).max() < 1e-8


def test_model_file_round_trip_and_refusals(beadscf, eng, tmp_path):
    """A saved network loads into another context with the same parameters
    and outputs; a truncated or foreign file is refused and leaves the loaded
    network as it was."""
    rng = np.random.default_rng([2000, 11])
    din, dout = 33, 7
    eng.guess_configure(din, dout)
    th = _theta(rng, din, dout)
    eng.guess_set_params(th)
    X, T, M = _rows(rng, 20, din, dout)
    Y0, _, _ = eng.guess_eval(X, T, M)
    path = str(tmp_path / "model.bin")
    eng.guess_save(path)
    e2 = beadscf.Engine(0)
    try:
        e2.guess_load(path)
        assert e2.guess_dims()[:2] == (din, dout)
        assert np.array_equal(e2.guess_params(), th)
        Y1, _, _ = e2.guess_eval(X, T, M)
        assert np.array_equal(Y0, Y1)
        raw = open(path, "rb").read()
        cut = str(tmp_path / "cut.bin")
        open(cut, "wb").write(raw[:len(raw) // 2])
        junk = str(tmp_path / "junk.bin")
        open(junk, "wb").write(b"\0" * 64)
        for bad in (cut, junk, str(tmp_path / "missing.bin")):
            with pytest.raises(beadscf.BscfError):
                e2.guess_load(bad)
            assert np.array_equal(e2.guess_params(), th)
    finally:
        e2.close()
