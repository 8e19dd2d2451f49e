"""Pins of the oracle's integrals against mathematics it does not use.

* Boys function against mpmath (defining integral / incomplete gamma) and its
  closed forms and recursion.
* s-type S, T, V and ERI against the closed forms; p and d functions against
  symbolic centre-derivatives of those closed forms (tests/_closed_forms.py).
* Szabo-Ostlund's printed H2/STO-3G integrals (tests/golden).
* Structural properties of the full ERI tensor: 8-fold symmetry, Cauchy-
  Schwarz, positive semidefinite supermatrix.
* Translational invariance of the ERI centre derivatives.
"""

import json
import math
import os

import mpmath
import numpy as np
import pytest

import inputs
import oracle
from tests import _closed_forms as cf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Boys
@pytest.mark.parametrize("T", [0.0, 1e-9, 1e-3, 0.3, 1.0, 2.5, 7.0, 12.0, 19.9, 29.9, 30.0,
                               30.1, 45.0, 80.0, 300.0])
def test_boys_against_mpmath(T):
    mpmath.mp.dps = 40
    F = oracle.boys(12, T)
    for m in range(13):
        ref = float(mpmath.quad(lambda t: t ** (2 * m) * mpmath.exp(-T * t * t), [0, 1]))
        assert abs(F[m] - ref) <= 2e-15 * abs(ref), (m, T, F[m], ref)


def test_boys_closed_forms():
    for m in range(10):
        assert oracle.boys(m, 0.0)[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)
    for T in [0.5, 3.0, 40.0]:
        assert oracle.boys(0, T)[0] == pytest.approx(
            0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T)), rel=1e-15)
    # large-T asymptotic (2m-1)!!/2^{m+1} sqrt(pi/T^{2m+1})
    T = 200.0
    F = oracle.boys(8, T)
    for m in range(9):
        df = 1.0
        for k in range(2 * m - 1, 0, -2):
            df *= k
        assert F[m] == pytest.approx(df / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1)),
                                     rel=1e-14)
    # recursion 2T F_{m+1} = (2m+1) F_m - exp(-T) and dF_m/dT = -F_{m+1}
    for T in [0.7, 8.0, 29.0, 33.0]:
        F = oracle.boys(9, T)
        for m in range(8):
            assert 2 * T * F[m + 1] == pytest.approx((2 * m + 1) * F[m] - math.exp(-T), rel=1e-13)
        h = 1e-5
        d = (oracle.boys(9, T + h) - oracle.boys(9, T - h)) / (2 * h)
        assert np.allclose(d[:8], -F[1:9], rtol=1e-8)


# ---------------------------------------------------- primitive basis helper
def _prim_basis(shells):
    """shells: list of (l, alpha, centre xyz, Z) -> oracle basis dict with one
    uncontracted primitive per shell, each on its own atom."""
    l, atom, nprim, pofs, bf, exps, coefs = [], [], [], [], [], [], []
    nbf = 0
    for k, (ll, a, _, _) in enumerate(shells):
        l.append(ll); atom.append(k); nprim.append(1); pofs.append(k); bf.append(nbf)
        exps.append(a)
        coefs.append((2 * a / math.pi) ** 0.75 * (4 * a) ** (ll / 2))
        nbf += (ll + 1) * (ll + 2) // 2
    i32 = lambda v: np.array(v, dtype=np.int32)
    return dict(l=i32(l), atom=i32(atom), nprim=i32(nprim), pofs=i32(pofs), bf=i32(bf),
                exps=np.array(exps), coefs=np.array(coefs), nbf=nbf, nsh=len(l),
                xyz=np.array([s[2] for s in shells], float), Z=i32([s[3] for s in shells]))


def _cart(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def _norm(a, t):
    l = sum(t)
    df = lambda n: math.prod(range(n, 0, -2)) if n > 0 else 1
    return (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2) / math.sqrt(
        df(2 * t[0] - 1) * df(2 * t[1] - 1) * df(2 * t[2] - 1))


def _values(shells, names):
    v = {}
    for (l, a, X, _), n in zip(shells, names):
        v[f"e{n}"] = a
        for k, c in enumerate("xyz"):
            v[f"{n}{c}"] = X[k]
    return v


RNG = np.random.default_rng(7)


def _rand_centre():
    return RNG.uniform(-1.2, 1.2, 3)


# ------------------------------------------------------ s-type closed forms
def test_s_type_closed_forms():
    mpmath.mp.dps = 30
    for _ in range(4):
        sh = [(0, RNG.uniform(0.1, 5.0), _rand_centre(), 1) for _ in range(4)]
        b = _prim_basis(sh)
        S, T, V = oracle.one_electron(b)
        vals = _values(sh, "ABCD")
        nrm = [_norm(s[1], (0, 0, 0)) for s in sh]
        assert S[0, 1] == pytest.approx(nrm[0] * nrm[1] * float(cf.evaluate(cf.s_overlap(), vals)), rel=1e-13)
        assert T[0, 1] == pytest.approx(nrm[0] * nrm[1] * float(cf.evaluate(cf.s_kinetic(), vals)), rel=1e-12)
        vsum = 0.0
        for k in range(4):
            vv = dict(vals, Nx=sh[k][2][0], Ny=sh[k][2][1], Nz=sh[k][2][2])
            vsum -= sh[k][3] * float(cf.evaluate(cf.s_nuclear(), vv))
        assert V[0, 1] == pytest.approx(nrm[0] * nrm[1] * vsum, rel=1e-13)
        eri = oracle.eri_quartet(b, 0, 1, 2, 3)
        ref = math.prod(nrm) * float(cf.evaluate(cf.s_eri(), vals))
        assert eri[0, 0, 0, 0] == pytest.approx(ref, rel=1e-13)


# --------------------------------------- any-l integrals by differentiation
ONE_E_CASES = [(1, 0), (0, 1), (1, 1), (2, 0), (2, 1), (2, 2)]


@pytest.mark.parametrize("la,lb", ONE_E_CASES)
def test_one_electron_higher_l(la, lb):
    mpmath.mp.dps = 30
    sh = [(la, RNG.uniform(0.2, 3.0), _rand_centre(), 2), (lb, RNG.uniform(0.2, 3.0), _rand_centre(), 3),
          (0, 1.0, _rand_centre(), 1)]
    b = _prim_basis(sh)
    S, T, V = oracle.one_electron(b)
    vals = _values(sh[:2], "AB")
    na = (la + 1) * (la + 2) // 2
    for i, ta in enumerate(_cart(la)):
        for j, tb in enumerate(_cart(lb)):
            nrm = _norm(sh[0][1], ta) * _norm(sh[1][1], tb)
            s_ref = cf.evaluate(cf.build(cf.s_overlap(), {"A": ta, "B": tb}), vals)
            t_ref = cf.evaluate(cf.build(cf.s_kinetic(), {"A": ta, "B": tb}), vals)
            assert S[i, na + j] == pytest.approx(nrm * float(s_ref), rel=1e-12, abs=1e-14)
            assert T[i, na + j] == pytest.approx(nrm * float(t_ref), rel=1e-12, abs=1e-14)
            vexpr = cf.build(cf.s_nuclear(), {"A": ta, "B": tb})
            v_ref = 0.0
            for k in range(3):
                vv = dict(vals, Nx=sh[k][2][0], Ny=sh[k][2][1], Nz=sh[k][2][2])
                v_ref -= sh[k][3] * float(cf.evaluate(vexpr, vv))
            assert V[i, na + j] == pytest.approx(nrm * v_ref, rel=1e-11, abs=1e-13)


ERI_CASES = [(1, 0, 0, 0), (0, 0, 1, 0), (1, 1, 0, 0), (1, 0, 1, 0), (2, 0, 0, 0), (0, 1, 0, 1),
             (2, 1, 0, 0), (2, 0, 1, 0), (1, 1, 1, 0), (0, 0, 2, 1)]


@pytest.mark.parametrize("ls", ERI_CASES)
def test_eri_higher_l(ls):
    mpmath.mp.dps = 30
    sh = [(l, RNG.uniform(0.2, 3.0), _rand_centre(), 1) for l in ls]
    b = _prim_basis(sh)
    blk = oracle.eri_quartet(b, 0, 1, 2, 3)
    vals = _values(sh, "ABCD")
    base = cf.s_eri()
    carts = [_cart(l) for l in ls]
    # check a handful of components per class (symbolic cost grows fast)
    idx = [(0, 0, 0, 0), tuple(len(c) - 1 for c in carts),
           tuple(RNG.integers(0, len(c)) for c in carts)]
    for ix in idx:
        ts = [carts[k][ix[k]] for k in range(4)]
        expr = cf.build(base, {"A": ts[0], "B": ts[1], "C": ts[2], "D": ts[3]})
        nrm = math.prod(_norm(sh[k][1], ts[k]) for k in range(4))
        ref = nrm * float(cf.evaluate(expr, vals))
        assert blk[ix] == pytest.approx(ref, rel=1e-11, abs=1e-14), (ix, blk[ix], ref)


# --------------------------------------------------------- textbook values
def test_szabo_ostlund_h2(sto3g):
    g = json.load(open(os.path.join(GOLD, "h2_sto3g_szabo_ostlund.json")))
    Z, x = inputs.h2_molecule(g["r_bohr"])
    b = oracle.build_basis(sto3g, Z, x)
    S, T, V = oracle.one_electron(b)
    H = T + V
    eri = oracle.eri_tensor(b)
    tol = g["tolerance"]
    assert abs(S[0, 1] - g["S12"]) < tol
    assert abs(T[0, 0] - g["T11"]) < tol and abs(T[0, 1] - g["T12"]) < tol
    assert abs(H[0, 0] - g["Hcore11"]) < tol and abs(H[0, 1] - g["Hcore12"]) < tol
    assert abs(eri[0, 0, 0, 0] - g["eri_11_11"]) < tol
    assert abs(eri[0, 0, 1, 1] - g["eri_11_22"]) < tol
    assert abs(eri[1, 0, 0, 0] - g["eri_21_11"]) < tol
    assert abs(eri[1, 0, 1, 0] - g["eri_21_21"]) < tol
    r = oracle.scf(b, 1e-12, 1e-10)
    eps = np.linalg.eigvalsh(r["X"].T @ r["F"] @ r["X"])
    assert abs(eps[0] - g["eps1"]) < tol and abs(eps[1] - g["eps2"]) < tol
    assert abs(r["E"] - g["E_total"]) < tol


# -------------------------------------------------- tensor-level structure
@pytest.fixture(scope="module")
def h2o_tensor(sto3g):
    w = inputs.workload("h2o_sto3g")
    Z, x = w["instances"][0]
    b = oracle.build_basis(sto3g, Z, x)
    return b, oracle.eri_tensor(b)


def test_eri_permutational_symmetry(h2o_tensor):
    _, g = h2o_tensor
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.abs(g - g.transpose(perm)).max() < 1e-13


def test_eri_schwarz_and_psd(h2o_tensor):
    b, g = h2o_tensor
    n = b["nbf"]
    M = g.reshape(n * n, n * n)
    d = np.sqrt(np.abs(np.diag(M)))
    assert np.all(np.abs(M) <= np.outer(d, d) * (1 + 1e-12) + 1e-15)
    assert np.linalg.eigvalsh(M).min() > -1e-12
    Q = oracle.schwarz(b)
    for a in range(b["nsh"]):
        for c in range(b["nsh"]):
            ia = slice(b["bf"][a], b["bf"][a] + (b["l"][a] + 1) * (b["l"][a] + 2) // 2)
            ic = slice(b["bf"][c], b["bf"][c] + (b["l"][c] + 1) * (b["l"][c] + 2) // 2)
            blk = g[ia, ic, ia, ic]
            m = max(abs(blk[i, j, i, j]) for i in range(blk.shape[0]) for j in range(blk.shape[1]))
            assert Q[a, c] == pytest.approx(math.sqrt(m), rel=1e-14)


def test_eri_far_field():
    """(ss|ss) -> S_ab S_cd / R_PQ when the two distributions are far apart."""
    sh = [(0, 1.3, np.zeros(3), 1), (0, 0.7, np.array([0.3, 0, 0]), 1),
          (0, 1.1, np.array([0, 0, 40.0]), 1), (0, 0.9, np.array([0, 0.2, 40.0]), 1)]
    b = _prim_basis(sh)
    S, _, _ = oracle.one_electron(b)
    eri = oracle.eri_quartet(b, 0, 1, 2, 3)[0, 0, 0, 0]
    P = (1.3 * sh[0][2] + 0.7 * sh[1][2]) / 2.0
    Qc = (1.1 * sh[2][2] + 0.9 * sh[3][2]) / 2.0
    assert eri == pytest.approx(S[0, 1] * S[2, 3] / np.linalg.norm(P - Qc), rel=1e-12)


def test_eri_derivative_translational_invariance(b631gs):
    Z, x = inputs.water_cluster(2, 11)
    b = oracle.build_basis(b631gs, Z, x)
    # shells: pick mixed classes including d
    for q in [(5, 2, 15, 12), (5, 5, 5, 4), (2, 0, 14, 13), (9, 4, 19, 18)]:
        blk, der = oracle.eri_quartet(b, *q, deriv=True)
        assert np.abs(der.sum(axis=0)).max() < 1e-11 * max(1.0, np.abs(der).max())
        # and against a central difference of the centre of shell q[0]'s atom
        # when that atom carries no other shell of the quartet
    sh = [(1, 0.9, _rand_centre(), 1), (2, 1.4, _rand_centre(), 1),
          (1, 0.6, _rand_centre(), 1), (0, 2.0, _rand_centre(), 1)]
    b = _prim_basis(sh)
    blk, der = oracle.eri_quartet(b, 0, 1, 2, 3, deriv=True)
    h = 1e-5
    for cen in range(4):
        for d in range(3):
            bp = dict(b, xyz=b["xyz"].copy())
            bm = dict(b, xyz=b["xyz"].copy())
            bp["xyz"][cen, d] += h
            bm["xyz"][cen, d] -= h
            fd = (oracle.eri_quartet(bp, 0, 1, 2, 3) - oracle.eri_quartet(bm, 0, 1, 2, 3)) / (2 * h)
            assert np.abs(fd - der[cen, d]).max() < 1e-8
