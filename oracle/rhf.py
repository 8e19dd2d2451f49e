"""Closed-shell Hartree-Fock (RHF) energy and analytic gradient, plain FP64.

TEST INFRASTRUCTURE (see package docstring).  Integrals come from the
McMurchie-Davidson C code in ``mdints.c``; the SCF iteration and the gradient
assembly are written here with numpy/scipy.

The paper (Section 3.1) runs its Gaussian-basis SCF with a density threshold of
1e-6 and an integral cutoff of 1e-12 and computes the analytic BO force of
every replica (Section 2).  The formulas are textbook:
  * Roothaan-Hall: F = H + J - K/2, FC = SCe, P = 2 C_occ C_occ^T,
    E = Tr[P(H+F)]/2 + E_nuc (Szabo and Ostlund, Sections 3.4.1-3.4.6).
  * Loewdin orthogonalisation X = S^{-1/2} (canonical if an eigenvalue of S is
    below 1e-7) (Szabo and Ostlund, Section 3.4.5).
  * Pulay DIIS on e = X^T(FPS - SPF)X, subspace 8 (Pulay 1980, 1982).
  * Converged when |E_k - E_{k-1}| < e_tol and max|e_k| < comm_tol; the energy,
    density and Fock matrix reported are those of the last Fock build.
  * Gradient dE/dX = sum P dH/dX - sum W dS/dX + 1/2 sum (mn|ls)^X
    [P_mn P_ls - 1/2 P_ml P_ns] + dE_nuc/dX with W = P F P / 2 (Pople,
    Krishnan, Schlegel and Binkley 1979).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdints.c")
_LIB = os.path.join(_HERE, "_mdints.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile mdints.c with gcc (OpenMP) into oracle/_mdints.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _c():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_jk.restype = ctypes.c_long
        _lib.or_grad_2e.restype = ctypes.c_long
        _lib.or_grad_2e_atoms.restype = ctypes.c_long
        _lib.or_grad_2e_kx.restype = ctypes.c_long
        _lib.or_jk_sample.restype = ctypes.c_long
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bargs(b):
    return [ctypes.c_int(b["nsh"]), ctypes.c_int(b["nbf"]), _p(b["l"]), _p(b["atom"]),
            _p(b["nprim"]), _p(b["pofs"]), _p(b["bf"]), _p(b["exps"]), _p(b["coefs"])]


def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    _c().or_boys(ctypes.c_int(mmax), ctypes.c_double(T), _p(F))
    return F


def one_electron(b):
    """S, T, V (V = -sum_C Z_C <m|1/r_C|n>), each n x n."""
    n = b["nbf"]
    S, T, V = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    Zi = np.ascontiguousarray(b["Z"], dtype=np.int32)
    _c().or_one_electron(*_bargs(b), ctypes.c_int(len(Zi)), _p(b["xyz"]), _p(Zi),
                         _p(S), _p(T), _p(V))
    return S, T, V


def eri_tensor(b) -> np.ndarray:
    n = b["nbf"]
    out = np.zeros((n, n, n, n))
    _c().or_eri_tensor(*_bargs(b), _p(b["xyz"]), _p(out))
    return out


def eri_quartet(b, a, bb, c, d, deriv: bool = False):
    """Contracted block (ab|cd) [na,nb,nc,nd]; with deriv also the centre
    derivatives [4 centres, 3 directions, na, nb, nc, nd]."""
    nc = [(int(b["l"][s]) + 1) * (int(b["l"][s]) + 2) // 2 for s in (a, bb, c, d)]
    out = np.zeros(nc)
    der = np.zeros([4, 3] + nc) if deriv else None
    _c().or_eri_quartet(*_bargs(b), _p(b["xyz"]), ctypes.c_int(a), ctypes.c_int(bb),
                        ctypes.c_int(c), ctypes.c_int(d), _p(out),
                        _p(der) if deriv else ctypes.c_void_p(0))
    return (out, der) if deriv else out


def schwarz(b) -> np.ndarray:
    Q = np.zeros((b["nsh"], b["nsh"]))
    _c().or_schwarz(*_bargs(b), _p(b["xyz"]), _p(Q))
    return Q


def jk(b, P, tau: float = 1e-12, Q=None):
    """Direct J and K at density P; returns (J, K, number of shell quartets)."""
    n = b["nbf"]
    if Q is None:
        Q = schwarz(b)
    P = np.ascontiguousarray(P, dtype=np.float64)
    J, K = np.zeros((n, n)), np.zeros((n, n))
    nq = _c().or_jk(*_bargs(b), _p(b["xyz"]), _p(np.ascontiguousarray(Q)),
                    ctypes.c_double(tau), _p(P), _p(J), _p(K))
    return J, K, int(nq)


def jk_sample(b, P, stride: int, nthreads: int = 0, tau: float = 1e-12, Q=None):
    """Timing sample of ``jk``: every stride-th canonical screened quartet
    only, on nthreads threads (0: the OpenMP default).  Returns (partial J,
    partial K, quartets evaluated)."""
    n = b["nbf"]
    if Q is None:
        Q = schwarz(b)
    P = np.ascontiguousarray(P, dtype=np.float64)
    J, K = np.zeros((n, n)), np.zeros((n, n))
    nq = _c().or_jk_sample(*_bargs(b), _p(b["xyz"]), _p(np.ascontiguousarray(Q)), ctypes.c_double(tau),
                           _p(P), ctypes.c_int(stride), ctypes.c_int(nthreads), _p(J), _p(K))
    return J, K, int(nq)


def jk_pairs(b, P, pairs, tau: float = 1e-12, Q=None):
    """J and K blocks of the shell pairs (a, b) in ``pairs`` by direct
    summation over every ket shell pair, each term screened by the Schwarz
    rule of its canonical quartet (as in ``jk``).  Returns n x n arrays J, K
    holding those blocks, NaN elsewhere."""
    n = b["nbf"]
    if Q is None:
        Q = schwarz(b)
    P = np.ascontiguousarray(P, dtype=np.float64)
    pa = np.ascontiguousarray([int(a) for a, _ in pairs], dtype=np.int32)
    pb = np.ascontiguousarray([int(c) for _, c in pairs], dtype=np.int32)
    J, K = np.full((n, n), np.nan), np.full((n, n), np.nan)
    _c().or_jk_pairs(*_bargs(b), _p(b["xyz"]), _p(np.ascontiguousarray(Q)), ctypes.c_double(tau),
                     _p(P), ctypes.c_int(len(pa)), _p(pa), _p(pb), _p(J), _p(K))
    return J, K


def nuclear_repulsion(Z, xyz) -> float:
    Z = np.asarray(Z, float)
    e = 0.0
    for i in range(len(Z)):
        for j in range(i):
            e += Z[i] * Z[j] / np.linalg.norm(xyz[i] - xyz[j])
    return e


def nuclear_repulsion_gradient(Z, xyz) -> np.ndarray:
    Z = np.asarray(Z, float)
    g = np.zeros((len(Z), 3))
    for i in range(len(Z)):
        for j in range(len(Z)):
            if i != j:
                r = xyz[i] - xyz[j]
                g[i] -= Z[i] * Z[j] * r / np.linalg.norm(r) ** 3
    return g


def fock_energy(b, H, P, tau=1e-12, Q=None, e_nuc=None):
    """F = H + J - K/2 and E = Tr[P(H+F)]/2 + E_nuc at density P."""
    J, K, _ = jk(b, P, tau, Q)
    F = H + J - 0.5 * K
    if e_nuc is None:
        e_nuc = nuclear_repulsion(b["Z"], b["xyz"])
    return F, 0.5 * np.sum(P * (H + F)) + e_nuc


def orthogonaliser(S, thresh=1e-7):
    s, U = np.linalg.eigh(S)
    if s.min() < thresh:
        keep = s >= thresh
        return U[:, keep] / np.sqrt(s[keep])
    return (U / np.sqrt(s)) @ U.T


def _density(Fp, X, nocc):
    e, Cp = scipy.linalg.eigh(Fp)
    C = X @ Cp
    Co = C[:, :nocc]
    return 2.0 * Co @ Co.T, C, e


def n_electrons(b, charge=0):
    return int(np.sum(b["Z"])) - charge


def scf(b, e_tol=1e-8, comm_tol=1e-6, max_iter=100, guess=None, tau=1e-12, diis_size=8,
        charge=0, verbose=False):
    """RHF SCF.  ``guess``: None (core Hamiltonian) or a density matrix.

    Returns dict(E, P, F, C, eps, n_iter, converged, S, H, X, history).
    """
    ne = n_electrons(b, charge)
    if ne % 2:
        raise ValueError("odd electron count")
    nocc = ne // 2
    S, T, V = one_electron(b)
    H = T + V
    X = orthogonaliser(S)
    Q = schwarz(b)
    e_nuc = nuclear_repulsion(b["Z"], b["xyz"])
    if guess is None:
        P, _, _ = _density(X.T @ H @ X, X, nocc)
    else:
        P = np.array(guess, dtype=np.float64)
    Fs, Es = [], []
    E_prev = None
    hist = []
    for k in range(max_iter):
        F, E = fock_energy(b, H, P, tau, Q, e_nuc)
        err = X.T @ (F @ P @ S - S @ P @ F) @ X
        emax = float(np.abs(err).max())
        hist.append((E, emax))
        if verbose:
            print(f"  iter {k:3d}  E = {E:.12f}  max|e| = {emax:.3e}")
        if E_prev is not None and abs(E - E_prev) < e_tol and emax < comm_tol:
            return dict(E=E, P=P, F=F, n_iter=k + 1, converged=True, S=S, H=H, X=X,
                        history=hist, Q=Q)
        E_prev = E
        Fs.append(F)
        Es.append(err)
        if len(Fs) > diis_size:
            Fs.pop(0)
            Es.pop(0)
        Fbar = F
        while len(Fs) >= 2:
            m = len(Fs)
            B = -np.ones((m + 1, m + 1))
            B[m, m] = 0.0
            for i in range(m):
                for j in range(m):
                    B[i, j] = np.sum(Es[i] * Es[j])
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            if np.linalg.cond(B) > 1e14:
                Fs.pop(0)
                Es.pop(0)
                continue
            c = np.linalg.solve(B, rhs)[:m]
            Fbar = sum(ci * Fi for ci, Fi in zip(c, Fs))
            break
        P, _, _ = _density(X.T @ Fbar @ X, X, nocc)
    return dict(E=E, P=P, F=F, n_iter=max_iter, converged=False, S=S, H=H, X=X, history=hist,
                Q=Q)


def gradient(b, P, F, tau=1e-12, Q=None, atoms=None, kx=1.0):
    """dE/dR [natom,3] at density P with Fock matrix F (W = P F P / 2).
    With ``atoms`` (indices) only those rows are computed; the others are NaN.
    ``kx`` is the share of exact exchange in the two-electron term (1 for
    Hartree-Fock; with kx != 1 every atom is computed)."""
    nat = len(b["Z"])
    P = np.ascontiguousarray(P, dtype=np.float64)
    W = np.ascontiguousarray(0.5 * P @ F @ P)
    Zi = np.ascontiguousarray(b["Z"], dtype=np.int32)
    if Q is None:
        Q = schwarz(b)
    Q = np.ascontiguousarray(Q)
    g1, g2 = np.zeros((nat, 3)), np.zeros((nat, 3))
    if atoms is None or kx != 1.0:
        _c().or_grad_1e(*_bargs(b), ctypes.c_int(nat), _p(b["xyz"]), _p(Zi), _p(P), _p(W), _p(g1))
        _c().or_grad_2e_kx(*_bargs(b), _p(b["xyz"]), ctypes.c_int(nat), _p(Q),
                           ctypes.c_double(tau), _p(P), ctypes.c_double(kx), _p(g2))
        return g1 + g2 + nuclear_repulsion_gradient(b["Z"], b["xyz"])
    mask = np.zeros(nat, np.int32)
    mask[np.asarray(atoms, int)] = 1
    _c().or_grad_1e_atoms(*_bargs(b), ctypes.c_int(nat), _p(b["xyz"]), _p(Zi), _p(P), _p(W),
                          _p(mask), _p(g1))
    _c().or_grad_2e_atoms(*_bargs(b), _p(b["xyz"]), ctypes.c_int(nat), _p(Q), ctypes.c_double(tau),
                          _p(P), _p(mask), _p(g2))
    g = g1 + g2 + nuclear_repulsion_gradient(b["Z"], b["xyz"])
    g[mask == 0] = np.nan
    return g
