"""Contracted Cartesian Gaussian shells for the oracle.

Primitive g = x_A^lx y_A^ly z_A^lz exp(-alpha r_A^2) with normalisation
N = (2 alpha/pi)^{3/4} (4 alpha)^{l/2} / sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!);
the contracted function sum_k d_k N_k g_k is rescaled to unit self-overlap.
Only the radial part (2 alpha/pi)^{3/4}(4 alpha)^{l/2} and the contraction
rescaling enter the coefficients returned here; the per-component
double-factorial factor is applied by the C code, so every Cartesian
component has unit norm.
"""

from __future__ import annotations

import math

import numpy as np


def _contracted_rescale(l: int, alphas, cs) -> float:
    """1/sqrt(<phi|phi>) for phi = sum_k c_k g_k with radially normalised
    primitives, using <g_k|g_j> = (2l-1)!! (pi/(a+b))^{3/2} / (2(a+b))^l for
    the x^l component (the double factorial cancels with the component norm)."""
    s = 0.0
    for a, ca in zip(alphas, cs):
        for b, cb in zip(alphas, cs):
            na = (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2)
            nb = (2 * b / math.pi) ** 0.75 * (4 * b) ** (l / 2)
            s += ca * cb * na * nb * (math.pi / (a + b)) ** 1.5 / (2 * (a + b)) ** l
    return 1.0 / math.sqrt(s)


def build_basis(basis: dict, Z, xyz) -> dict:
    """Shell arrays for one molecule.

    Returns dict with int32 arrays l, atom, nprim, pofs, bf; float64 arrays
    exps, coefs; nbf, nsh; and the geometry (xyz [natom,3] bohr, Z int32).
    Shells follow atom order, then the order of the basis file.
    """
    Z = np.asarray(Z, dtype=np.int32)
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    by_z = {v["Z"]: v for v in basis["elements"].values()}
    L, atom, nprim, pofs, bf, exps, coefs = [], [], [], [], [], [], []
    nbf = 0
    for ia, z in enumerate(Z):
        if int(z) not in by_z:
            raise ValueError(f"element Z={int(z)} not in basis {basis['name']}")
        for sh in by_z[int(z)]["shells"]:
            l = int(sh["l"])
            al = [float(a) for a in sh["exponents"]]
            d = [float(c) for c in sh["coefficients"]]
            r = _contracted_rescale(l, al, d)
            L.append(l)
            atom.append(ia)
            nprim.append(len(al))
            pofs.append(len(exps))
            bf.append(nbf)
            for a, c in zip(al, d):
                exps.append(a)
                coefs.append(c * r * (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2))
            nbf += (l + 1) * (l + 2) // 2
    i32 = lambda v: np.ascontiguousarray(np.array(v, dtype=np.int32))
    return dict(l=i32(L), atom=i32(atom), nprim=i32(nprim), pofs=i32(pofs), bf=i32(bf),
                exps=np.array(exps, np.float64), coefs=np.array(coefs, np.float64),
                nbf=nbf, nsh=len(L), xyz=xyz, Z=Z)
