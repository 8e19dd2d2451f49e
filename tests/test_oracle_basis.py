"""Pins of the oracle's contracted-shell normalisation (oracle/basis.py).

Every Cartesian component of every contracted shell must have unit
self-overlap.  Two independent checks:
  * the oracle's overlap matrix (its McMurchie-Davidson S, itself pinned by
    the s-type closed forms and their symbolic centre-derivatives) has a unit
    diagonal for one atom of each element of both basis files;
  * the self-overlap of the x^l component is summed here over primitive pairs
    from one-dimensional Gaussian moments found by numerical quadrature,
    int x^2l exp(-(a+b) x^2) dx, with no closed form shared with the oracle.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import inputs
import oracle


@pytest.mark.parametrize("name", ["sto-3g", "6-31g*"])
def test_unit_diagonal_overlap_for_every_shell(name):
    basis = inputs.load_basis(name)
    seen_l = set()
    for el in basis["elements"].values():
        b = oracle.build_basis(basis, [el["Z"]], [[0.1, -0.2, 0.3]])
        S, _, _ = oracle.one_electron(b)
        assert np.abs(np.diag(S) - 1.0).max() < 1e-13, (name, el["Z"], np.diag(S))
        seen_l.update(int(l) for l in b["l"])
    assert seen_l >= ({0, 1, 2} if name == "6-31g*" else {0, 1})


def _moment(n, g):
    """int_-inf^inf x^n exp(-g x^2) dx by quadrature."""
    v, err = integrate.quad(lambda x: x ** n * math.exp(-g * x * x), -np.inf, np.inf,
                            epsabs=0, epsrel=1e-13, limit=200)
    return v


@pytest.mark.parametrize("name", ["sto-3g", "6-31g*"])
def test_contracted_self_overlap_by_quadrature(name):
    basis = inputs.load_basis(name)
    for el in basis["elements"].values():
        b = oracle.build_basis(basis, [el["Z"]], [[0.0, 0.0, 0.0]])
        for s in range(b["nsh"]):
            l, p0, n = int(b["l"][s]), int(b["pofs"][s]), int(b["nprim"][s])
            a = b["exps"][p0:p0 + n]
            c = b["coefs"][p0:p0 + n]
            # the x^l component: the C code multiplies the stored coefficient by
            # 1/sqrt((2l-1)!!) for this component
            dfac = math.prod(range(2 * l - 1, 0, -2)) if l > 0 else 1
            tot = 0.0
            for i in range(n):
                for j in range(n):
                    g = a[i] + a[j]
                    tot += c[i] * c[j] / dfac * _moment(2 * l, g) * _moment(0, g) ** 2
            assert abs(tot - 1.0) < 1e-11, (name, el["Z"], s, l, tot)
