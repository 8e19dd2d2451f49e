"""Independent pins for Gaussian integrals of any angular momentum.

Closed forms for s-type primitives (Szabo and Ostlund, Appendix A):
  S   = (pi/p)^{3/2} K_AB
  T   = mu (3 - 2 mu R_AB^2) S
  V_C = (2 pi/p) K_AB F_0(p |P-C|^2)               (for <a|1/r_C|b>)
  ERI = 2 pi^{5/2} / (p q sqrt(p+q)) K_AB K_CD F_0(rho |P-Q|^2)
with p = a+b, mu = ab/p, K_AB = exp(-mu R_AB^2), rho = pq/(p+q).
Higher angular momentum follows from differentiating with respect to the
centre: g_{l+1_i} = (d/dA_i g_l + l_i g_{l-1_i}) / (2 alpha), applied here
symbolically with sympy (dF_m/dT = -F_{m+1}) and evaluated in mpmath.  This
shares nothing with the McMurchie-Davidson code it checks.
"""

from __future__ import annotations

import functools

import mpmath
import sympy as sp


class Boys(sp.Function):
    nargs = 2

    def fdiff(self, argindex=2):
        m, T = self.args
        return -Boys(m + 1, T)


def mp_boys(m, T):
    m = int(m)
    T = mpmath.mpf(T)
    if T == 0:
        return mpmath.mpf(1) / (2 * m + 1)
    return mpmath.gammainc(m + mpmath.mpf(1) / 2, 0, T) / (2 * T ** (m + mpmath.mpf(1) / 2))


CEN = {k: sp.symbols(f"{k}x {k}y {k}z", real=True) for k in "ABCDN"}
EXP = {k: sp.Symbol(f"e{k}", positive=True) for k in "ABCD"}


def _r2(U, V):
    return sum((u - v) ** 2 for u, v in zip(U, V))


def _pair(a, A, b, B):
    p = a + b
    mu = a * b / p
    P = [(a * u + b * v) / p for u, v in zip(A, B)]
    return p, mu, P, sp.exp(-mu * _r2(A, B))


def s_overlap():
    p, mu, P, K = _pair(EXP["A"], CEN["A"], EXP["B"], CEN["B"])
    return (sp.pi / p) ** sp.Rational(3, 2) * K


def s_kinetic():
    p, mu, P, K = _pair(EXP["A"], CEN["A"], EXP["B"], CEN["B"])
    return mu * (3 - 2 * mu * _r2(CEN["A"], CEN["B"])) * (sp.pi / p) ** sp.Rational(3, 2) * K


def s_nuclear():
    p, mu, P, K = _pair(EXP["A"], CEN["A"], EXP["B"], CEN["B"])
    return 2 * sp.pi / p * K * Boys(0, p * _r2(P, CEN["N"]))


def s_eri():
    p, _, P, Kab = _pair(EXP["A"], CEN["A"], EXP["B"], CEN["B"])
    q, _, Q, Kcd = _pair(EXP["C"], CEN["C"], EXP["D"], CEN["D"])
    rho = p * q / (p + q)
    return 2 * sp.pi ** sp.Rational(5, 2) / (p * q * sp.sqrt(p + q)) * Kab * Kcd * \
        Boys(0, rho * _r2(P, Q))


def raise_l(expr_of, centre: str, l: tuple):
    """Integral with Cartesian powers ``l`` on ``centre`` from the l = 0 form
    ``expr_of()`` (a memoised callable of the lower tuples)."""
    alpha = EXP[centre]
    X = CEN[centre]

    @functools.lru_cache(maxsize=None)
    def f(t):
        if min(t) < 0:
            return sp.Integer(0)
        if sum(t) == 0:
            return expr_of()
        i = next(k for k in range(3) if t[k] > 0)
        lo = list(t)
        lo[i] -= 1
        lo2 = list(t)
        lo2[i] -= 2
        return (sp.diff(f(tuple(lo)), X[i]) + (t[i] - 1) * f(tuple(lo2))) / (2 * alpha)

    return f(tuple(l))


def build(base, tuples: dict):
    """Apply raise_l for each centre in ``tuples`` (e.g. {"A": (1,0,0)})."""
    expr = base
    for c, t in tuples.items():
        prev = expr
        expr = raise_l(lambda e=prev: e, c, t)
    return expr


def evaluate(expr, values: dict):
    """Evaluate at {symbol name: value} with mpmath (Boys via gammainc)."""
    syms = sorted(expr.free_symbols, key=lambda s: s.name)
    fn = sp.lambdify(syms, expr, modules=[{"Boys": mp_boys}, "mpmath"])
    return fn(*[mpmath.mpf(values[s.name]) for s in syms])
