"""Exchange-correlation quadrature for closed-shell B3LYP: the level of theory
of the paper's runs (Section 3.1, B3LYP/6-31G*; Section 3.2, B3LYP/6-31G**),
which replaces part of the exact exchange K of Hartree-Fock by a density
functional integrated on a molecular grid.

TEST INFRASTRUCTURE (see the package docstring).  Plain NumPy, written from
the published definitions; it shares no code with the HIP path.

Grid (the paper names none; this is the reading used by both sides):
  * per atom, n_rad radial points from Becke's mapping r = R (1 + x)/(1 - x)
    of Gauss-Chebyshev nodes of the second kind x_i = cos(i pi / (n + 1)),
    i = 1..n (Becke, J. Chem. Phys. 88, 2547 (1988)), R = 1.0 bohr for H and
    0.6 bohr for O, radial weight pi/(n+1) sin^2(.) r^2 dr/dx / sqrt(1 - x^2);
  * per radial shell, the product of n_th Gauss-Legendre nodes in cos(theta)
    and 2 n_th equally spaced phi (exact for spherical harmonics of degree
    below 2 n_th);
  * Becke's fuzzy-cell partition with three iterations of
    p(mu) = 1.5 mu - 0.5 mu^3 and no atomic size adjustment.
Functional (Stephens, Devlin, Chabalowski and Frisch 1994, closed shell,
rho = total density, sigma = |grad rho|^2):
  e_xc = 0.8 e_x^Slater + 0.72 de_x^B88 + 0.19 e_c^VWN + 0.81 e_c^LYP,
  and 0.2 of the exact exchange (F = H + J - 0.1 K + V_xc).
  * Slater exchange: -(3/4)(3/pi)^(1/3) rho^(4/3);
  * Becke 88 gradient correction (Becke 1988, beta = 0.0042), per spin
    density rho_s = rho/2 with x_s = |grad rho_s| / rho_s^(4/3):
    -beta rho_s^(4/3) x_s^2 / (1 + 6 beta x_s asinh x_s), both spins;
  * VWN correlation, the paramagnetic fit of Vosko, Wilk and Nusair (1980)
    to the random-phase-approximation correlation energy (the form the
    common definition of B3LYP takes): A = 0.0310907, x0 = -0.409286,
    b = 13.0720, c = 42.7198, x = sqrt(rs), rs = (3 / (4 pi rho))^(1/3),
    e_c/rho = A [ln(x^2/X) + 2b/Q atan(Q/(2x+b)) - b x0/X(x0) (ln((x-x0)^2/X)
    + 2(b+2x0)/Q atan(Q/(2x+b)))], X = x^2 + bx + c, Q = sqrt(4c - b^2);
  * LYP correlation (Lee, Yang and Parr 1988) in the gradient form of
    Miehlich, Savin, Stoll and Preuss (1989), a = 0.04918, b = 0.132,
    c = 0.2533, d = 0.349, here for rho_a = rho_b = rho/2.
Potentials v_rho = de/drho and v_sigma = de/dsigma come from complex-step
differentiation of the energy densities (Squire and Trapp 1998), exact to
rounding, so no derivative formula is written twice.  The matrix is
  V_mn = sum_g w_g [v_rho phi_m phi_n + 2 v_sigma grad(rho) . grad(phi_m phi_n)].
"""

from __future__ import annotations

import math

import numpy as np

from . import rhf

A0_EXACT = 0.20      # exact-exchange share
AX_B88 = 0.72        # Becke 88 gradient correction
AC_LYP = 0.81        # LYP share of the correlation (VWN the rest)
RADIUS = {1: 1.0, 8: 0.6}
RHO_MIN = 1e-14      # densities below this contribute nothing


# ------------------------------------------------------------------ the grid

def radial_grid(n: int, R: float):
    i = np.arange(1, n + 1)
    t = i * math.pi / (n + 1)
    x = np.cos(t)
    w = math.pi / (n + 1) * np.sin(t) ** 2
    r = R * (1 + x) / (1 - x)
    drdx = 2 * R / (1 - x) ** 2
    return r, w * r * r * drdx / np.sqrt(1 - x * x)


def angular_grid(n_th: int):
    ct, wt = np.polynomial.legendre.leggauss(n_th)
    nphi = 2 * n_th
    phi = 2 * math.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - ct * ct)
    u = np.stack([np.outer(st, np.cos(phi)).ravel(), np.outer(st, np.sin(phi)).ravel(),
                  np.repeat(ct, nphi)], axis=1)
    w = np.repeat(wt, nphi) * (2 * math.pi / nphi)
    return u, w


def _norm(v, axis=-1):
    """Euclidean length, written out so that complex coordinates (the
    complex-step derivatives below) pass through analytically."""
    return np.sqrt(np.sum(v * v, axis=axis))


def becke_weights(points, xyz, owner):
    """Becke partition weight of each point's own atom."""
    nat = len(xyz)
    d = _norm(points[:, None, :] - xyz[None, :, :], axis=2)    # [npt, nat]
    P = np.ones((len(points), nat), dtype=d.dtype)
    for A in range(nat):
        for B in range(nat):
            if A == B:
                continue
            mu = (d[:, A] - d[:, B]) / _norm(xyz[A] - xyz[B])
            for _ in range(3):
                mu = 1.5 * mu - 0.5 * mu ** 3
            P[:, A] *= 0.5 * (1 - mu)
    return P[np.arange(len(points)), owner] / P.sum(axis=1)


def molecular_grid(Z, xyz, n_rad=60, n_th=12):
    """Points [npt, 3] and weights [npt] of the molecular grid."""
    xyz = np.asarray(xyz)
    xyz = xyz.astype(np.result_type(xyz, float))
    u, wa = angular_grid(n_th)
    pts, wts, own = [], [], []
    for A, z in enumerate(Z):
        r, wr = radial_grid(n_rad, RADIUS[int(z)])
        pts.append((xyz[A][None, None, :] + r[:, None, None] * u[None, :, :]).reshape(-1, 3))
        wts.append((wr[:, None] * wa[None, :]).ravel())
        own.append(np.full(len(r) * len(wa), A))
    pts, wts, own = np.concatenate(pts), np.concatenate(wts), np.concatenate(own)
    return pts, wts * becke_weights(pts, xyz, own)


# ----------------------------------------------------------- basis on points

def _cart(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def _dfact(n):
    return 1.0 if n <= 0 else n * _dfact(n - 2)


def basis_values(b, points):
    """phi [npt, nbf] and grad phi [3, npt, nbf] of the oracle basis."""
    npt = len(points)
    dt = np.result_type(points, b["xyz"], float)   # complex for complex-step derivatives
    phi = np.zeros((npt, b["nbf"]), dtype=dt)
    dphi = np.zeros((3, npt, b["nbf"]), dtype=dt)
    for s in range(b["nsh"]):
        l, A = int(b["l"][s]), b["xyz"][int(b["atom"][s])]
        p0, nprim, f0 = int(b["pofs"][s]), int(b["nprim"][s]), int(b["bf"][s])
        d = points - A[None, :]
        r2 = np.sum(d * d, axis=1)
        rad = np.zeros(npt, dtype=dt)
        drad = np.zeros(npt, dtype=dt)        # d(rad)/d(r^2)
        for k in range(nprim):
            a, cf = b["exps"][p0 + k], b["coefs"][p0 + k]
            e = cf * np.exp(-a * r2)
            rad += e
            drad += -a * e
        for i, (lx, ly, lz) in enumerate(_cart(l)):
            cn = 1.0 / math.sqrt(_dfact(2 * lx - 1) * _dfact(2 * ly - 1) * _dfact(2 * lz - 1))
            ang = d[:, 0] ** lx * d[:, 1] ** ly * d[:, 2] ** lz
            phi[:, f0 + i] = cn * ang * rad
            for ax, le in enumerate((lx, ly, lz)):
                lo = [lx, ly, lz]
                lo[ax] -= 1
                dang = le * d[:, 0] ** lo[0] * d[:, 1] ** lo[1] * d[:, 2] ** lo[2] if le > 0 else 0.0
                dphi[ax, :, f0 + i] = cn * (dang * rad + ang * 2.0 * d[:, ax] * drad)
    return phi, dphi


# ------------------------------------------------------------- the functional

def e_slater(rho):
    return -0.75 * (3.0 / math.pi) ** (1.0 / 3.0) * rho ** (4.0 / 3.0)


def e_b88(rho, sigma):
    beta = 0.0042
    rs = rho / 2
    x = np.sqrt(sigma) / 2 / rs ** (4.0 / 3.0)
    return -2.0 * beta * rs ** (4.0 / 3.0) * x * x / (1 + 6 * beta * x * np.arcsinh(x))


def e_vwn(rho):
    A, x0, b, c = 0.0310907, -0.409286, 13.0720, 42.7198
    rs = (3.0 / (4.0 * math.pi * rho)) ** (1.0 / 3.0)
    x = np.sqrt(rs)
    X = x * x + b * x + c
    X0 = x0 * x0 + b * x0 + c
    Q = math.sqrt(4 * c - b * b)
    at = np.arctan(Q / (2 * x + b))
    ec = A * (np.log(x * x / X) + 2 * b / Q * at
              - b * x0 / X0 * (np.log((x - x0) ** 2 / X) + 2 * (b + 2 * x0) / Q * at))
    return rho * ec


def lyp_miehlich(ra, rb, saa, sbb, sab):
    """LYP in the Miehlich form for spin densities ra, rb and the gradient
    products saa = |grad ra|^2, sbb = |grad rb|^2, sab = grad ra . grad rb."""
    a, b, c, d = 0.04918, 0.132, 0.2533, 0.349
    rho = ra + rb
    cf = 0.3 * (3 * math.pi ** 2) ** (2.0 / 3.0)
    r13 = rho ** (-1.0 / 3.0)
    om = np.exp(-c * r13) / (1 + d * r13) * rho ** (-11.0 / 3.0)
    de = c * r13 + d * r13 / (1 + d * r13)
    s = saa + sbb + 2 * sab
    t = (ra * rb * (2 ** (11.0 / 3.0) * cf * (ra ** (8.0 / 3.0) + rb ** (8.0 / 3.0))
                   + (47.0 / 18 - 7 * de / 18) * s - (2.5 - de / 18) * (saa + sbb)
                   - (de - 11) / 9 * (ra / rho * saa + rb / rho * sbb))
         - 2.0 / 3 * rho * rho * s + (2.0 / 3 * rho * rho - ra * ra) * sbb
         + (2.0 / 3 * rho * rho - rb * rb) * saa)
    return -a * 4 / (1 + d * r13) * ra * rb / rho - a * b * om * t


def e_lyp(rho, sigma):
    """Closed shell: rho_a = rho_b = rho/2, every gradient product sigma/4."""
    a, b, c, d = 0.04918, 0.132, 0.2533, 0.349
    cf = 0.3 * (3 * math.pi ** 2) ** (2.0 / 3.0)
    r13 = rho ** (-1.0 / 3.0)
    de = c * r13 + d * r13 / (1 + d * r13)
    g = np.exp(-c * r13) / (1 + d * r13)
    return (-a * rho / (1 + d * r13)
            - a * b * g * (cf * rho - rho ** (-5.0 / 3.0) * sigma * (1.0 / 24 + 7 * de / 72)))


def e_b3lyp(rho, sigma):
    return ((1 - A0_EXACT) * e_slater(rho) + AX_B88 * e_b88(rho, sigma)
            + (1 - AC_LYP) * e_vwn(rho) + AC_LYP * e_lyp(rho, sigma))


def potentials(rho, sigma, func=e_b3lyp):
    """(e, v_rho, v_sigma) by complex-step differentiation.  The sigma step is
    relative to max(sigma, rho^(8/3)) (the scale of sigma in the reduced
    gradient), so it stays non-zero where sigma vanishes."""
    h = 1e-30
    e = func(rho, sigma)
    vr = np.imag(func(rho + 1j * h * rho, sigma + 0j)) / (h * rho)
    hs = h * np.maximum(sigma, rho ** (8.0 / 3.0))
    vs = np.imag(func(rho + 0j, sigma + 1j * hs)) / hs
    return e, vr, vs


# ------------------------------------------------------------ energy, matrix

def xc(b, P, grid=None, n_rad=60, n_th=12, func=e_b3lyp):
    """E_xc and V_xc [nbf, nbf] at density P."""
    pts, w = grid if grid is not None else molecular_grid(b["Z"], b["xyz"], n_rad, n_th)
    phi, dphi = basis_values(b, pts)
    Zm = phi @ P
    rho = np.sum(phi * Zm, axis=1)
    grad = 2.0 * np.einsum("xgm,gm->gx", dphi, Zm)
    sigma = np.sum(grad * grad, axis=1)
    keep = rho > RHO_MIN
    e, vr, vs = np.zeros_like(rho), np.zeros_like(rho), np.zeros_like(rho)
    e[keep], vr[keep], vs[keep] = potentials(rho[keep], sigma[keep], func)
    Exc = float(np.sum(w * e))
    X = (w * 0.5 * vr)[:, None] * phi + (w * 2.0 * vs)[:, None] * np.einsum("gx,xgm->gm", grad, dphi)
    V = phi.T @ X
    return Exc, V + V.T


def ks_fock_energy(b, H, P, grid, tau=1e-12, Q=None, e_nuc=None):
    """Kohn-Sham F = H + J - (a0/2) K + V_xc and E = Tr[P H] + Tr[P J]/2 -
    (a0/4) Tr[P K] + E_xc + E_nuc at density P."""
    J, K, _ = rhf.jk(b, P, tau, Q)
    Exc, V = xc(b, P, grid)
    if e_nuc is None:
        e_nuc = rhf.nuclear_repulsion(b["Z"], b["xyz"])
    F = H + J - 0.5 * A0_EXACT * K + V
    E = np.sum(P * H) + 0.5 * np.sum(P * J) - 0.25 * A0_EXACT * np.sum(P * K) + Exc + e_nuc
    return F, E


def ks_scf(b, e_tol=1e-8, comm_tol=1e-6, max_iter=100, n_rad=60, n_th=12, charge=0):
    """B3LYP SCF: core guess, Pulay DIIS on X^T(FPS - SPF)X (as rhf.scf)."""
    nocc = (int(np.sum(b["Z"])) - charge) // 2
    S, T, V = rhf.one_electron(b)
    H = T + V
    X = rhf.orthogonaliser(S)
    Q = rhf.schwarz(b)
    grid = molecular_grid(b["Z"], b["xyz"], n_rad, n_th)
    e_nuc = rhf.nuclear_repulsion(b["Z"], b["xyz"])
    P, _, _ = rhf._density(X.T @ H @ X, X, nocc)
    Fs, Es, E_prev = [], [], None
    for k in range(max_iter):
        F, E = ks_fock_energy(b, H, P, grid, 1e-12, Q, e_nuc)
        err = X.T @ (F @ P @ S - S @ P @ F) @ X
        if E_prev is not None and abs(E - E_prev) < e_tol and np.abs(err).max() < comm_tol:
            return dict(E=E, P=P, F=F, n_iter=k + 1, converged=True)
        E_prev = E
        Fs.append(F)
        Es.append(err)
        if len(Fs) > 8:
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
        P, _, _ = rhf._density(X.T @ Fbar @ X, X, nocc)
    return dict(E=E, P=P, F=F, n_iter=max_iter, converged=False)


# ------------------------------------------------------------------- forces

def xc_energy(b, P, grid, func=e_b3lyp):
    """E_xc = sum_g w_g e(rho_g, sigma_g) at density P on the given grid.  Real
    or complex: with complex atom positions (and the grid built from them) the
    imaginary part carries the complex-step derivative."""
    pts, w = grid
    phi, dphi = basis_values(b, pts)
    Zm = phi @ P
    rho = np.sum(phi * Zm, axis=1)
    grad = 2.0 * np.einsum("xgm,gm->gx", dphi, Zm)
    sigma = np.sum(grad * grad, axis=1)
    keep = np.real(rho) > RHO_MIN
    return np.sum(w[keep] * func(rho[keep], sigma[keep]))


def xc_gradient(b, P, n_rad=60, n_th=12, func=e_b3lyp, h=1e-20):
    """dE_xc/dR [natom, 3] at fixed density P: the derivative of the quadrature
    energy itself, with the grid points moving with their atoms, the Becke
    weights and the basis functions following the nuclei.  Each coordinate by
    one complex-step evaluation (Squire and Trapp 1998), exact to rounding."""
    xyz = np.asarray(b["xyz"], float)
    nat = len(xyz)
    g = np.zeros((nat, 3))
    for A in range(nat):
        for i in range(3):
            xc_ = xyz.astype(complex)
            xc_[A, i] += 1j * h
            bc = dict(b, xyz=xc_)
            E = xc_energy(bc, P, molecular_grid(b["Z"], xc_, n_rad, n_th), func)
            g[A, i] = np.imag(E) / h
    return g


def ks_gradient(b, P, F, tau=1e-12, Q=None, n_rad=60, n_th=12):
    """dE/dR of B3LYP at density P with Kohn-Sham Fock matrix F: the one-
    electron, nuclear and two-electron terms of rhf.gradient with the exact
    exchange scaled by a0 (the Pulay term W = P F P / 2 from the Kohn-Sham F),
    plus the exchange-correlation term at fixed P."""
    return (rhf.gradient(b, P, F, tau, Q, kx=A0_EXACT)
            + xc_gradient(b, P, n_rad, n_th))
