"""Seeded geometry generators for the water-cluster workloads.

Random streams: ``numpy.random.default_rng([seed, stream])`` with stream 0 for
the base geometry, 1 + b for bead b, 1000 for velocities, 3000 for cluster
sizes of the uneven batch.  Lengths are generated in Angstrom and returned in
bohr (CODATA 2018, a0 = 0.529177210903 Angstrom).
"""

from __future__ import annotations

import json
import math
import os

import numpy as np

ANGSTROM = 0.529177210903          # Angstrom per bohr
BOHR_PER_ANGSTROM = 1.0 / ANGSTROM
KB_HARTREE_PER_K = 3.166811563e-6   # Boltzmann constant in Eh/K
AMU_IN_ME = 1822.888486209          # unified atomic mass unit in electron masses
MASS_AMU = {1: 1.008, 8: 15.999}

_BASIS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "basis")
_BASIS_FILES = {"sto-3g": "sto-3g.json", "6-31g*": "6-31gs.json"}

# Water monomer: O-H 0.9572 Angstrom, H-O-H 104.52 degrees.
R_OH = 0.9572
THETA_HOH = 104.52
# Per-component Gaussian displacement of a bead, Angstrom.
SIGMA_BEAD = {1: 0.05, 8: 0.02}
LATTICE_A = 3.1          # cubic site spacing, Angstrom
MIN_INTER_ATOM = 1.6     # Angstrom, orientation redrawn below this


def basis_path(name: str) -> str:
    return os.path.join(_BASIS_DIR, _BASIS_FILES[name.lower()])


def load_basis(name: str) -> dict:
    """Parse a basis JSON file (element -> list of {l, exponents, coefficients})."""
    with open(basis_path(name)) as f:
        return json.load(f)


def water_monomer() -> tuple[np.ndarray, np.ndarray]:
    """O at the origin, the two H in the xz plane; Angstrom."""
    h = math.radians(THETA_HOH) / 2.0
    xyz = np.array([[0.0, 0.0, 0.0],
                    [R_OH * math.sin(h), 0.0, R_OH * math.cos(h)],
                    [-R_OH * math.sin(h), 0.0, R_OH * math.cos(h)]])
    return np.array([8, 1, 1], dtype=np.int32), xyz


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation matrix from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(n_waters: int, seed: int, stream: int = 0):
    """(H2O)_n on random cubic-lattice sites with random orientations.

    Sites are spaced 3.1 Angstrom (O-O >= 2.7 Angstrom by construction); a
    molecule's orientation is redrawn (up to 1000 times) while any of its atoms
    sits closer than 1.6 Angstrom to an atom of an already placed molecule.
    Returns (Z[int32 3n], xyz[3n,3] bohr), atoms ordered O,H,H per water.
    """
    rng = np.random.default_rng([seed, stream])
    k = int(math.ceil((2 * n_waters) ** (1.0 / 3.0)))
    sites = np.array([(i, j, l) for i in range(k) for j in range(k) for l in range(k)], float)
    pick = rng.choice(len(sites), size=n_waters, replace=False)
    z_mono, xyz_mono = water_monomer()
    placed = []
    for s in pick:
        centre = sites[s] * LATTICE_A
        for _ in range(1000):
            mol = xyz_mono @ random_rotation(rng).T + centre
            if not placed:
                break
            prev = np.concatenate(placed)
            d = np.linalg.norm(mol[:, None, :] - prev[None, :, :], axis=-1)
            if d.min() >= MIN_INTER_ATOM:
                break
        else:
            raise RuntimeError("could not place water without close contacts")
        placed.append(mol)
    xyz = np.concatenate(placed) - np.concatenate(placed).mean(axis=0)
    Z = np.tile(z_mono, n_waters).astype(np.int32)
    return Z, xyz * BOHR_PER_ANGSTROM


def beads(Z: np.ndarray, xyz_bohr: np.ndarray, n_beads: int, seed: int) -> np.ndarray:
    """Path-integral beads: base geometry plus an isotropic Gaussian displacement
    per Cartesian component (sigma 0.05 Angstrom for H, 0.02 for O).
    Returns [n_beads, n_atoms, 3] bohr."""
    sig = np.array([SIGMA_BEAD[int(z)] for z in Z]) * BOHR_PER_ANGSTROM
    out = np.empty((n_beads,) + xyz_bohr.shape)
    for b in range(n_beads):
        rng = np.random.default_rng([seed, 1 + b])
        out[b] = xyz_bohr + sig[:, None] * rng.standard_normal(xyz_bohr.shape)
    return out


def maxwell_boltzmann(Z: np.ndarray, n_beads: int, temperature: float, seed: int) -> np.ndarray:
    """Velocities [n_beads, n_atoms, 3] in bohr per (hbar/Eh): sigma = sqrt(kT/m)."""
    rng = np.random.default_rng([seed, 1000])
    m = np.array([MASS_AMU[int(z)] for z in Z]) * AMU_IN_ME
    sig = np.sqrt(KB_HARTREE_PER_K * temperature / m)
    v = sig[None, :, None] * rng.standard_normal((n_beads, len(Z), 3))
    # remove the centre-of-mass velocity of each bead
    vcm = (m[None, :, None] * v).sum(axis=1, keepdims=True) / m.sum()
    return v - vcm


def zundel_path(n_images: int, r_oo_angstrom: float = 2.75):
    """Proton transfer in H5O2+ (a synthetic reaction for the string method):
    O1 at the origin, O2 on +x at r_oo; in the reactant the shared proton sits
    0.99 Angstrom from O1 on the O-O axis, O1 carries two more H (H3O+
    pyramid, O-H 0.98 Angstrom, 112 degrees from the axis) and O2 a water
    (O-H 0.9572 Angstrom, H-O-H 104.52 degrees, bisector along +x).  The
    product is the reactant mirrored through the plane x = r_oo / 2 with the
    roles of the two waters exchanged, so the reaction is symmetric.
    Returns (Z[7] atoms O1, O2, H*, H, H on O1, H, H on O2; images
    [n_images, 7, 3] bohr) on the straight line from reactant to product."""
    R = r_oo_angstrom
    th = math.radians(112.0)
    u = [(math.cos(th), s * math.sin(th) * math.sin(math.radians(60.0)),
          -math.sin(th) * math.cos(math.radians(60.0))) for s in (1.0, -1.0)]
    half = math.radians(104.52 / 2)
    react = np.array([
        [0.0, 0.0, 0.0], [R, 0.0, 0.0], [0.99, 0.0, 0.0],
        [0.98 * u[0][0], 0.98 * u[0][1], 0.98 * u[0][2]],
        [0.98 * u[1][0], 0.98 * u[1][1], 0.98 * u[1][2]],
        [R + 0.9572 * math.cos(half), 0.9572 * math.sin(half), 0.0],
        [R + 0.9572 * math.cos(half), -0.9572 * math.sin(half), 0.0]])
    mirror = lambda p: np.array([R - p[0], p[1], p[2]])
    partner = [1, 0, 2, 5, 6, 3, 4]
    prod = np.array([mirror(react[partner[k]]) for k in range(7)])
    t = np.linspace(0.0, 1.0, n_images)[:, None, None]
    Z = np.array([8, 8, 1, 1, 1, 1, 1], np.int32)
    return Z, (react[None] + t * (prod - react)[None]) * BOHR_PER_ANGSTROM


def h2_molecule(r_bohr: float = 1.4):
    """H2 along z, used for the Szabo-Ostlund STO-3G worked example."""
    return np.array([1, 1], np.int32), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r_bohr]])


def _single_water(seed: int):
    rng = np.random.default_rng([seed, 0])
    z, xyz = water_monomer()
    xyz = xyz @ random_rotation(rng).T + rng.uniform(-2.0, 2.0, size=3)
    return z, xyz * BOHR_PER_ANGSTROM


def workload(name: str, n_beads: int | None = None, n_clusters: int | None = None):
    """Named synthetic workloads.

    Returns a dict with keys ``basis`` (name), ``instances`` (list of
    (Z[int32], xyz[n,3] bohr)), ``e_tol``, ``comm_tol`` and a ``label``.

    * ``h2o_sto3g``: one water, STO-3G, seeded rotation and translation.
    * ``w8_beads``: (H2O)_8, 6-31G*, 16 beads (default).
    * ``w16_beads``: (H2O)_16, 6-31G*, 32 beads.
    * ``w32_beads``: (H2O)_32, 6-31G*, 32 beads.
    * ``uneven``: 48 clusters of 2..24 waters, 4 beads each, 6-31G*.
    * ``wN``: (H2O)_N single geometry (N given in the name), 6-31G*.
    """
    if name == "h2o_sto3g":
        z, xyz = _single_water(1)
        return dict(basis="sto-3g", instances=[(z, xyz)], e_tol=1e-10, comm_tol=1e-8,
                    label="H2O RHF/STO-3G, 1 bead")
    table = {"w8_beads": (8, 16, 2), "w16_beads": (16, 32, 3), "w32_beads": (32, 32, 4)}
    if name in table:
        nw, nb, seed = table[name]
        nb = n_beads if n_beads is not None else nb
        z, xyz = water_cluster(nw, seed)
        bx = beads(z, xyz, nb, seed)
        return dict(basis="6-31g*", instances=[(z, bx[b]) for b in range(nb)],
                    e_tol=1e-8, comm_tol=1e-6,
                    label=f"(H2O){nw} RHF/6-31G*, {nb} beads")
    if name == "uneven":
        seed = 5
        nc = n_clusters if n_clusters is not None else 48
        nb = n_beads if n_beads is not None else 4
        rng = np.random.default_rng([seed, 3000])
        sizes = rng.integers(2, 25, size=nc)
        inst = []
        for c, nw in enumerate(sizes):
            z, xyz = water_cluster(int(nw), seed, stream=10000 + c)
            bx = beads(z, xyz, nb, seed * 1000 + c)
            inst += [(z, bx[b]) for b in range(nb)]
        return dict(basis="6-31g*", instances=inst, e_tol=1e-8, comm_tol=1e-6,
                    label=f"{nc} clusters of 2-24 waters, {nb} beads each, RHF/6-31G*",
                    sizes=[int(s) for s in sizes])
    if name.startswith("w") and name[1:].isdigit():
        nw = int(name[1:])
        z, xyz = water_cluster(nw, 100 + nw)
        return dict(basis="6-31g*", instances=[(z, xyz)], e_tol=1e-8, comm_tol=1e-6,
                    label=f"(H2O){nw} RHF/6-31G*")
    raise KeyError(name)
