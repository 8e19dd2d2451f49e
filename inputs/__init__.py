"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no electronic-structure arithmetic: it only places atoms
(water clusters, path-integral beads, velocities) from seeded random streams
and locates the basis-set data files.  Both the oracle and the HIP path read
what it produces; neither depends on the other.

The workloads follow the path-integral MD of water clusters in the paper's
Section 3.1 (replicas of one system whose BO energies and forces are needed
every step), with RHF and Cartesian 6-31G* in place of B3LYP and spherical d.
"""

from .geometry import (  # noqa: F401
    ANGSTROM,
    BOHR_PER_ANGSTROM,
    basis_path,
    load_basis,
    water_monomer,
    random_rotation,
    water_cluster,
    beads,
    maxwell_boltzmann,
    workload,
    h2_molecule,
    zundel_path,
)
