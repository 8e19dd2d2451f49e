"""Plain FP64 CPU oracle for batched RHF energies and forces.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  It
shares no code with the HIP path (``paper_1601_02713_amd``) and never imports
it; the two meet only in the seeded inputs of ``inputs/``.

Contents
  mdints.c   McMurchie-Davidson integrals, direct J/K, gradient terms (C, OpenMP)
  basis.py   shells and normalisation from a basis JSON file
  rhf.py     SCF (core guess, Pulay DIIS, Loewdin orthogonalisation) and
             analytic gradient assembly
  mlp.py     numpy FP64 forward/backward/Adam of the density-guess MLP

The paper (Section 3.1) names a Gaussian-basis SCF with analytic BO forces,
a density threshold of 1e-6 and an integral cutoff of 1e-12; everything else
is textbook and cited where it is written.
"""

from .basis import build_basis  # noqa: F401
from .rhf import (  # noqa: F401
    boys,
    one_electron,
    eri_tensor,
    eri_quartet,
    schwarz,
    jk,
    jk_pairs,
    jk_sample,
    nuclear_repulsion,
    scf,
    gradient,
    fock_energy,
)
