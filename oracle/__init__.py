"""FP64 CPU oracle for the DFPT Hubbard-response path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library (no kernels, headers, tables or helpers); the only thing the two have
in common is the seeded input generator in ``synth``.

The oracle is written from the paper (Timrov, Marzari, Cococcioni, "HP - A code
for the calculation of Hubbard parameters using density-functional
perturbation theory"): Eqs. 7-9 (susceptibilities and U/V), Eq. 12
(monochromatic sum over q), Eq. 13 (response occupations), Eq. 6 (ortho-atomic
projectors by Loewdin orthogonalization), Eq. 5 (the on-site ground-state Hubbard
potential in the unperturbed Hamiltonian), the spin-resolved forms of Eqs. 3 and
10-15, fractional occupations of metallic ground states (cold smearing, the split
Sternheimer right-hand side and the Fermi-level shift at q = 0), the search for equivalent sites and the reconstruction of the response
matrices (paper, linear-response and post-processing steps), Eqs. 14-18
(q-specific Sternheimer equation, perturbing potential, valence and
conduction projectors, the alpha shift).  Each function cites the passage it
follows.
"""
from .hp_oracle import (Oracle, ScfParams, hubbard_params, assemble_chi, nearest_neighbours, loewdin,
                        ortho_atomic_phi, equivalent_sites, supercell_distances, reconstruct_chi)
from . import pz81

__all__ = ["Oracle", "ScfParams", "hubbard_params", "assemble_chi", "nearest_neighbours", "loewdin",
           "ortho_atomic_phi", "equivalent_sites", "supercell_distances", "reconstruct_chi", "pz81"]
