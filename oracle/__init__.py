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
projectors by Loewdin orthogonalization), Eqs. 14-18
(q-specific Sternheimer equation, perturbing potential, valence and
conduction projectors, the alpha shift).  Each function cites the passage it
follows.
"""
from .hp_oracle import Oracle, ScfParams, hubbard_params, assemble_chi, nearest_neighbours, loewdin, ortho_atomic_phi
from . import pz81

__all__ = ["Oracle", "ScfParams", "hubbard_params", "assemble_chi", "nearest_neighbours", "loewdin",
           "ortho_atomic_phi", "pz81"]
