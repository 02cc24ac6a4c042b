"""Seeded synthetic inputs for the Hubbard-response Sternheimer path.

This package builds the ground-state data that both the CPU oracle and the
GPU library consume: a periodic cell, a local potential on the FFT grid,
Kleinman-Bylander projectors, non-orthogonalized atomic d orbitals (the
Hubbard projectors), the full atomic orbital set (s, p and d) whose Loewdin
orthogonalization gives ortho-atomic projectors, optionally a collinear
spin-polarized ground state (an exchange field on the d sites, one block of
k-entries per spin), plane-wave spheres per k-point and the occupied
eigenpairs of the unperturbed Hamiltonian.  It holds none of the linear
response arithmetic: no Sternheimer solve, no response density, no
occupation response.  The eigenpairs are computed with a Hamiltonian apply
written here, independently of the oracle and of the GPU kernels.
"""
from .system import (SystemSpec, GroundState, KEntry, build_ground_state, spec_by_name, SPECS, atomic_orbitals,
                     atomic_orbital_tables)

__all__ = ["SystemSpec", "GroundState", "KEntry", "build_ground_state", "spec_by_name", "SPECS", "atomic_orbitals",
           "atomic_orbital_tables"]
