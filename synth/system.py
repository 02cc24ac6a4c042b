"""Synthetic periodic systems and their occupied ground states.

Everything is in Hartree atomic units.  Conventions (fixed here and used by
both consumers of these inputs):

* cell rows are the lattice vectors a1, a2, a3 (bohr); reciprocal rows
  b = 2*pi*inv(A)^T; a plane wave at k has wavevector k + G with
  G = m @ b, m an integer Miller triple;
* the basis at k is {G : |k+G|^2 / 2 <= E_cut(k)};
* a lattice-periodic function is stored by its coefficients c(G) with
  u(r) = Omega^{-1/2} sum_G c(G) exp(i G.r) and sum |c|^2 = 1;
* grid point j = (j1, j2, j3) sits at r_j = sum_i (j_i / N_i) a_i, and
  Miller index m lands on grid index m mod N;
* the local potential is a real array on that grid;
* projector tables are the lattice-periodic Bloch sums of localized
  functions f(r - tau):  fbar_k(G) = Omega^{-1/2} ftilde(k+G) exp(-i(k+G).tau)
  with ftilde(p) = 4 pi (-i)^l Y_lm(p^) int r^2 j_l(p r) R(r) dr.

The Hubbard orbitals are non-orthogonalized atomic d orbitals (the
"atomic" projector choice of the paper's section on Hubbard projectors),
R(r) = N r^2 exp(-zeta r).  The Kleinman-Bylander projectors have Gaussian
radial parts r^l exp(-r^2 / 2 s^2), l = 0 and l = 1, normalized to one.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Specifications of the workloads
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class SystemSpec:
    """Shape of one synthetic workload (sizes and value distributions)."""

    name: str
    cfg_id: int                      # entropy for the seed sequence
    cell: Tuple[float, float, float]  # orthorhombic edge lengths (bohr)
    n_atoms: int
    n_hub: int                       # the first n_hub atoms carry d manifolds
    fft: Tuple[int, int, int]
    ecut: float                      # Ha
    n_occ: int
    kmesh: Tuple[int, int, int]
    qmesh: Tuple[int, int, int]
    min_sep: float = 2.5             # minimum image distance between atoms (bohr)
    fixed_frac: Optional[Tuple[Tuple[float, float, float], ...]] = None
    ecut_jitter: float = 0.0         # relative cutoff jitter drawn per {k,-k} pair
    base: Optional[str] = None       # replicate this spec ...
    rep: Tuple[int, int, int] = (1, 1, 1)  # ... this many times
    n_guard: int = 8                 # extra bands solved to measure the gap
    gap_min: float = 0.02            # Ha, required between band n_occ and n_occ+1
    depth: Tuple[float, float] = (1.0, 3.0)    # Gaussian well depths (Ha)
    width: Tuple[float, float] = (0.6, 1.2)    # Gaussian widths (bohr)
    n_gauss: int = 3
    center_jitter: float = 0.5
    noise: float = 0.01              # Ha, white noise amplitude on the grid
    zeta: Tuple[float, float] = (1.0, 1.5)     # d-orbital decay (1/bohr)
    kb_s: Tuple[float, float] = (0.5, 1.0)     # KB Gaussian widths (bohr)
    kb_d: Tuple[float, float] = (0.5, 2.0)     # KB strengths (Ha)
    max_attempts: int = 40
    # collinear spin polarization: V_up/dn = V_loc -/+ spin_field sum_I sign_I g_I(r), with
    # g_I a periodic Gaussian of width spin_width on Hubbard site I and sign_I from
    # spin_signs (default alternating +1, -1, ...: antiferromagnetic order); 0 = unpolarized
    spin_field: float = 0.0
    spin_width: float = 0.8
    spin_signs: Optional[Tuple[int, ...]] = None
    # ground-state Hubbard potential (on-site U, Ha): one DFT+U step, M^{I s} =
    # hub_u0 (delta/2 - n^{I s}) from the occupations of the plain solution, then the
    # occupied states of H + sum_I M^I |phi^I><phi^I|; 0 = plain DFT ground state
    hub_u0: float = 0.0
    # metallic ground state: Marzari-Vanderbilt (cold) smearing of width degauss (Ha) and
    # n_el electrons per cell; n_occ is then the number of bands kept (partially occupied
    # ones included); 0 = insulator with 2 n_occ electrons
    degauss: float = 0.0
    n_el: float = 0.0
    # eigen-residual the iterative solver converges the occupied states to; the olivine-shaped
    # cells use 1e-12 so that states built on different devices (or thread counts) agree to
    # far below the 1e-10 parity bar (their difference is ~ residual / gap)
    gs_tol: float = 1e-10


SPECS = {}


def _reg(s: SystemSpec) -> SystemSpec:
    SPECS[s.name] = s
    return s


# The tiny simple-cubic case: 8 bohr cube, one atom with a d manifold, ~500 PWs
# (515 at Gamma for E_cut = 7.75 Ha), FFT 24^3, Gamma only, q = 0, 8 bands.
SC1 = _reg(SystemSpec(name="sc1_gamma", cfg_id=0, cell=(8.0, 8.0, 8.0), n_atoms=1, n_hub=1,
                      fft=(24, 24, 24), ecut=7.75, n_occ=8, kmesh=(1, 1, 1), qmesh=(1, 1, 1),
                      fixed_frac=((0.0, 0.0, 0.0),)))
# The same cell sampled with k and q meshes 2x1x1, and its 2x1x1 supercell at Gamma:
# the monochromatic q-sum must reproduce the supercell response.
SC1_K2 = _reg(replace(SC1, name="sc1_k211", kmesh=(2, 1, 1), qmesh=(2, 1, 1)))
SC2_SUPER = _reg(replace(SC1, name="sc1_super211", cell=(16.0, 8.0, 8.0), n_atoms=2, n_hub=2,
                         fft=(48, 24, 24), n_occ=16, base="sc1_k211", rep=(2, 1, 1)))
SC1_K22 = _reg(replace(SC1, name="sc1_k221", kmesh=(2, 2, 1), qmesh=(2, 2, 1)))
SC1_K3 = _reg(replace(SC1, name="sc1_k311", kmesh=(3, 1, 1), qmesh=(3, 1, 1)))
SC4_SUPER = _reg(replace(SC1, name="sc1_super221", cell=(16.0, 16.0, 8.0), n_atoms=4, n_hub=4,
                         fft=(48, 48, 24), n_occ=32, base="sc1_k221", rep=(2, 2, 1)))
# A small three-atom, two-site orthorhombic cell for GPU parity: ragged PW counts,
# several k-points, a q-mesh with k+q off the k-mesh, band count not a tile multiple.
DUO = _reg(SystemSpec(name="duo_k221", cfg_id=7, cell=(10.0, 7.5, 7.0), n_atoms=3, n_hub=2,
                      fft=(30, 24, 24), ecut=10.0, n_occ=12, kmesh=(2, 3, 1), qmesh=(1, 2, 1),
                      min_sep=2.5, depth=(5.5, 6.5), width=(0.55, 0.65), center_jitter=0.15,
                      kb_d=(0.2, 0.6)))
# The two-site cell on a grid with odd edges (25 = 5 x 5 along y, 27 = 9 x 3 along z) and no
# compile-time plane or stick transform: the runtime-size kernels with odd radix chains.
DUO_ODD = _reg(replace(DUO, name="duo_odd", fft=(30, 25, 27)))
# Olivine-shaped cell: 19.6 x 11.3 x 8.9 bohr, 28 atoms, 4 d sites, ~10^4 PWs,
# FFT 72x45x40, 112 bands, k 2x3x4, q 1x2x2.
# Each atom's well (three narrow Gaussians, 5.5-6.5 Ha deep) binds one s and three p
# states well below its other levels, so 28 atoms fill 112 bands below a gap.
OLIVINE = _reg(SystemSpec(name="olivine28", cfg_id=1, cell=(19.6, 11.3, 8.9), n_atoms=28, n_hub=4,
                          fft=(72, 45, 40), ecut=22.45, n_occ=112, kmesh=(2, 3, 4), qmesh=(1, 2, 2),
                          depth=(5.5, 6.5), width=(0.55, 0.65), center_jitter=0.15, kb_d=(0.2, 0.6),
                          gs_tol=1e-12))
# The same cell (same seed: atoms, wells, noise, projectors) sampled at Gamma only with a
# 1x2x1 q mesh (entries Gamma and (0, 1/2, 0)): the full-size grid, sphere and band count at
# a cost the oracle affords for a stored full-size reference.
OLIVINE_G = _reg(replace(OLIVINE, name="olivine28_gamma", kmesh=(1, 1, 1), qmesh=(1, 2, 1)))
# The same system (same seed: atoms, wells, noise, projectors) with a 4x4x2 k-mesh
# (k+q stays on the mesh) and a cutoff jittered per {k,-k} pair so that PW counts spread
# over ~9,600-10,400.
OLIVINE_K442 = _reg(replace(OLIVINE, name="olivine28_k442", cfg_id=1, kmesh=(4, 4, 2),
                            ecut_jitter=0.0265, base=None, gs_tol=1e-10))
# 2x1x1 supercell of the olivine-shaped cell: 56 atoms, 8 d sites, ~2x10^4 PWs.
# (the cutoff stays the base cell's 22.45 Ha so that the supercell is an exact replica:
# ~2x10^4 plane waves)
OLIVINE_SC = _reg(replace(OLIVINE, name="olivine56_sc211", cfg_id=4, cell=(39.2, 11.3, 8.9),
                          n_atoms=56, n_hub=8, fft=(144, 45, 40), ecut=22.45, n_occ=224,
                          base="olivine28", rep=(2, 1, 1), gs_tol=1e-10))
# Its Gamma-only form (q mesh 1x2x1): the 144x45x40 grid, ~2x10^4 plane waves and 224 bands
# for a stored full-size reference, folded from the Gamma-only primitive cell.
OLIVINE_SC_G = _reg(replace(OLIVINE_SC, name="olivine56_gamma", kmesh=(1, 1, 1), qmesh=(1, 2, 1),
                            base="olivine28_gamma", gs_tol=1e-12))
# Collinear spin-polarized variants (the same atoms and wells; an exchange field of
# 0.15 Ha on the d sites): one site (polarized), two sites and the olivine-shaped cell
# with antiferromagnetic order (+, -, +, - over the d sites; equal electron counts per
# spin, zero net moment).
SC1_FM = _reg(replace(SC1, name="sc1_gamma_spin", spin_field=0.15, spin_signs=(1,)))
DUO_AFM = _reg(replace(DUO, name="duo_k221_afm", spin_field=0.15))
OLIVINE_AFM = _reg(replace(OLIVINE, name="olivine28_afm", spin_field=0.15, gs_tol=1e-10))
# its Gamma-only form (entries Gamma and (0, 1/2, 0) per spin): full-size checks of the
# spin-resolved kernels at a small ground-state cost
OLIVINE_AFM_G = _reg(replace(OLIVINE_AFM, name="olivine28_afm_gamma", kmesh=(1, 1, 1), qmesh=(1, 2, 1)))
# Ground states with an on-site Hubbard potential (U = 0.15 Ha ~ 4 eV): one site, the
# antiferromagnetic two-site cell (spin-dependent potential) and the olivine-shaped cell;
# and a 2x1x1 replica of the one-site cell whose two sites are equivalent by translation.
SC1_U = _reg(replace(SC1, name="sc1_gamma_u", hub_u0=0.15))
DUO_AFM_U = _reg(replace(DUO, name="duo_k221_afm_u", spin_field=0.15, hub_u0=0.15))
OLIVINE_U = _reg(replace(OLIVINE, name="olivine28_u", hub_u0=0.15, gs_tol=1e-10))
OLIVINE_U_G = _reg(replace(OLIVINE_U, name="olivine28_u_gamma", kmesh=(1, 1, 1), qmesh=(1, 2, 1)))
# Metallic variants (15 electrons in the 8 kept bands, cold smearing 0.01 Ha): the one-site
# cell at Gamma (band 8 half filled) and on the 2x1x1 k mesh (bands 7-8 cross the Fermi level).
SC1_METAL = _reg(replace(SC1, name="sc1_gamma_metal", degauss=0.01, n_el=15.0))
SC1_K2_METAL = _reg(replace(SC1_K2, name="sc1_k211_metal", degauss=0.01, n_el=15.0))
# The olivine-shaped cell with one electron removed (223 in 112 kept bands, cold smearing
# 0.01 Ha): the top valence band crosses the Fermi level, the next band stays 1.18 Ha above.
OLIVINE_METAL = _reg(replace(OLIVINE, name="olivine28_metal", degauss=0.01, n_el=223.0, gs_tol=1e-10))
# its Gamma-only form (entries Gamma and (0, 1/2, 0)): full-size metallic checks against the
# oracle at a small ground-state cost
OLIVINE_METAL_G = _reg(replace(OLIVINE_METAL, name="olivine28_metal_gamma", kmesh=(1, 1, 1), qmesh=(1, 2, 1),
                               gs_tol=1e-12))
# The two-site cell with one electron removed (23 in 12 kept bands): a metal on a 2x3x1 k mesh.
DUO_METAL = _reg(replace(DUO, name="duo_k221_metal", degauss=0.01, n_el=23.0))


def spec_by_name(name: str) -> SystemSpec:
    return SPECS[name]


# ---------------------------------------------------------------------------
# Ground-state container
# ---------------------------------------------------------------------------


@dataclass
class KEntry:
    k_frac: np.ndarray          # (3,) fractional coordinates (units of b)
    weight: float               # 1/N_k on the mesh, 0 for k+q-only entries
    ecut: float
    miller: np.ndarray          # (npw, 3) int32
    eps: np.ndarray             # (n_occ,) Ha
    u: np.ndarray               # (n_occ, npw) complex128, orthonormal rows
    beta: np.ndarray            # (n_beta, npw) complex128
    phi: np.ndarray             # (n_hub*5, npw) complex128
    eps_next: float = float("nan")   # first unoccupied eigenvalue
    resid: float = 0.0               # max eigen-residual norm of the occupied set

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])


@dataclass
class GroundState:
    spec: SystemSpec
    seed_used: int
    cell: np.ndarray            # (3,3) rows a1..a3
    fft: Tuple[int, int, int]
    vloc: np.ndarray            # (N1,N2,N3) float64
    rho0: np.ndarray            # (N1,N2,N3) float64, electrons / bohr^3
    tau: np.ndarray             # (n_atoms,3) cartesian bohr
    hub_atoms: np.ndarray       # (n_hub,) atom index of each Hubbard site
    hub_zeta: np.ndarray        # (n_hub,)
    kb_s: np.ndarray            # (n_atoms,2) widths for l=0,1
    kb_d: np.ndarray            # (n_atoms,2) strengths for l=0,1
    d_kb: np.ndarray            # (n_beta,) strength of each beta row
    n_occ: int
    kmesh: Tuple[int, int, int]
    qmesh: Tuple[int, int, int]
    kpts: List[KEntry]
    n_mesh: int
    spin_factor: int = 2
    gap: float = float("nan")
    nspin: int = 1              # 2: kpts holds a spin-up then a spin-down block of the same k
                                # list, vloc/rho0 are (2, N1, N2, N3), one electron per state
    hub_pot: Optional[np.ndarray] = None   # (nspin, n_hub, 5, 5) complex: the ground-state
                                           # Hubbard potential sum M |phi_m1><phi_m2| in H
    degauss: float = 0.0        # metallic: cold-smearing width (Ha), 0 = insulator
    efermi: float = 0.0         # metallic: Fermi energy (Ha)

    @property
    def n_hub(self) -> int:
        return int(self.hub_atoms.shape[0])

    @property
    def n_beta(self) -> int:
        return int(self.d_kb.shape[0])

    @property
    def hub_tau(self) -> np.ndarray:
        return self.tau[self.hub_atoms]

    @property
    def omega(self) -> float:
        return float(abs(np.linalg.det(self.cell)))

    @property
    def n_electrons(self) -> int:
        return self.spin_factor * self.n_occ * self.nspin

    def qpoints(self) -> np.ndarray:
        return mesh_points(self.qmesh)


# ---------------------------------------------------------------------------
# Geometry, meshes, spheres
# ---------------------------------------------------------------------------


def recip(cell: np.ndarray) -> np.ndarray:
    return 2.0 * np.pi * np.linalg.inv(cell).T


def mesh_points(mesh: Sequence[int]) -> np.ndarray:
    """Gamma-centred mesh in fractional coordinates, last index fastest."""
    n1, n2, n3 = mesh
    pts = [(i / n1, j / n2, l / n3) for i in range(n1) for j in range(n2) for l in range(n3)]
    return np.array(pts, dtype=np.float64)


def sphere(cell: np.ndarray, k_frac: np.ndarray, ecut: float, fft: Sequence[int]) -> np.ndarray:
    """Miller indices of {G : |k+G|^2/2 <= ecut}, sorted by kinetic energy then index."""
    b = recip(cell)
    gmax = math.sqrt(2.0 * ecut)
    # bound each Miller component through the dual basis
    a = cell
    rng = [int(math.ceil(gmax * np.linalg.norm(a[i]) / (2 * np.pi) + abs(k_frac[i]))) + 1 for i in range(3)]
    m1 = np.arange(-rng[0], rng[0] + 1)
    m2 = np.arange(-rng[1], rng[1] + 1)
    m3 = np.arange(-rng[2], rng[2] + 1)
    M = np.stack(np.meshgrid(m1, m2, m3, indexing="ij"), -1).reshape(-1, 3)
    p = (M + k_frac[None, :]) @ b
    kin = 0.5 * np.einsum("ij,ij->i", p, p)
    sel = kin <= ecut
    M = M[sel]
    kin = kin[sel]
    order = np.lexsort((M[:, 2], M[:, 1], M[:, 0], np.round(kin, 12)))
    M = M[order].astype(np.int32)
    for i in range(3):
        span = int(M[:, i].max() - M[:, i].min() + 1)
        if span > fft[i]:
            raise ValueError(f"FFT dimension {i} ({fft[i]}) cannot hold sphere span {span}")
    return M


def grid_points(cell: np.ndarray, fft: Sequence[int]) -> np.ndarray:
    n1, n2, n3 = fft
    f = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2, np.arange(n3) / n3,
                             indexing="ij"), -1)
    return f @ cell  # (N1,N2,N3,3)


# ---------------------------------------------------------------------------
# Radial transforms and real spherical harmonics (closed forms)
# ---------------------------------------------------------------------------


def real_ylm(l: int, p: np.ndarray) -> np.ndarray:
    """Real spherical harmonics of direction p (n,3); rows ordered
    l=0: (1); l=1: (x, y, z); l=2: (z^2, xz, yz, x^2-y^2, xy).  Zero at p = 0 for l >= 1."""
    r = np.linalg.norm(p, axis=1)
    safe = np.where(r > 0, r, 1.0)
    x, y, z = p[:, 0] / safe, p[:, 1] / safe, p[:, 2] / safe
    if l == 0:
        return np.full((1, p.shape[0]), 0.5 / math.sqrt(math.pi))
    zero = r == 0
    if l == 1:
        c = math.sqrt(3.0 / (4 * math.pi))
        out = np.stack([c * x, c * y, c * z])
    elif l == 2:
        c1 = math.sqrt(5.0 / (16 * math.pi))
        c2 = math.sqrt(15.0 / (4 * math.pi))
        c3 = math.sqrt(15.0 / (16 * math.pi))
        out = np.stack([c1 * (3 * z * z - 1.0), c2 * x * z, c2 * y * z, c3 * (x * x - y * y), c2 * x * y])
    else:
        raise ValueError(l)
    out[:, zero] = 0.0
    return out


def d_radial_ft(p: np.ndarray, zeta: float) -> np.ndarray:
    """4 pi int r^2 j_2(p r) R(r) dr for R = N r^2 exp(-zeta r), N = sqrt((2 zeta)^7 / 720)."""
    nrm = math.sqrt((2 * zeta) ** 7 / 720.0)
    return 4 * math.pi * nrm * 48.0 * zeta * p * p / (p * p + zeta * zeta) ** 4


def kb_radial_ft(p: np.ndarray, l: int, s: float) -> np.ndarray:
    """4 pi int r^2 j_l(p r) R(r) dr for R = N r^l exp(-r^2 / 2 s^2), unit norm."""
    if l == 0:
        nrm = math.sqrt(4.0 / (math.sqrt(math.pi) * s ** 3))
        return 4 * math.pi * nrm * math.sqrt(math.pi / 2) * s ** 3 * np.exp(-0.5 * (p * s) ** 2)
    if l == 1:
        nrm = math.sqrt(8.0 / (3 * math.sqrt(math.pi) * s ** 5))
        return 4 * math.pi * nrm * math.sqrt(math.pi / 2) * s ** 5 * p * np.exp(-0.5 * (p * s) ** 2)
    raise ValueError(l)


def sto_radial_ft(p: np.ndarray, l: int, zeta: float) -> np.ndarray:
    """4 pi int r^2 j_l(p r) R(r) dr for the Slater-type R = N r^l exp(-zeta r) of unit norm:
    int r^(l+2) j_l(p r) exp(-zeta r) dr = 2^(l+1) (l+1)! zeta p^l / (p^2 + zeta^2)^(l+2) and
    N^2 = (2 zeta)^(2l+3) / (2l+2)!  (l = 2 is d_radial_ft)."""
    nrm = math.sqrt((2 * zeta) ** (2 * l + 3) / math.factorial(2 * l + 2))
    return 4 * math.pi * nrm * (2 ** (l + 1)) * math.factorial(l + 1) * zeta * p ** l / (p * p + zeta * zeta) ** (l + 2)


def projector_tables(gs_like, k_frac: np.ndarray, miller: np.ndarray):
    """beta (n_beta, npw) and phi (n_hub*5, npw) at k.  beta rows: per atom, l=0 then the
    three l=1 components; phi rows: per Hubbard site, the five d components."""
    cell, tau = gs_like.cell, gs_like.tau
    omega = abs(np.linalg.det(cell))
    p = (miller + k_frac[None, :]) @ recip(cell)
    pn = np.linalg.norm(p, axis=1)
    rows = []
    for a in range(tau.shape[0]):
        ph = np.exp(-1j * (p @ tau[a]))
        for l in (0, 1):
            rad = kb_radial_ft(pn, l, gs_like.kb_s[a, l])
            y = real_ylm(l, p)
            for m in range(y.shape[0]):
                rows.append(((-1j) ** l) * y[m] * rad * ph)
    beta = np.array(rows, dtype=np.complex128) / math.sqrt(omega)
    rows = []
    for s, a in enumerate(gs_like.hub_atoms):
        ph = np.exp(-1j * (p @ tau[a]))
        rad = d_radial_ft(pn, gs_like.hub_zeta[s])
        y = real_ylm(2, p)
        for m in range(5):
            rows.append(-1.0 * y[m] * rad * ph)
    phi = np.array(rows, dtype=np.complex128).reshape(-1, p.shape[0]) / math.sqrt(omega)
    return beta, phi


# ---------------------------------------------------------------------------
# Random system construction
# ---------------------------------------------------------------------------


def _children(cfg_id: int, attempt: int):
    ss = np.random.SeedSequence([2203, 15684, cfg_id + 1000 * attempt])
    return [np.random.default_rng(c) for c in ss.spawn(6)]


def _orbital_zeta_draw(spec: SystemSpec, attempt: int, n_atoms: int) -> np.ndarray:
    # a seventh child of the system's seed sequence (the first six are untouched)
    ss = np.random.SeedSequence([2203, 15684, spec.cfg_id + 1000 * attempt])
    return np.random.default_rng(ss.spawn(7)[6]).uniform(1.0, 1.5, (n_atoms, 2))


def orbital_zeta(gs) -> np.ndarray:
    """(n_atoms, 2) exponents of every atom's s and p Slater-type orbitals (a replicated
    supercell repeats its base cell's, atom by atom)."""
    spec = gs.spec
    if spec.base is None:
        return _orbital_zeta_draw(spec, gs.seed_used, gs.tau.shape[0])
    base_spec = SPECS[spec.base]
    bat, _, _ = _draw_atoms(base_spec, gs.seed_used)
    nat = bat.tau.shape[0]
    zb = _orbital_zeta_draw(base_spec, gs.seed_used, nat)
    nimg = int(np.prod(spec.rep))
    hub_set = set(bat.hub_atoms.tolist())
    order = [a for a in list(bat.hub_atoms) + [a for a in range(nat) if a not in hub_set] for _ in range(nimg)]
    return zb[order]


def atomic_orbitals(gs, k_frac: np.ndarray, miller: np.ndarray):
    """All atomic orbitals at k, the set whose Loewdin orthogonalization gives the ortho-atomic
    Hubbard projectors (Eq. 6): per atom an s and three p Slater-type orbitals, then on Hubbard
    atoms the five d orbitals of the atomic projectors.  Returns (rows (n_atwfc, npw),
    hub_rows (n_hub*5,): the row of d orbital m of Hubbard site s at 5 s + m)."""
    cell, tau = gs.cell, gs.tau
    omega = abs(np.linalg.det(cell))
    p = (miller + np.asarray(k_frac)[None, :]) @ recip(cell)
    pn = np.linalg.norm(p, axis=1)
    zsp = orbital_zeta(gs)
    site_of = {int(a): s for s, a in enumerate(gs.hub_atoms)}
    rows = []
    hub_rows = np.zeros(5 * len(site_of), dtype=np.int32)
    y0, y1, y2 = real_ylm(0, p), real_ylm(1, p), real_ylm(2, p)
    for a in range(tau.shape[0]):
        ph = np.exp(-1j * (p @ tau[a]))
        rows.append(y0[0] * sto_radial_ft(pn, 0, zsp[a, 0]) * ph)
        rad = sto_radial_ft(pn, 1, zsp[a, 1])
        for m in range(3):
            rows.append(-1j * y1[m] * rad * ph)
        if a in site_of:
            s = site_of[a]
            rad = d_radial_ft(pn, gs.hub_zeta[s])
            for m in range(5):
                hub_rows[5 * s + m] = len(rows)
                rows.append(-1.0 * y2[m] * rad * ph)
    return np.array(rows, dtype=np.complex128) / math.sqrt(omega), hub_rows


def atomic_orbital_tables(gs):
    """atomic_orbitals of every k-entry of gs: ([rows of entry e], hub_rows)."""
    tabs = [atomic_orbitals(gs, e.k_frac, e.miller) for e in gs.kpts]
    return [t[0] for t in tabs], tabs[0][1]


def _min_image_dist(cell, f1, f2):
    d = f1 - f2
    d -= np.round(d)
    return np.linalg.norm(d @ cell)


@dataclass
class _Atoms:
    cell: np.ndarray
    tau: np.ndarray
    hub_atoms: np.ndarray
    hub_zeta: np.ndarray
    kb_s: np.ndarray
    kb_d: np.ndarray
    gauss: list          # per atom list of (center cart, depth, width)
    seed_used: int


def _draw_atoms(spec: SystemSpec, attempt: int) -> _Atoms:
    rp, rv, rn, rz, rk, rj = _children(spec.cfg_id, attempt)
    cell = np.diag(np.array(spec.cell, dtype=np.float64))
    if spec.fixed_frac is not None:
        frac = np.array(spec.fixed_frac, dtype=np.float64)
    else:
        frac = []
        tries = 0
        while len(frac) < spec.n_atoms:
            tries += 1
            if tries > 200000:
                raise RuntimeError("could not place atoms")
            f = rp.random(3)
            if all(_min_image_dist(cell, f, g) >= spec.min_sep for g in frac):
                frac.append(f)
        frac = np.array(frac)
    tau = frac @ cell
    gauss = []
    for a in range(spec.n_atoms):
        lst = []
        for _ in range(spec.n_gauss):
            d = rv.uniform(*spec.depth)
            w = rv.uniform(*spec.width)
            off = rv.uniform(-spec.center_jitter, spec.center_jitter, 3)
            lst.append((tau[a] + off, d, w))
        gauss.append(lst)
    hub_atoms = np.arange(spec.n_hub, dtype=np.int64)
    hub_zeta = rz.uniform(*spec.zeta, spec.n_hub)
    kb_s = rk.uniform(*spec.kb_s, (spec.n_atoms, 2))
    kb_d = rk.uniform(*spec.kb_d, (spec.n_atoms, 2))
    return _Atoms(cell, tau, hub_atoms, hub_zeta, kb_s, kb_d, gauss, attempt), rn, rj


def _vloc_grid(spec: SystemSpec, at: _Atoms, rn) -> np.ndarray:
    """Sum of attractive periodic Gaussians -D exp(-|r-c|^2 / 2 w^2) plus white noise.

    The cell is orthorhombic, so each Gaussian factorizes over the three axes and
    its periodic images are summed per axis out to 8 w."""
    L = np.diag(at.cell)
    if not np.allclose(at.cell, np.diag(L)):
        raise ValueError("orthorhombic cells only")
    axes = [np.arange(n) / n * L[i] for i, n in enumerate(spec.fft)]
    v = np.zeros(spec.fft)
    for lst in at.gauss:
        for (c, d, w) in lst:
            f = []
            for i in range(3):
                nimg = int(math.ceil(8 * w / L[i])) + 1
                acc = np.zeros(spec.fft[i])
                for n in range(-nimg, nimg + 1):
                    dx = axes[i] - c[i] - n * L[i]
                    m = np.abs(dx) < 8 * w
                    acc[m] += np.exp(-dx[m] ** 2 / (2 * w * w))
                f.append(acc)
            v -= d * np.einsum("i,j,k->ijk", f[0], f[1], f[2])
    v += rn.uniform(-spec.noise, spec.noise, spec.fft)
    return v


def _spin_field_grid(spec: SystemSpec, at: _Atoms) -> np.ndarray:
    """sum_I sign_I exp(-|r - tau_I|^2 / 2 w^2) over the Hubbard sites (periodic images)."""
    L = np.diag(at.cell)
    w = spec.spin_width
    signs = spec.spin_signs or tuple(1 if i % 2 == 0 else -1 for i in range(len(at.hub_atoms)))
    axes = [np.arange(n) / n * L[i] for i, n in enumerate(spec.fft)]
    out = np.zeros(spec.fft)
    for sgn, a in zip(signs, at.hub_atoms):
        c = at.tau[a]
        f = []
        for i in range(3):
            nimg = int(math.ceil(8 * w / L[i])) + 1
            acc = np.zeros(spec.fft[i])
            for n in range(-nimg, nimg + 1):
                dx = axes[i] - c[i] - n * L[i]
                m = np.abs(dx) < 8 * w
                acc[m] += np.exp(-dx[m] ** 2 / (2 * w * w))
            f.append(acc)
        out += sgn * np.einsum("i,j,k->ijk", f[0], f[1], f[2])
    return out


# ---------------------------------------------------------------------------
# Hamiltonian apply and eigensolvers (generator-side implementation)
# ---------------------------------------------------------------------------


class _Ham:
    """H = -1/2 nabla^2 + V_loc(grid) + sum_i D_i |beta_i><beta_i| on one k-sphere."""

    def __init__(self, gs_like, vloc, k_frac, miller, beta, d_kb, xp="numpy", device="cpu"):
        self.fft = tuple(vloc.shape)
        b = recip(gs_like.cell)
        p = (miller + k_frac[None, :]) @ b
        self.kin = 0.5 * np.einsum("ij,ij->i", p, p)
        self.idx = np.ravel_multi_index(tuple((miller % np.array(self.fft)).T), self.fft)
        self.npw = miller.shape[0]
        self.xp = xp
        if xp == "torch":
            import torch
            self.torch = torch
            self.dev = torch.device(device)
            self.t_kin = torch.from_numpy(self.kin).to(self.dev)
            self.t_idx = torch.from_numpy(self.idx.astype(np.int64)).to(self.dev)
            self.t_v = torch.from_numpy(np.ascontiguousarray(vloc)).to(self.dev)
            self.t_beta = torch.from_numpy(beta).to(self.dev)
            self.t_d = torch.from_numpy(d_kb.astype(np.complex128)).to(self.dev)
        else:
            self.v = vloc
            self.beta = beta
            self.d = d_kb

    def apply(self, X):
        """X: (nb, npw) rows are vectors."""
        if self.xp == "torch":
            torch = self.torch
            nb = X.shape[0]
            N = self.fft[0] * self.fft[1] * self.fft[2]
            out = torch.empty_like(X)
            chunk = max(1, min(nb, 64))
            for s in range(0, nb, chunk):
                x = X[s:s + chunk]
                g = torch.zeros((x.shape[0], N), dtype=torch.complex128, device=self.dev)
                g[:, self.t_idx] = x
                g = g.reshape(x.shape[0], *self.fft)
                r = torch.fft.ifftn(g, dim=(1, 2, 3))
                r = r * self.t_v
                g = torch.fft.fftn(r, dim=(1, 2, 3)).reshape(x.shape[0], N)
                out[s:s + chunk] = g[:, self.t_idx]
            out += X * self.t_kin
            proj = (X @ self.t_beta.conj().T.contiguous()) * self.t_d  # (nb, n_beta)
            out += proj @ self.t_beta
            return out
        nb = X.shape[0]
        g = np.zeros((nb,) + self.fft, dtype=np.complex128).reshape(nb, -1)
        g[:, self.idx] = X
        g = g.reshape((nb,) + self.fft)
        r = np.fft.ifftn(g, axes=(1, 2, 3)) * self.v
        g = np.fft.fftn(r, axes=(1, 2, 3)).reshape(nb, -1)
        out = g[:, self.idx] + X * self.kin
        out += ((X @ self.beta.conj().T) * self.d) @ self.beta
        return out


def _dense_h(gs_like, vloc, k_frac, miller, beta, d_kb):
    fft = np.array(vloc.shape)
    vhat = np.fft.fftn(vloc) / vloc.size
    dm = (miller[:, None, :] - miller[None, :, :]) % fft
    H = vhat[dm[..., 0], dm[..., 1], dm[..., 2]]
    p = (miller + k_frac[None, :]) @ recip(gs_like.cell)
    H = H + np.diag(0.5 * np.einsum("ij,ij->i", p, p))
    H = H + (beta.T * d_kb) @ beta.conj()
    return 0.5 * (H + H.conj().T)


def _lobpcg_torch(ham: _Ham, X0, nconv: int, tol: float, maxiter: int):
    torch = ham.torch
    dev = ham.dev
    X = torch.from_numpy(X0).to(dev)  # (m, npw) rows

    def orth_rows(S):
        G = S.conj() @ S.T  # (m,m) Gram of rows
        G = 0.5 * (G + G.conj().T)
        L, Q = torch.linalg.eigh(G.cpu())
        keep = L > 1e-13 * L.max()
        T = (Q[:, keep] / torch.sqrt(L[keep])).to(dev)
        return T

    T = orth_rows(X)
    X = T.T @ X
    HX = ham.apply(X)
    A = (X.conj() @ HX.T).cpu()
    A = 0.5 * (A + A.conj().T)
    th, C = torch.linalg.eigh(A)
    C = C.to(dev)
    X = C.T @ X
    HX = C.T @ HX
    th = th.to(dev)
    m = X.shape[0]
    P = None
    HP = None
    kin = ham.t_kin
    it = 0
    rn = None
    for it in range(maxiter):
        R = HX - th[:, None] * X
        rn = torch.linalg.norm(R, dim=1)
        if float(rn[:nconv].max()) < tol:
            break
        # preconditioner: Teter-like diagonal scaling against the kinetic energy
        ek = torch.clamp(th.real, min=0.0)[:, None]
        den = 1.0 + torch.clamp(kin[None, :] - th[:, None].real, min=0.0) + 0.0 * ek
        W = R / den
        # orthogonalize W against X twice, normalize rows
        for _ in range(2):
            W = W - (W.conj() @ X.T).conj() @ X
        W = W / torch.clamp(torch.linalg.norm(W, dim=1, keepdim=True), min=1e-300)
        HW = ham.apply(W)
        if P is not None:
            S = torch.cat([X, W, P], 0)
            HS = torch.cat([HX, HW, HP], 0)
        else:
            S = torch.cat([X, W], 0)
            HS = torch.cat([HX, HW], 0)
        T = orth_rows(S)
        S2 = T.T @ S
        HS2 = T.T @ HS
        A = (S2.conj() @ HS2.T).cpu()
        A = 0.5 * (A + A.conj().T)
        th_all, C = torch.linalg.eigh(A)
        C = C[:, :m].to(dev)
        Cs = T @ C  # coefficients in the original S rows
        Xn = Cs.T @ S
        HXn = Cs.T @ HS
        Cwp = Cs[m:]
        if P is not None:
            P = Cwp.T @ torch.cat([W, P], 0)
            HP = Cwp.T @ torch.cat([HW, HP], 0)
        else:
            P = Cwp.T @ W
            HP = Cwp.T @ HW
        X, HX = Xn, HXn
        th = th_all[:m].to(dev)
        # re-orthonormalize X occasionally to keep rounding at bay
        if it % 10 == 9:
            T = orth_rows(X)
            X = T.T @ X
            HX = T.T @ HX
            A = (X.conj() @ HX.T).cpu()
            A = 0.5 * (A + A.conj().T)
            th2, C2 = torch.linalg.eigh(A)
            C2 = C2.to(dev)
            X = C2.T @ X
            HX = C2.T @ HX
            th = th2.to(dev)
            P = None
            HP = None
    # final Rayleigh-Ritz polish
    T = orth_rows(X)
    X = T.T @ X
    HX = ham.apply(X)
    A = (X.conj() @ HX.T).cpu()
    A = 0.5 * (A + A.conj().T)
    th, C = torch.linalg.eigh(A)
    C = C.to(dev)
    X = C.T @ X
    HX = C.T @ HX
    th = th.to(dev)
    R = HX - th[:, None] * X
    rn = torch.linalg.norm(R, dim=1)
    return th.cpu().numpy(), X.cpu().numpy(), rn.cpu().numpy(), it


# ---------------------------------------------------------------------------
# Ground-state assembly
# ---------------------------------------------------------------------------


def _k_entries(spec: SystemSpec):
    """Mesh k-points followed by the extra k+q entries not on the mesh (unreduced k+q)."""
    mesh = mesh_points(spec.kmesh)
    qs = mesh_points(spec.qmesh)
    extra = []

    def on_mesh(k):
        d = k[None, :] - mesh
        return np.any(np.all(np.abs(d - np.round(d)) < 1e-9, axis=1))

    def known(k):
        return any(np.all(np.abs((k - e) - np.round(k - e)) < 1e-9) for e in extra)

    for q in qs:
        for k in mesh:
            kq = k + q
            if not on_mesh(kq) and not known(kq):
                extra.append(kq)
    return mesh, np.array(extra).reshape(-1, 3)


def _ecut_for(spec: SystemSpec, k_frac: np.ndarray, rj) -> float:
    """Cutoff per k; jittered per {k,-k} pair (keyed by the pair's canonical representative)."""
    if spec.ecut_jitter == 0.0:
        return spec.ecut
    raise RuntimeError("use _jitter_table")


def _pair_key(k):
    a = tuple(np.round((k % 1.0) * 1e6).astype(np.int64) % 1000000)
    b = tuple(np.round(((-k) % 1.0) * 1e6).astype(np.int64) % 1000000)
    return min(a, b)


def build_ground_state(spec: SystemSpec | str, *, backend: str = "auto", device: str = "cpu",
                       tol: Optional[float] = None, verbose: bool = False) -> GroundState:
    """Build the seeded synthetic system and its occupied eigenpairs at every k-entry.

    backend: 'dense' (numpy eigh; small spheres), 'lobpcg' (block iterative solver on
    torch, CPU or GPU device), or 'auto' (dense below 3000 plane waves).  tol: eigen-residual
    of the iterative solver (default: the spec's gs_tol)."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    if tol is None:
        tol = spec.gs_tol
    if spec.base is not None:
        return _build_replicated(spec, backend=backend, device=device, tol=tol, verbose=verbose)
    last_err = None
    for attempt in range(spec.max_attempts):
        at, rn, rj = _draw_atoms(spec, attempt)
        vloc = _vloc_grid(spec, at, rn)
        gs = _solve_all(spec, at, vloc, rj, backend, device, tol, verbose)
        if gs is not None:
            return gs
        last_err = attempt
    raise RuntimeError(f"{spec.name}: no gapped system within {spec.max_attempts} seeds ({last_err})")


class _KSolver:
    """Occupied (plus guard) eigenpairs at arbitrary k for one system; reuses time-reversal
    partners (c_{-k}(G) = conj(c_k(-G)), same energies) and carries the last solution over
    as the initial subspace of the next k."""

    def __init__(self, shell, vloc, d_kb, nb, nconv, backend, device, tol, verbose, fft, spec):
        self.shell, self.vloc, self.d_kb = shell, vloc, d_kb
        self.nb, self.nconv = nb, nconv
        self.backend, self.device, self.tol, self.verbose = backend, device, tol, verbose
        self.fft, self.spec = fft, spec
        self.solved = {}
        self.last_full = None

    def solve(self, k, miller, beta):
        """Returns (eps_all[nb], U[nb, npw], max residual of the first nconv-1 states)."""
        for kk, (m_p, e_p, u_p, r_p) in self.solved.items():
            kp = np.array(kk)
            s = k + kp
            if np.all(np.abs(s - np.round(s)) < 1e-9):
                g0 = np.round(k + kp).astype(np.int64)   # k = -kp + g0
                lut = {tuple(m): j for j, m in enumerate(m_p)}
                src = np.array([lut[tuple(-m - g0)] for m in miller])
                return e_p, np.conj(u_p[:, src]), r_p
        npw = miller.shape[0]
        use_dense = self.backend == "dense" or (self.backend == "auto" and npw <= 3000)
        if use_dense:
            H = _dense_h(self.shell, self.vloc, k, miller, beta, self.d_kb)
            w, V = np.linalg.eigh(H)
            eps_all = w[:self.nb]
            U = V[:, :self.nb].T.copy()
            m = self.nconv - 1
            res = float(np.linalg.norm(H @ U[:m].T - U[:m].T * eps_all[:m], axis=0).max())
        else:
            ham = _Ham(self.shell, self.vloc, k, miller, beta, self.d_kb, xp="torch", device=self.device)
            if self.last_full is not None:
                X0 = _map_guess(self.last_full, miller)
            else:
                X0 = _initial_guess(self.shell, self.vloc, k, miller, beta, self.d_kb, self.nb, self.spec)
            eps_all, U, rn, nit = _lobpcg_torch(ham, X0, self.nconv, self.tol, 400)
            self.last_full = (miller, U)
            res = float(rn[:self.nconv - 1].max())
            if self.verbose:
                print(f"  k={np.round(k, 4)} npw={npw} lobpcg iters={nit} resid={res:.2e}", flush=True)
        self.solved[tuple(np.asarray(k, dtype=np.float64))] = (miller, eps_all, U, res)
        return eps_all, U, res


def _d_kb_of(at):
    return np.concatenate([[at.kb_d[a, 0], at.kb_d[a, 1], at.kb_d[a, 1], at.kb_d[a, 1]]
                           for a in range(at.tau.shape[0])])


def _finish_metal(spec, at, vloc, entries, n_mesh, verbose, d_kb):
    """Metallic ground state: Fermi level of n_el electrons over the kept bands (and the first
    excluded band, which must stay empty: occupation below 1e-12 and at least 6 widths above
    every band with occupation above 1e-12, else None and the next seed is tried); density
    with the cold-smearing weights."""
    sig = spec.degauss
    ef = _fermi_level([np.append(e.eps, e.eps_next) for e in entries[:n_mesh]],
                      [e.weight for e in entries[:n_mesh]], spec.n_el, sig)
    top = max(float(e.eps[_cold_occupation((ef - e.eps) / sig) > 1e-12].max()) for e in entries)
    nxt = min(e.eps_next for e in entries)
    if _cold_occupation((ef - nxt) / sig) > 1e-12 or nxt - top < 6 * sig:
        if verbose:
            print(f"{spec.name} attempt {at.seed_used}: first excluded band occupied or too close", flush=True)
        return None  # the next seed is tried
    omega = abs(np.linalg.det(at.cell))
    fft = tuple(spec.fft)
    N = int(np.prod(fft))
    rho = np.zeros(fft)
    for e in entries[:n_mesh]:
        f = _cold_occupation((ef - e.eps) / sig)
        idx = np.ravel_multi_index(tuple((e.miller % np.array(fft)).T), fft)
        g = np.zeros((e.u.shape[0], N), dtype=np.complex128)
        g[:, idx] = e.u
        r = np.fft.ifftn(g.reshape((e.u.shape[0],) + fft), axes=(1, 2, 3)) * N
        rho += 2.0 * e.weight * np.einsum("i,ixyz->xyz", f, np.abs(r) ** 2) / omega
    if verbose:
        print(f"{spec.name}: e_F {ef:.6f} Ha, first excluded band {nxt - ef:.4f} Ha above", flush=True)
    return GroundState(spec=spec, seed_used=at.seed_used, cell=at.cell, fft=fft, vloc=vloc, rho0=rho, tau=at.tau,
                       hub_atoms=at.hub_atoms, hub_zeta=at.hub_zeta, kb_s=at.kb_s, kb_d=at.kb_d, d_kb=d_kb,
                       n_occ=spec.n_occ, kmesh=tuple(spec.kmesh), qmesh=tuple(spec.qmesh), kpts=entries,
                       n_mesh=n_mesh, gap=nxt - top, degauss=sig, efermi=ef)


def _finish(spec, at, vloc, entries, n_mesh, forced_gap_check, verbose, d_kb, nspin=1, hub_pot=None):
    homo = max(float(e.eps.max()) for e in entries)
    lumo = min(e.eps_next for e in entries)
    gap = lumo - homo
    if verbose:
        print(f"{spec.name} attempt {at.seed_used}: gap {gap:.4f} Ha", flush=True)
    if forced_gap_check and gap < spec.gap_min:
        return None
    fft = tuple(spec.fft)
    if nspin == 1:
        rho0 = _density(spec, at.cell, fft, entries[:n_mesh])
    else:  # one electron per state and spin channel
        nks = len(entries) // 2
        rho0 = np.stack([0.5 * _density(spec, at.cell, fft, entries[s * nks:s * nks + n_mesh]) for s in range(2)])
    return GroundState(spec=spec, seed_used=at.seed_used, cell=at.cell, fft=fft, vloc=vloc,
                       rho0=rho0, tau=at.tau, hub_atoms=at.hub_atoms, hub_zeta=at.hub_zeta,
                       kb_s=at.kb_s, kb_d=at.kb_d, d_kb=d_kb, n_occ=spec.n_occ, kmesh=tuple(spec.kmesh),
                       qmesh=tuple(spec.qmesh), kpts=entries, n_mesh=n_mesh, gap=gap,
                       spin_factor=2 if nspin == 1 else 1, nspin=nspin, hub_pot=hub_pot)


def _cold_occupation(x):
    """Marzari-Vanderbilt occupation of x = (e_F - e) / sigma: the integral of
    (1/sqrt(pi)) exp(-u^2) (1 - sqrt(2) u), u = t - 1/sqrt(2), from -infinity to x."""
    from scipy.special import erf
    u = np.asarray(x, dtype=np.float64) - 1.0 / math.sqrt(2.0)
    return 0.5 * (1.0 + erf(u)) + np.exp(-u * u) / math.sqrt(2.0 * math.pi)


def _fermi_level(eps_mesh, weights, n_el, sigma):
    """e_F with 2 sum_k w_k sum_i occ((e_F - e_ki) / sigma) = n_el (bisection)."""
    lo, hi = min(e.min() for e in eps_mesh) - 20 * sigma, max(e.max() for e in eps_mesh) + 20 * sigma

    def count(ef):
        return sum(2.0 * w * _cold_occupation((ef - e) / sigma).sum() for e, w in zip(eps_mesh, weights))

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if count(mid) < n_el:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _solve_all(spec, at, vloc, rj, backend, device, tol, verbose, forced_gap_check=True):
    mesh, extra = _k_entries(spec)
    ks = list(mesh) + list(extra)
    jit = {}
    if spec.ecut_jitter:
        keys = sorted({_pair_key(k) for k in ks})
        vals = rj.uniform(-spec.ecut_jitter, spec.ecut_jitter, len(keys))
        jit = dict(zip(keys, vals))
    d_kb = _d_kb_of(at)
    shell = _Shell(at.cell, at.tau, at.hub_atoms, at.hub_zeta, at.kb_s, at.kb_d)
    nb = spec.n_occ + spec.n_guard
    if spec.spin_field:
        m = spec.spin_field * _spin_field_grid(spec, at)
        vs = [vloc - m, vloc + m]       # spin up is attracted to the sites of sign +1
    else:
        vs = [vloc]
    def solve_block(v, mhub):
        """Entries of one spin channel; mhub (n_hub, 5, 5) adds the Hubbard potential, written
        as extra projector rows: per site M = W diag(lam) W^+, rows W^T phi with strengths lam."""
        lam = None
        if mhub is not None:
            ev = [np.linalg.eigh(mhub[s]) for s in range(mhub.shape[0])]
            lam = np.concatenate([e[0] for e in ev])
        solver = _KSolver(shell, v, d_kb if lam is None else np.concatenate([d_kb, lam]), nb, spec.n_occ + 1,
                          backend, device, tol, verbose, spec.fft, spec)
        out = []
        for i, k in enumerate(ks):
            ecut = spec.ecut * (1.0 + jit.get(_pair_key(k), 0.0))
            miller = sphere(at.cell, k, ecut, spec.fft)
            beta, phi = projector_tables(shell, k, miller)
            rows = beta
            if lam is not None:
                rows = np.concatenate([beta] + [ev[s][1].T @ phi[5 * s:5 * s + 5] for s in range(len(ev))])
            eps_all, U, res = solver.solve(np.asarray(k, dtype=np.float64), miller, rows)
            w = 1.0 / len(mesh) if i < len(mesh) else 0.0
            out.append(KEntry(k_frac=np.array(k, dtype=np.float64), weight=w, ecut=ecut, miller=miller,
                              eps=np.array(eps_all[:spec.n_occ]), u=np.ascontiguousarray(U[:spec.n_occ]),
                              beta=beta, phi=phi, eps_next=float(eps_all[spec.n_occ]), resid=res))
        return out

    blocks = [solve_block(v, None) for v in vs]
    hub_pot = None
    if spec.hub_u0:
        # occupations n^{I s}_{m1 m2} = sum_k w_k sum_v <phi_m1|u_v><u_v|phi_m2> of each spin channel
        nh = len(at.hub_atoms)
        hub_pot = np.zeros((len(vs), nh, 5, 5), dtype=np.complex128)
        for si, blk in enumerate(blocks):
            n = np.zeros((nh, 5, 5), dtype=np.complex128)
            for e in blk[:len(mesh)]:
                A = e.phi.conj() @ e.u.T
                for st in range(nh):
                    a = A[5 * st:5 * st + 5]
                    n[st] += e.weight * (a @ a.conj().T)
            hub_pot[si] = spec.hub_u0 * (0.5 * np.eye(5)[None] - n)
        blocks = [solve_block(v, hub_pot[si]) for si, v in enumerate(vs)]
    entries = [e for blk in blocks for e in blk]
    vout = vloc if len(vs) == 1 else np.stack(vs)
    if spec.degauss:
        return _finish_metal(spec, at, vout, entries, len(mesh), verbose, d_kb)
    return _finish(spec, at, vout, entries, len(mesh), forced_gap_check, verbose, d_kb, nspin=len(vs),
                   hub_pot=hub_pot)


@dataclass
class _Shell:
    cell: np.ndarray
    tau: np.ndarray
    hub_atoms: np.ndarray
    hub_zeta: np.ndarray
    kb_s: np.ndarray
    kb_d: np.ndarray


def _initial_guess(shell, vloc, k, miller, beta, d_kb, nb, spec):
    """Lowest states of H restricted to the lowest-kinetic-energy plane waves."""
    nsub = min(miller.shape[0], max(4 * nb, 2500))
    H = _dense_h(shell, vloc, k, miller[:nsub], beta[:, :nsub], d_kb)
    w, V = np.linalg.eigh(H)
    X = np.zeros((nb, miller.shape[0]), dtype=np.complex128)
    X[:, :nsub] = V[:, :nb].T
    return X


def _map_guess(last, miller):
    """Previous k-point's states carried over plane wave by plane wave (Miller index match)."""
    m_old, U_old = last
    lut = {tuple(m): j for j, m in enumerate(m_old)}
    X = np.zeros((U_old.shape[0], miller.shape[0]), dtype=np.complex128)
    for j, m in enumerate(miller):
        i = lut.get(tuple(m))
        if i is not None:
            X[:, j] = U_old[:, i]
    return X


def _density(spec, cell, fft, mesh_entries):
    """rho(r_j) = (2 / (N_k Omega)) sum_kv |sum_G c(G) e^{iG.r_j}|^2."""
    omega = abs(np.linalg.det(cell))
    N = int(np.prod(fft))
    rho = np.zeros(fft)
    for e in mesh_entries:
        idx = np.ravel_multi_index(tuple((e.miller % np.array(fft)).T), fft)
        for s in range(0, e.u.shape[0], 32):
            blk = e.u[s:s + 32]
            g = np.zeros((blk.shape[0], N), dtype=np.complex128)
            g[:, idx] = blk
            r = np.fft.ifftn(g.reshape((blk.shape[0],) + tuple(fft)), axes=(1, 2, 3)) * N
            rho += np.sum(np.abs(r) ** 2, axis=0)
    return rho * 2.0 / (len(mesh_entries) * omega)


def _build_replicated(spec, *, backend, device, tol, verbose):
    """Supercell made of spec.rep copies of the base cell (atoms, potential grid, projector
    parameters replicated exactly).  Its occupied states at a supercell k are the base cell's
    states at the folded k_p = (k + j) / rep (j over the folds), with the same coefficients on
    the supercell Miller indices m_sc = rep * m_p + j (same cutoff, so the supercell sphere is
    the union of the folded primitive spheres): no supercell eigensolve is needed."""
    base_spec = SPECS[spec.base]
    from . import cache  # the base cell of a large supercell is usually cached already
    big = base_spec.n_occ >= 100
    base = cache.load(base_spec.name) if big else None
    if base is None:  # the base cell at its own tolerance, kept for later users of it
        base = build_ground_state(base_spec, backend=backend, device=device, verbose=verbose)
        if big:
            cache.save(base)
    rep = np.array(spec.rep, dtype=np.int64)
    r1, r2, r3 = spec.rep
    cell = np.diag(np.array(spec.cell, dtype=np.float64))
    bcell = base.cell
    if abs(spec.ecut - base_spec.ecut) > 1e-12 or spec.ecut_jitter or base_spec.ecut_jitter:
        raise ValueError("a replicated supercell must keep the base cutoff")
    taus, hubs, zetas, kbs, kbd = [], [], [], [], []
    nat = base.tau.shape[0]
    imgs = [(i, j, l) for i in range(r1) for j in range(r2) for l in range(r3)]
    hub_set = set(base.hub_atoms.tolist())
    order = [(a, im) for a in list(base.hub_atoms) + [a for a in range(nat) if a not in hub_set] for im in imgs]
    for n, (a, (i, j, l)) in enumerate(order):
        taus.append(base.tau[a] + i * bcell[0] + j * bcell[1] + l * bcell[2])
        kbs.append(base.kb_s[a])
        kbd.append(base.kb_d[a])
        if a in hub_set:
            hubs.append(n)
            zetas.append(base.hub_zeta[list(base.hub_atoms).index(a)])
    at = _Atoms(cell, np.array(taus), np.array(hubs, dtype=np.int64), np.array(zetas),
                np.array(kbs), np.array(kbd), [], base.seed_used)
    vloc = np.tile(base.vloc, (r1, r2, r3))
    assert vloc.shape == tuple(spec.fft)
    # primitive solver on the base system
    bshell = _Shell(base.cell, base.tau, base.hub_atoms, base.hub_zeta, base.kb_s, base.kb_d)
    nb_p = base_spec.n_occ + base_spec.n_guard
    psolver = _KSolver(bshell, base.vloc, base.d_kb, nb_p, base_spec.n_occ + 1, backend, device, tol, verbose,
                       base_spec.fft, base_spec)
    d_kb = _d_kb_of(at)
    shell = _Shell(at.cell, at.tau, at.hub_atoms, at.hub_zeta, at.kb_s, at.kb_d)
    mesh, extra = _k_entries(spec)
    entries = []
    folds = [np.array(f) for f in imgs]
    for i, k in enumerate(list(mesh) + list(extra)):
        k = np.asarray(k, dtype=np.float64)
        miller = sphere(cell, k, spec.ecut, spec.fft)
        lut = {tuple(m): idx for idx, m in enumerate(miller)}
        cand_e, cand_u = [], []
        res = 0.0
        for j in folds:
            kp = (k + j) / rep
            mp = sphere(bcell, kp, base_spec.ecut, base_spec.fft)
            bp, _ = projector_tables(bshell, kp, mp)
            e_all, U, r = psolver.solve(kp, mp, bp)
            res = max(res, r)
            cols = np.array([lut[tuple(rep * m + j)] for m in mp])
            full = np.zeros((U.shape[0], miller.shape[0]), dtype=np.complex128)
            full[:, cols] = U
            cand_e.append(e_all)
            cand_u.append(full)
        e = np.concatenate(cand_e)
        U = np.concatenate(cand_u)
        o = np.argsort(e, kind="stable")
        e, U = e[o], U[o]
        beta, phi = projector_tables(shell, k, miller)
        w = 1.0 / len(mesh) if i < len(mesh) else 0.0
        entries.append(KEntry(k_frac=k, weight=w, ecut=spec.ecut, miller=miller, eps=e[:spec.n_occ].copy(),
                              u=np.ascontiguousarray(U[:spec.n_occ]), beta=beta, phi=phi,
                              eps_next=float(e[spec.n_occ]), resid=res))
    gs = _finish(spec, at, vloc, entries, len(mesh), False, verbose, d_kb)
    return gs
