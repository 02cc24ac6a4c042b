"""Pins of the oracle's collinear spin-polarized response (spin-resolved Eqs. 3, 10-15 with
the perturbation of Eq. 16 on both spins) against references that do not reuse the
arithmetic they pin:
  * the LSDA functional: its unpolarized limit equals the unpolarized LDA, potentials and
    kernel are derivatives of the energy density (finite differences), the kernel is
    symmetric, and both Perdew-Zunger fits are continuous with a continuous slope at
    r_s = 1 (a property the published constants satisfy);
  * the whole spin path on a polarized system against finite differences of the
    self-consistent polarized ground state (Eq. 7 by its definition), chi0 and chi;
  * a "polarized" copy of an unpolarized system (both spin blocks equal) gives the
    unpolarized response;
  * chi real symmetric after the q-sum and the Hubbard-site screening on an
    antiferromagnetic two-site system.
"""
import copy
import functools

import numpy as np
import pytest

import oracle
from oracle import pz81
from conftest import ground_state

TIGHT = oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11)


# ------------------------------------------------------------------ LSDA functional

def _densities():
    rng = np.random.default_rng(5)
    ru = 10 ** rng.uniform(-4, 0.3, 64)
    rd = ru * rng.uniform(0.2, 1.8, 64)
    return ru, rd


def test_lsda_unpolarized_limit():
    ru, _ = _densities()
    assert np.abs(pz81.eps_xc_spin(ru, ru) - pz81.eps_xc(2 * ru)).max() < 1e-15
    v = pz81.v_xc_spin(ru, ru)
    assert np.abs(v[0] - pz81.v_xc(2 * ru)).max() < 1e-14 and np.abs(v[1] - v[0]).max() < 1e-14
    f = pz81.f_xc_spin(ru, ru)
    fu = pz81.f_xc(2 * ru)
    # an equal change of both spin densities: dv = (f_uu + f_ud) drho / 2
    assert np.abs(0.5 * (f[0, 0] + f[0, 1]) - fu).max() < 1e-13 * np.abs(fu).max()


def test_lsda_potential_and_kernel_are_derivatives():
    ru, rd = _densities()
    h = 1e-6

    def energy(a, b):
        return (a + b) * pz81.eps_xc_spin(a, b)

    v = pz81.v_xc_spin(ru, rd)
    for s, (a, b) in enumerate((((1 + h) * ru, rd), (ru, (1 + h) * rd))):
        am, bm = (((1 - h) * ru, rd), (ru, (1 - h) * rd))[s]
        step = 2 * h * (ru if s == 0 else rd)
        fd = (energy(a, b) - energy(am, bm)) / step
        assert np.abs(fd - v[s]).max() < 1e-8 * np.abs(v[s]).max()
    f = pz81.f_xc_spin(ru, rd)
    for t in range(2):
        a, b = ((1 + h) * ru, rd) if t == 0 else (ru, (1 + h) * rd)
        am, bm = ((1 - h) * ru, rd) if t == 0 else (ru, (1 - h) * rd)
        step = 2 * h * (ru if t == 0 else rd)
        fd = (pz81.v_xc_spin(a, b) - pz81.v_xc_spin(am, bm)) / step
        for s in range(2):
            assert np.abs(fd[s] - f[s, t]).max() < 1e-7 * np.abs(f[s, t]).max(), (s, t)
    assert np.abs(f[0, 1] - f[1, 0]).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("prm", [pz81.U_PARAMS, pz81.P_PARAMS])
def test_pz81_fits_join_smoothly_at_rs_1(prm):
    g, b1, b2, a, b, c, d = prm
    hi = g / (1 + b1 + b2)
    lo = b + d
    assert abs(hi - lo) < 1e-3 * abs(hi)
    d_hi = -g * (0.5 * b1 + b2) / (1 + b1 + b2) ** 2
    d_lo = a + c + d
    assert abs(d_hi - d_lo) < 1e-3 * abs(d_hi)


def test_lsda_zero_below_threshold():
    z = np.array([0.0, 1e-12])
    assert np.all(pz81.f_xc_spin(z, z) == 0.0) and np.all(pz81.v_xc_spin(z, z) == 0.0)


# ----------------------------------------------------------------- response (oracle)

@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


@functools.lru_cache(maxsize=None)
def scf(name, site, q):
    return orc(name).scf(site, np.array(q, dtype=float), TIGHT)


@functools.lru_cache(maxsize=None)
def fd_chi(hxc):
    o = orc("sc1_gamma_spin")
    lam = 1e-3
    c1 = o.fd_occupation_response(0, lam, hxc=hxc)
    c2 = o.fd_occupation_response(0, lam / 2, hxc=hxc)
    return (4 * c2 - c1) / 3


def test_spin_ground_state_is_polarized():
    gs = ground_state("sc1_gamma_spin")
    assert gs.nspin == 2 and len(gs.kpts) == 2 and gs.vloc.shape == (2,) + tuple(gs.fft)
    r = gs.rho0
    for s in range(2):
        assert abs(r[s].sum() * gs.omega / r[s].size - gs.n_occ) < 1e-10
    assert np.abs(r[0] - r[1]).max() > 1e-2 * r.max()
    o = orc("sc1_gamma_spin")
    for ie in range(2):  # the states are eigenstates of their own spin's Hamiltonian
        e = gs.kpts[ie]
        res = o.h_apply(ie, e.u) - e.eps[:, None] * e.u
        assert np.abs(res).max() < 1e-9


def test_spin_chi_equals_finite_difference():
    r = scf("sc1_gamma_spin", 0, (0, 0, 0))
    chi = np.trace(r["dn"][0])
    assert abs(chi.imag) < 1e-12
    assert abs(chi.real - fd_chi(True)[0]) < 2e-8 * abs(chi.real)


def test_spin_chi0_equals_finite_difference():
    r = scf("sc1_gamma_spin", 0, (0, 0, 0))
    chi0 = np.trace(r["dn0"][0]).real
    assert abs(chi0 - fd_chi(False)[0]) < 2e-8 * abs(chi0)


def _as_polarized(gs):
    """Both spin blocks equal to the unpolarized system, one electron per state."""
    g = copy.copy(gs)
    g.kpts = list(gs.kpts) + list(gs.kpts)
    g.vloc = np.stack([gs.vloc, gs.vloc])
    g.rho0 = np.stack([0.5 * gs.rho0, 0.5 * gs.rho0])
    g.nspin = 2
    g.spin_factor = 1
    return g


def test_equal_spin_blocks_give_the_unpolarized_response():
    gs = ground_state("sc1_gamma")
    ref = oracle.Oracle(gs).scf(0, np.zeros(3), TIGHT)
    pol = oracle.Oracle(_as_polarized(gs)).scf(0, np.zeros(3), TIGHT)
    for key in ("dn0", "dn"):
        assert np.abs(pol[key] - ref[key]).max() < 1e-11 * np.abs(ref[key]).max()


def test_afm_response_matrix_symmetric_and_screened():
    o = orc("duo_k221_afm")
    chi0, chi, im, _, _ = o.response_matrix(oracle.ScfParams(cg_tol=1e-9, conv_thr_chi=1e-8, conv_thr_v=1e-6))
    assert im < 1e-7 * np.abs(chi).max()
    assert np.abs(chi0 - chi0.T).max() < 1e-7 * np.abs(chi0).max()
    assert np.abs(chi - chi.T).max() < 1e-6 * np.abs(chi).max()
    d0, d = np.diag(chi0), np.diag(chi)
    assert np.all(d0 < 0) and np.all(d < 0) and np.all(np.abs(d) < np.abs(d0))
