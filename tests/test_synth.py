"""Checks of the seeded input generator (shapes, closed forms, ground-state quality)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from conftest import ground_state
from synth import system as S


def test_sc1_shapes_and_gap():
    gs = ground_state("sc1_gamma")
    e = gs.kpts[0]
    assert e.npw == 515                      # ~500 plane waves at Gamma
    assert gs.fft == (24, 24, 24)
    assert gs.n_occ == 8 and gs.n_hub == 1 and gs.n_beta == 4
    assert gs.gap >= 0.02
    # orthonormal occupied states, tiny eigen-residual
    G = e.u.conj() @ e.u.T
    assert np.abs(G - np.eye(8)).max() < 1e-13
    assert e.resid < 1e-12
    # density integrates to the electron count
    assert abs(gs.rho0.sum() * gs.omega / gs.rho0.size - 16.0) < 1e-10


@pytest.mark.parametrize("name", ["sc1_k211", "sc1_k311", "duo_k221"])
def test_meshes_closed_under_inversion(name):
    gs = ground_state(name)
    mesh = [e.k_frac for e in gs.kpts[:gs.n_mesh]]
    for k in mesh:
        assert any(np.allclose(((-k - m) + 0.5) % 1.0 - 0.5, 0.0, atol=1e-12) for m in mesh)
    # every mesh k + q is loaded
    for q in gs.qpoints():
        for k in mesh:
            assert any(np.allclose(((k + q - e.k_frac) + 0.5) % 1.0 - 0.5, 0.0, atol=1e-12) for e in gs.kpts)


def test_time_reversal_partner_spheres():
    gs = ground_state("sc1_k311")
    a, b = gs.kpts[1], gs.kpts[2]          # k = 1/3 and 2/3 = -1/3 + 1
    g0 = np.round(a.k_frac + b.k_frac).astype(int)
    sa = {tuple(m) for m in a.miller}
    sb = {tuple(-m - g0) for m in b.miller}
    assert sa == sb
    np.testing.assert_allclose(a.eps, b.eps, atol=1e-12)


def test_d_radial_closed_form_against_quadrature():
    zeta = 1.23
    nrm = math.sqrt((2 * zeta) ** 7 / 720.0)
    for p in [0.0, 0.3, 1.7, 4.0]:
        f = lambda r: r * r * special.spherical_jn(2, p * r) * nrm * r * r * math.exp(-zeta * r)
        val, _ = integrate.quad(f, 0, 80, limit=400, epsabs=1e-14, epsrel=1e-13)
        ref = S.d_radial_ft(np.array([p]), zeta)[0] / (4 * math.pi)
        assert abs(val - ref) < 1e-12
    # normalization of the radial function
    val, _ = integrate.quad(lambda r: r * r * (nrm * r * r * math.exp(-zeta * r)) ** 2, 0, 80, epsabs=1e-14)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("l", [0, 1])
def test_kb_radial_closed_form_against_quadrature(l):
    s = 0.77
    nrm = {0: math.sqrt(4.0 / (math.sqrt(math.pi) * s ** 3)), 1: math.sqrt(8.0 / (3 * math.sqrt(math.pi) * s ** 5))}[l]
    rad = lambda r: nrm * r ** l * math.exp(-r * r / (2 * s * s))
    val, _ = integrate.quad(lambda r: r * r * rad(r) ** 2, 0, 40, epsabs=1e-14)
    assert abs(val - 1.0) < 1e-12
    for p in [0.0, 0.5, 2.5]:
        v, _ = integrate.quad(lambda r: r * r * special.spherical_jn(l, p * r) * rad(r), 0, 40, epsabs=1e-14, limit=200)
        ref = S.kb_radial_ft(np.array([p]), l, s)[0] / (4 * math.pi)
        assert abs(v - ref) < 1e-12


def test_real_harmonics_orthonormal():
    # Lebedev-free check: Gauss-Legendre in cos(theta) x uniform phi is exact for these degrees
    x, w = np.polynomial.legendre.leggauss(16)
    ph = np.arange(32) * 2 * np.pi / 32
    ct, pp = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(pp), st * np.sin(pp), ct], -1).reshape(-1, 3)
    wt = (w[:, None] * np.full(32, 2 * np.pi / 32)[None, :]).reshape(-1)
    Y = np.concatenate([S.real_ylm(0, dirs), S.real_ylm(1, dirs), S.real_ylm(2, dirs)])
    M = (Y * wt) @ Y.T
    assert np.abs(M - np.eye(9)).max() < 1e-13


def test_projectors_are_time_reversal_real():
    """beta and phi are Bloch sums of real functions: table(-k)(G) = conj(table(k)(-G))."""
    gs = ground_state("sc1_k311")
    a, b = gs.kpts[1], gs.kpts[2]
    g0 = np.round(a.k_frac + b.k_frac).astype(int)
    lut = {tuple(m): i for i, m in enumerate(b.miller)}
    src = np.array([lut[tuple(-m - g0)] for m in a.miller])
    np.testing.assert_allclose(a.phi, np.conj(b.phi[:, src]), atol=1e-14)
    np.testing.assert_allclose(a.beta, np.conj(b.beta[:, src]), atol=1e-14)


def test_supercell_replicates_primitive():
    gk = ground_state("sc1_k211")
    gsc = ground_state("sc1_super211")
    np.testing.assert_array_equal(gsc.vloc[:24], gk.vloc)
    np.testing.assert_array_equal(gsc.vloc[24:], gk.vloc)
    assert gsc.kpts[0].npw == sum(e.npw for e in gk.kpts)
    # the supercell Gamma spectrum is the union of the primitive k spectra
    e_sc = np.sort(gsc.kpts[0].eps)
    e_pr = np.sort(np.concatenate([e.eps for e in gk.kpts]))
    np.testing.assert_allclose(e_sc, e_pr, atol=1e-11)
