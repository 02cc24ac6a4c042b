"""Ortho-atomic Hubbard projectors (Eq. 6): the oracle's Loewdin orthogonalization and the
response computed with them, pinned without reusing the oracle's formula.

* orthonormality of the whole orthogonalized set;
* Loewdin orthonormalization is the polar factor of the row matrix: rows = U S V^H (SVD)
  gives U V^H (an independent routine and the textbook characterization);
* it is the orthonormal set closest to the original one: random unitary rotations of it
  never come closer;
* already orthonormal rows are returned unchanged;
* the generator's atomic orbitals: radial transforms against quadrature, and their d rows
  equal the atomic projectors;
* chi and chi0 with ortho-atomic projectors against finite differences of the ground
  state perturbed by lambda sum_m |phi~_m><phi~_m| (Eq. 7 by definition)."""
import functools
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from conftest import ground_state
from synth import system


def test_sto_radial_transforms_against_quadrature():
    for l in (0, 1, 2):
        for zeta in (1.0, 1.4):
            nrm = math.sqrt((2 * zeta) ** (2 * l + 3) / math.factorial(2 * l + 2))
            for p in (0.3, 1.1, 3.0):
                f = lambda r: r * r * special.spherical_jn(l, p * r) * nrm * r ** l * math.exp(-zeta * r)
                q = 4 * math.pi * integrate.quad(f, 0, 80, limit=400)[0]
                assert abs(system.sto_radial_ft(np.array([p]), l, zeta)[0] - q) < 1e-10 * max(1.0, abs(q))


@pytest.mark.parametrize("name", ["sc1_gamma", "duo_k221"])
def test_atomic_set_contains_the_hubbard_projectors(name):
    gs = ground_state(name)
    for e in gs.kpts[:3]:
        rows, hub = system.atomic_orbitals(gs, e.k_frac, e.miller)
        assert rows.shape == (4 * gs.tau.shape[0] + 5 * gs.n_hub, e.npw)
        np.testing.assert_allclose(rows[hub], e.phi, rtol=0, atol=1e-14)


def _rows(name, entry=0):
    gs = ground_state(name)
    e = gs.kpts[entry]
    return system.atomic_orbitals(gs, e.k_frac, e.miller)


@pytest.mark.parametrize("name,entry", [("sc1_gamma", 0), ("duo_k221", 0), ("duo_k221", 7)])
def test_loewdin_orthonormal_and_polar_factor(name, entry):
    rows, _ = _rows(name, entry)
    t = oracle.loewdin(rows)
    assert np.abs(t.conj() @ t.T - np.eye(rows.shape[0])).max() < 1e-12
    # polar factor: rows^T = U S V^H in the (column-vector) convention -> U V^H
    U, S, Vh = np.linalg.svd(rows.T, full_matrices=False)
    polar = (U @ Vh).T
    assert np.abs(t - polar).max() < 1e-12


def test_loewdin_is_the_closest_orthonormal_set():
    rows, _ = _rows("duo_k221", 2)
    t = oracle.loewdin(rows)
    d0 = np.linalg.norm(t - rows) ** 2
    rng = np.random.default_rng(5)
    n = rows.shape[0]
    for _ in range(20):
        h = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        h = 0.05 * (h - h.conj().T)          # anti-Hermitian: exp(h) is unitary
        w, v = np.linalg.eig(h)
        W = (v * np.exp(w)) @ np.linalg.inv(v)
        assert np.linalg.norm(W @ t - rows) ** 2 > d0


def test_loewdin_keeps_orthonormal_rows():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((7, 40)) + 1j * rng.standard_normal((7, 40))
    q, _ = np.linalg.qr(a.T)
    rows = q.T
    assert np.abs(oracle.loewdin(rows) - rows).max() < 1e-13


def test_ortho_atomic_projectors_differ_from_atomic_where_orbitals_overlap():
    gs = ground_state("duo_k221")
    e = gs.kpts[0]
    phi = oracle.ortho_atomic_phi(gs, e)
    assert np.abs(phi - e.phi).max() > 1e-3 * np.abs(e.phi).max()
    # still orthonormal among themselves (they are rows of an orthonormal set)
    assert np.abs(phi.conj() @ phi.T - np.eye(phi.shape[0])).max() < 1e-12


@functools.lru_cache(maxsize=None)
def _ortho_oracle():
    return oracle.Oracle(ground_state("sc1_gamma"), projectors="ortho-atomic")


@functools.lru_cache(maxsize=None)
def _fd(hxc):
    o = _ortho_oracle()
    lam = 1e-3
    c1 = o.fd_occupation_response(0, lam, hxc=hxc)
    c2 = o.fd_occupation_response(0, lam / 2, hxc=hxc)
    return (4 * c2 - c1) / 3


def test_ortho_atomic_chi_equals_finite_differences():
    o = _ortho_oracle()
    r = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11))
    chi0, chi = np.trace(r["dn0"][0]).real, np.trace(r["dn"][0]).real
    assert abs(chi - _fd(True)[0]) < 2e-8 * abs(chi)
    assert abs(chi0 - _fd(False)[0]) < 2e-8 * abs(chi0)
    # the projectors changed the answer (normalization on the cutoff sphere)
    ra = oracle.Oracle(ground_state("sc1_gamma")).scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-12))
    assert abs(np.trace(ra["dn"][0]).real - chi) > 1e-6 * abs(chi)
