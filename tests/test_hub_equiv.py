"""Pins of the oracle's ground-state Hubbard potential (Eq. 5, on-site part, in the
unperturbed Hamiltonian of Eq. 15) and of the equivalent-site reduction with the
reconstruction of the response matrices (paper: the search for atoms to perturb by their
occupation traces with docc_thr, and the post-processing that fills the missing columns by
comparing distances with dist_thr), against references that do not reuse the arithmetic
they pin:
  * the generator's DFT+U states (its own Hamiltonian, the potential written as
    eigen-decomposed projector rows) are eigenstates of the oracle's Hamiltonian;
  * the FFT apply with the potential equals the dense matrix;
  * chi and chi0 with the potential against finite differences of the perturbed ground
    state (Eq. 7 by definition; the potential is frozen, as the paper excludes its response);
  * replicas of a one-site cell: all sites share one class; on the 2x1x1 replica (sites
    related by a translation) the response matrix rebuilt from one perturbed site equals
    the one from perturbing every site.
"""
import functools

import numpy as np
import pytest

import oracle
from conftest import ground_state

TIGHT = oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11)


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


@pytest.mark.parametrize("name", ["sc1_gamma_u", "duo_k221_afm_u"])
def test_dftu_states_are_eigenstates_of_the_oracle_hamiltonian(name):
    gs = ground_state(name)
    assert gs.hub_pot is not None and gs.hub_pot.shape == (gs.nspin, gs.n_hub, 5, 5)
    o = orc(name)
    worst = max(np.abs(o.h_apply(ie, e.u) - e.eps[:, None] * e.u).max() for ie, e in enumerate(gs.kpts))
    assert worst < 1e-9
    # ... and not of the Hamiltonian without the potential
    p = oracle.Oracle(gs)
    p.hub_pot = None
    e = gs.kpts[0]
    assert np.abs(p.h_apply(0, e.u) - e.eps[:, None] * e.u).max() > 1e-4


def test_hubbard_potential_fft_apply_equals_dense():
    o = orc("duo_k221_afm_u")
    rng = np.random.default_rng(3)
    for ie in (0, o.nk_spin + 1):
        e = o.kpts[ie]
        X = rng.standard_normal((3, e.npw)) + 1j * rng.standard_normal((3, e.npw))
        np.testing.assert_allclose(o.h_apply(ie, X), (o.h_dense(ie) @ X.T).T, atol=1e-12)


@functools.lru_cache(maxsize=None)
def fd_chi(hxc):
    o = orc("sc1_gamma_u")
    lam = 1e-3
    c1 = o.fd_occupation_response(0, lam, hxc=hxc)
    c2 = o.fd_occupation_response(0, lam / 2, hxc=hxc)
    return (4 * c2 - c1) / 3


def test_chi_with_hubbard_potential_equals_finite_difference():
    r = orc("sc1_gamma_u").scf(0, np.zeros(3), TIGHT)
    chi, chi0 = np.trace(r["dn"][0]).real, np.trace(r["dn0"][0]).real
    assert abs(chi - fd_chi(True)[0]) < 2e-8 * abs(chi)
    assert abs(chi0 - fd_chi(False)[0]) < 2e-8 * abs(chi0)


def test_equivalent_sites_by_occupation_trace():
    tr, mom = orc("sc1_super221").site_traces()
    assert np.abs(tr - tr[0]).max() < 1e-10 and np.all(mom == 0)
    assert list(oracle.equivalent_sites(tr)) == [0, 0, 0, 0]
    tr2, _ = orc("duo_k221").site_traces()
    assert list(oracle.equivalent_sites(tr2)) == [0, 1]
    # the threshold decides: traces 1e-4 apart are one class only above that threshold
    assert list(oracle.equivalent_sites([1.0, 1.0 + 1e-4], 5e-5)) == [0, 1]
    assert list(oracle.equivalent_sites([1.0, 1.0 + 1e-4], 2e-4)) == [0, 0]


def test_supercell_distances_closed_form():
    D = oracle.supercell_distances(np.diag([16.0, 16.0, 8.0]), np.array([[0, 0, 0], [8, 0, 0], [0, 8, 0], [8, 8, 0]],
                                                                         dtype=float), (1, 1, 1))
    want = np.array([[0, 8, 8, 8 * 2 ** 0.5], [8, 0, 8 * 2 ** 0.5, 8], [8, 8 * 2 ** 0.5, 0, 8],
                     [8 * 2 ** 0.5, 8, 8, 0]])
    np.testing.assert_allclose(D, want, atol=1e-12)


def test_reconstructed_response_equals_full_response():
    """2x1x1 replica (two sites related by a lattice translation of the replica, so every
    pair at equal distance is equivalent): chi0 rebuilt from the representative's column
    equals the column of the other site computed directly."""
    gs = ground_state("sc1_super211")
    o = orc("sc1_super211")
    p = oracle.ScfParams(cg_tol=1e-13, hxc=False)
    full = np.array([np.einsum("smm->s", o.scf(sp, np.zeros(3), p)["dn0"]).real for sp in range(2)]).T
    rep = oracle.equivalent_sites(o.site_traces()[0])
    assert list(rep) == [0, 0]
    part = np.zeros_like(full)
    part[:, 0] = full[:, 0]               # only the class representative was perturbed
    rec = oracle.reconstruct_chi(part, rep, gs.cell, gs.hub_tau, gs.qmesh)
    assert np.abs(rec - full).max() < 1e-10 * np.abs(full).max()
    assert abs(full[0, 0] - full[0, 1]) > 1e-3 * abs(full[0, 0])   # the rebuilt column is not trivial


def test_reconstruction_fails_loudly_without_a_match():
    cell = np.diag([10.0, 10.0, 10.0])
    tau = np.array([[0.0, 0, 0], [3.0, 0, 0], [0, 4.0, 0]])
    chi = np.eye(3)
    with pytest.raises(ValueError):   # site 2 claimed equivalent to 0, but no pair at its distances
        oracle.reconstruct_chi(chi, [0, 1, 0], cell, tau, (1, 1, 1))
