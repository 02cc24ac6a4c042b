"""Pins of the oracle's metallic path (fractional occupations with cold smearing; the paper's
generalization of Eq. 15 to metals) against references that do not reuse its arithmetic:
  * the smearing functions: the occupation integrates the delta function (quadrature), the
    occupations sum to one band, and the split step satisfies step(x) + step(-x) = 1;
  * the Sternheimer solution of every kept band at q != 0 equals the direct sum over the
    whole spectrum of (f_i - f_j)/(e_i - e_j) theta_ji |u_j><u_j|dV|u_i> (brute force on the
    dense Hamiltonian), which is what the projected equation stands for;
  * chi and chi0 at Gamma (where the Fermi level moves) against finite differences of the
    self-consistent smeared ground state with a fixed electron count (Eq. 7 by definition);
  * the generator's states are eigenstates of the oracle's Hamiltonian.
"""
import functools
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from oracle.hp_oracle import cold_delta, cold_occupation, smooth_step
from conftest import ground_state

TIGHT = oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11)


def test_cold_smearing_functions():
    for x in (-3.0, -0.7, 0.0, 0.4, 2.5):
        val, _ = quad(lambda t: float(cold_delta(t)), -12.0, x, epsabs=1e-14, epsrel=1e-13)
        assert abs(val - float(cold_occupation(x))) < 1e-12
    assert abs(float(cold_occupation(12.0)) - 1.0) < 1e-14 and abs(float(cold_occupation(-12.0))) < 1e-14
    x = np.linspace(-4, 4, 17)
    assert np.abs(smooth_step(x) + smooth_step(-x) - 1.0).max() < 1e-15
    # closed form at x = 0: u = -1/sqrt(2), occupation (1 + erf(u))/2 + exp(-u^2)/sqrt(2 pi)
    assert abs(float(cold_occupation(0.0)) - (0.5 * (1 + math.erf(-1 / math.sqrt(2)))
                                              + math.exp(-0.5) / math.sqrt(2 * math.pi))) < 1e-15


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


@pytest.mark.parametrize("name", ["sc1_gamma_metal", "sc1_k211_metal"])
def test_metal_states_and_occupations(name):
    gs = ground_state(name)
    o = orc(name)
    assert o.metal and gs.degauss == 0.01
    for ie, e in enumerate(gs.kpts):
        assert np.abs(o.h_apply(ie, e.u) - e.eps[:, None] * e.u).max() < 1e-9
    n_el = sum(2.0 * o.kpts[ik].weight * o.f[ik].sum() for ik in o.mesh)
    assert abs(n_el - 15.0) < 1e-9
    assert any(((f > 0.05) & (f < 0.95)).any() for f in o.f)      # a band crosses the Fermi level


def test_metal_sternheimer_equals_sum_over_states():
    o = orc("sc1_k211_metal")
    q = np.array([0.5, 0.0, 0.0])
    rng = np.random.default_rng(2)
    dv = 0.05 * (rng.standard_normal(o.fft) + 1j * rng.standard_normal(o.fft))
    for ik in o.mesh:
        j, _ = o.kq_entry(ik, q)
        x, _ = o.solve(ik, q, o.rhs(ik, q, 0, dv), None, oracle.ScfParams(cg_tol=1e-14))
        # brute force: the whole spectrum at k+q
        w, V = np.linalg.eigh(o.h_dense(j))
        U = V.T
        fj = cold_occupation((o.efermi - w) / o.degauss)
        ei = o.kpts[ik].eps
        fi = o.f[ik]
        X = o.perturbed_vectors(ik, q, 0, dv)
        M = X @ U.conj().T                              # M[i, j] = <u_j|dV|u_i>
        d = ei[:, None] - w[None, :]
        F = (fi[:, None] - fj[None, :]) / d             # no equal energies across k and k+q here
        assert np.abs(d).min() > 1e-6
        sos = (F * smooth_step(-d / o.degauss) * M) @ U
        assert np.abs(x - sos).max() < 1e-10 * np.abs(sos).max(), ik


@functools.lru_cache(maxsize=None)
def fd_chi(hxc):
    o = orc("sc1_gamma_metal")
    lam = 2.5e-4        # the partially filled band makes the response strongly nonlinear
    c1 = o.fd_occupation_response(0, lam, hxc=hxc)
    c2 = o.fd_occupation_response(0, lam / 2, hxc=hxc)
    return (4 * c2 - c1) / 3


def test_metal_chi_and_chi0_equal_finite_differences():
    r = orc("sc1_gamma_metal").scf(0, np.zeros(3), TIGHT)
    chi, chi0 = np.trace(r["dn"][0]).real, np.trace(r["dn0"][0]).real
    assert abs(chi0 - fd_chi(False)[0]) < 1e-8 * abs(chi0)
    assert abs(chi - fd_chi(True)[0]) < 1e-8 * abs(chi)


def test_metal_without_fermi_shift_misses_finite_differences():
    """The q = 0 Fermi-level term matters: dropping it moves chi0 far from the reference."""
    o = oracle.Oracle(ground_state("sc1_gamma_metal"))
    o.fermi_shift = lambda X: 0.0
    r = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-12, hxc=False))
    chi0 = np.trace(r["dn0"][0]).real
    assert abs(chi0 - fd_chi(False)[0]) > 1e-3 * abs(chi0)


def test_metal_path_with_full_bands_is_the_insulator():
    """Fermi level mid-gap, all kept bands fully occupied: the metallic right-hand side and the
    (vanishing) Fermi shift reproduce the insulating response."""
    import copy
    gs = ground_state("sc1_k211")
    g = copy.copy(gs)
    top = max(e.eps.max() for e in gs.kpts)
    nxt = min(e.eps_next for e in gs.kpts)
    g.degauss = 0.002
    g.efermi = 0.5 * (top + nxt)
    om = oracle.Oracle(g)
    assert om.metal and min(f.min() for f in om.f) > 1 - 1e-12
    p = oracle.ScfParams(cg_tol=1e-11, conv_thr_chi=1e-10, conv_thr_v=1e-8)   # same path, same stopping
    for q in ((0.0, 0, 0), (0.5, 0, 0)):
        a = om.scf(0, np.array(q), p)
        b = oracle.Oracle(gs).scf(0, np.array(q), p)
        for key in ("dn0", "dn"):
            assert np.abs(a[key] - b[key]).max() < 1e-10 * np.abs(b[key]).max(), (q, key)


def test_metal_q0_self_consistency_converges_on_a_k_mesh():
    """Regression: the Fermi-level shift must keep the response linear over the complex numbers
    (the mixing extrapolates with complex coefficients); taking its real part stalled the q = 0
    loop of this metal at a residual of ~1e-3."""
    o = orc("duo_k221_metal")
    r = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-10, conv_thr_chi=1e-10, conv_thr_v=1e-8, niter_max=60))
    assert r["converged"] and r["iters"] < 45
