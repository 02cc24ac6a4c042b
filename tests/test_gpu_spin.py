"""Collinear spin-polarized response on the GPU against the oracle (spin-resolved
Eqs. 3, 10-15, Eq. 16 on both spins, LSDA kernel).

Small sizes: H applies per spin block (each entry sees its own spin's potential),
first-order solves with a spin-resolved response potential, Delta n and chi against the
oracle (FP64 bar 1e-10 relative, mixed 1e-6), and an equal-spin-block copy of an
unpolarized system against the unpolarized GPU result.  Full olivine-shaped size
(antiferromagnetic order on the four d sites): sampled H applies and one spin-down
k-point's solve against the oracle's Sternheimer equation.
"""
import copy
import functools

import numpy as np
import pytest

import oracle
from conftest import ground_state

pytestmark = pytest.mark.gpu
HA_MEV = 27211.386245988
TIGHT_O = oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11)


def _hp():
    from paper_2203_15684_amd import hp
    return hp


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


def tight_gpu(precision=0, lowp=0, cg_tol=1e-13):
    return _hp().ScfParams(conv_thr_chi=1e-13, conv_thr_v=1e-11, cg_tol=cg_tol, niter_max=100, max_cg_iter=3000,
                           precision=precision, lowp_gemm=lowp)


@functools.lru_cache(maxsize=None)
def ctx(name):
    return _hp().hp_ground_state_load(ground_state(name))


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


@pytest.mark.parametrize("name", ["sc1_gamma_spin", "duo_k221_afm"])
def test_spin_apply_h_every_entry(name):
    hp = _hp()
    o = orc(name)
    rng = np.random.default_rng(1)
    for ie, e in enumerate(o.kpts):
        X = rng.standard_normal((3, e.npw)) + 1j * rng.standard_normal((3, e.npw))
        assert rel(hp.hp_apply_h(ctx(name), ie, X), o.h_apply(ie, X)) < 1e-13, f"entry {ie}"


def test_spin_first_order_solve_with_spin_resolved_potential():
    hp = _hp()
    name = "duo_k221_afm"
    o = orc(name)
    q = (0, 0.5, 0)
    rng = np.random.default_rng(4)
    dv = 0.05 * (rng.standard_normal((2,) + o.fft) + 1j * rng.standard_normal((2,) + o.fft))
    for sp in range(2):
        for k in (0, o.n_mesh - 1):
            ik = sp * o.nk_spin + k                # oracle entry index
            j, _ = o.kq_entry(ik, q)
            x_ref, _ = o.solve(ik, q, o.rhs(ik, q, 1, dv), None, oracle.ScfParams(cg_tol=1e-14))
            du, st = hp.hp_solve_first_order(ctx(name), 1, q, sp * o.n_mesh + k, dv,
                                             hp.ScfParams(cg_tol=1e-13, max_cg_iter=3000), o.kpts[j].npw)
            assert st == 0
            assert rel(du, x_ref) < 1e-10, (sp, k)


@pytest.mark.parametrize("name,site,q", [("sc1_gamma_spin", 0, (0, 0, 0)), ("duo_k221_afm", 1, (0, 0.5, 0))])
def test_spin_scf_matches_oracle(name, site, q):
    hp = _hp()
    dn0, dn, st, status = hp.hp_sternheimer_scf(ctx(name), site, q, tight_gpu())
    assert status == 0, st
    ref = orc(name).scf(site, np.array(q, dtype=float), TIGHT_O)
    assert rel(dn0, ref["dn0"]) < 1e-10
    assert rel(dn, ref["dn"]) < 1e-10


@functools.lru_cache(maxsize=None)
def _orc_response(name):
    return orc(name).response_matrix(TIGHT_O)


@pytest.mark.parametrize("precision,lowp,bar", [(0, 0, 1e-10), (1, 0, 1e-6), (1, 1, 1e-6)])
def test_spin_response_matrix_and_uv(precision, lowp, bar):
    hp = _hp()
    name = "duo_k221_afm"
    tol = 1e-13 if precision == 0 else 1e-10
    chi0, chi, mim, st, status = hp.hp_response_matrix(ctx(name), (1, 2, 1), tight_gpu(precision, lowp, tol))
    assert status == 0
    if precision == 1:
        assert st["h_applies_lowp"] > 0
    c0, c1, _, _, _ = _orc_response(name)
    assert rel(chi0, c0) < bar and rel(chi, c1) < bar
    uv = hp.hp_hubbard_params(chi0, chi)
    assert np.abs(uv - oracle.hubbard_params(c0, c1)).max() * HA_MEV < (1e-3 if precision == 0 else 5.0)


def test_equal_spin_blocks_reproduce_the_unpolarized_gpu_result():
    hp = _hp()
    gs = ground_state("duo_k221")
    g = copy.copy(gs)
    g.kpts = list(gs.kpts) + list(gs.kpts)
    g.vloc = np.stack([gs.vloc, gs.vloc])
    g.rho0 = np.stack([0.5 * gs.rho0, 0.5 * gs.rho0])
    g.nspin = 2
    g.spin_factor = 1
    q = (0, 0.5, 0)
    ref = hp.hp_sternheimer_scf(ctx("duo_k221"), 1, q, tight_gpu())
    pol = hp.hp_sternheimer_scf(hp.hp_ground_state_load(g), 1, q, tight_gpu())
    assert ref[3] == 0 and pol[3] == 0
    for i in (0, 1):
        assert rel(pol[i], ref[i]) < 1e-11


# ------------------------------------------------------------------ full size

@functools.lru_cache(maxsize=None)
def gs_full():
    # the antiferromagnetic olivine-shaped cell at Gamma (+ the k+q entry (0, 1/2, 0)), per spin:
    # full-size grid, spheres and bands
    from synth import cache
    return cache.get("olivine28_afm_gamma")


@functools.lru_cache(maxsize=None)
def ctx_full():
    return _hp().hp_ground_state_load(gs_full())


@functools.lru_cache(maxsize=None)
def orc_full():
    return oracle.Oracle(gs_full(), cache_limit_bytes=1.0e9)


def test_spin_fullsize_shapes():
    g = gs_full()
    assert g.nspin == 2 and len(g.kpts) == 4 and g.n_mesh == 1 and g.n_occ == 112 and g.fft == (72, 45, 40)
    assert g.gap > 0.02


@pytest.mark.parametrize("entry", [0, 1, 2, 3])
def test_spin_fullsize_apply_h_sampled(entry):
    hp = _hp()
    e = gs_full().kpts[entry]
    rng = np.random.default_rng(entry)
    X = rng.standard_normal((2, e.npw)) + 1j * rng.standard_normal((2, e.npw))
    assert rel(hp.hp_apply_h(ctx_full(), entry, X), orc_full().h_apply(entry, X)) < 1e-13


def test_spin_fullsize_first_order_solve_spin_down():
    """The spin-down mesh point at q = (0, 1/2, 0), site 1, with a spin-resolved response
    potential: the GPU solution satisfies the oracle's Sternheimer equation."""
    hp = _hp()
    o = orc_full()
    q = (0.0, 0.5, 0.0)
    ik = o.nk_spin
    j, _ = o.kq_entry(ik, q)
    rng = np.random.default_rng(2)
    dv = 0.01 * (rng.standard_normal((2,) + o.fft) + 1j * rng.standard_normal((2,) + o.fft))
    du, st = hp.hp_solve_first_order(ctx_full(), 1, q, o.n_mesh, dv,
                                     hp.ScfParams(cg_tol=1e-12, max_cg_iter=2000), gs_full().kpts[j].npw)
    assert st == 0
    b = o.rhs(ik, q, 1, dv)
    r = o.sternheimer_op(ik, q, du) - b
    assert np.linalg.norm(r, axis=1).max() / np.linalg.norm(b, axis=1).max() < 1e-10
