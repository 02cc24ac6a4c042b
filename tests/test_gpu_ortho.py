"""Ortho-atomic Hubbard projectors (Eq. 6) on the GPU against the oracle's Loewdin
orthogonalization of the same atomic orbital set.

The library builds the projectors itself at load time (overlaps and expansion on the
matrix cores, O^-1/2 by Jacobi on the host); every response quantity downstream is then
compared with Oracle(projectors="ortho-atomic"): occupation responses and chi at the
small sizes (FP64 bar 1e-10 relative, mixed bar 1e-6), and at the full olivine-shaped
size one k-point's Sternheimer solve against the oracle's ortho-atomic right-hand side.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
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
    hp = _hp()
    return hp.ScfParams(conv_thr_chi=1e-13, conv_thr_v=1e-11, cg_tol=cg_tol, niter_max=100, max_cg_iter=3000,
                        precision=precision, lowp_gemm=lowp)


@functools.lru_cache(maxsize=None)
def ctx(name):
    gs = ground_state(name)
    atw, hub_rows = synth.atomic_orbital_tables(gs)
    return _hp().hp_ground_state_load(gs, atwfc=atw, hub_rows=hub_rows)


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name), projectors="ortho-atomic")


@pytest.mark.parametrize("name,site,q", [("sc1_gamma", 0, (0, 0, 0)), ("duo_k221", 1, (0, 0.5, 0))])
def test_ortho_scf_matches_oracle(name, site, q):
    hp = _hp()
    dn0, dn, st, status = hp.hp_sternheimer_scf(ctx(name), site, q, tight_gpu())
    assert status == 0, st
    ref = orc(name).scf(site, np.array(q), TIGHT_O)
    assert rel(dn0, ref["dn0"]) < 1e-10
    assert rel(dn, ref["dn"]) < 1e-10
    # the projectors really changed: the atomic-projector response differs
    plain = oracle.Oracle(ground_state(name)).scf(site, np.array(q), TIGHT_O)
    assert rel(plain["dn0"], ref["dn0"]) > 1e-3


@pytest.mark.parametrize("precision,lowp,bar", [(0, 0, 1e-10), (1, 1, 1e-6)])
def test_ortho_response_matrix_and_uv(precision, lowp, bar):
    hp = _hp()
    name = "duo_k221"
    tol = 1e-13 if precision == 0 else 1e-10
    chi0, chi, mim, st, status = hp.hp_response_matrix(ctx(name), (1, 2, 1), tight_gpu(precision, lowp, tol))
    assert status == 0
    c0, c1, _, _, _ = _orc_response(name)
    assert rel(chi0, c0) < bar and rel(chi, c1) < bar
    uv = hp.hp_hubbard_params(chi0, chi)
    assert np.abs(uv - oracle.hubbard_params(c0, c1)).max() * HA_MEV < (1e-3 if precision == 0 else 5.0)


@functools.lru_cache(maxsize=None)
def _orc_response(name):
    return orc(name).response_matrix(TIGHT_O)


def test_ortho_linearly_dependent_orbitals_are_singular():
    """An orbital set with a repeated row has a singular overlap: the load refuses it."""
    hp = _hp()
    gs = ground_state("sc1_gamma")
    atw, hub_rows = synth.atomic_orbital_tables(gs)
    dup = [np.vstack([a, a[:1]]) for a in atw]
    with pytest.raises(hp.HpError) as e:
        hp.hp_ground_state_load(gs, atwfc=dup, hub_rows=hub_rows)
    assert e.value.status == hp.HP_ERR_SINGULAR


def test_ortho_fullsize_first_order_solve_one_k():
    """Full olivine-shaped size (132 atomic orbitals per entry, 48 entries): one k-point's
    Hubbard-only first-order solve (mesh index 7, q = (0, 1/2, 0), site 2) satisfies the
    oracle's Sternheimer equation with the oracle's ortho-atomic right-hand side."""
    from synth import cache
    hp = _hp()
    g = cache.get("olivine28")
    atw, hub_rows = synth.atomic_orbital_tables(g)
    assert atw[0].shape[0] == 4 * 28 + 5 * g.n_hub
    c = hp.hp_ground_state_load(g, atwfc=atw, hub_rows=hub_rows)
    del atw
    o = oracle.Oracle(g, cache_limit_bytes=1.0e9, projectors="ortho-atomic")
    q = (0.0, 0.5, 0.0)
    ik = 7
    j, _ = o.kq_entry(ik, q)
    du, st = hp.hp_solve_first_order(c, 2, q, ik, None, hp.ScfParams(cg_tol=1e-12, max_cg_iter=2000),
                                     g.kpts[j].npw)
    assert st == 0
    b = o.rhs(ik, q, 2, None)
    r = o.sternheimer_op(ik, q, du) - b
    assert np.linalg.norm(r, axis=1).max() / np.linalg.norm(b, axis=1).max() < 1e-10
