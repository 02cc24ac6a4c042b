"""Ground-state Hubbard potential in the unperturbed Hamiltonian (Eq. 5, on-site part) and the
equivalent-site reduction of the response matrices on the GPU, against the oracle.

The library carries the potential as extra rows of its stacked projector table (scale +1
and -1 blocks from the eigenpairs of each site's 5 x 5 matrix), so every H apply of the
Sternheimer solves includes it.  Checks: H applies on every entry (also with ortho-atomic
projectors), Delta n and chi against the oracle (FP64 1e-10, mixed 1e-6) on a one-site
system and on the antiferromagnetic two-site system (spin-dependent potential), at full
size sampled H applies and a solve against the oracle's equation; occupation traces,
moments and classes against the oracle, chi rebuilt from one perturbed site of a
translation-equivalent pair equal to chi from perturbing both, and chi with the -q partners
of a q mesh taken from time reversal equal to solving every q.
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


def tight_gpu(precision=0, lowp=0, cg_tol=1e-13, **kw):
    return _hp().ScfParams(conv_thr_chi=1e-13, conv_thr_v=1e-11, cg_tol=cg_tol, niter_max=100, max_cg_iter=3000,
                           precision=precision, lowp_gemm=lowp, **kw)


@functools.lru_cache(maxsize=None)
def ctx(name):
    return _hp().hp_ground_state_load(ground_state(name))


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


@pytest.mark.parametrize("name", ["sc1_gamma_u", "duo_k221_afm_u"])
def test_hub_apply_h_every_entry(name):
    hp = _hp()
    o = orc(name)
    rng = np.random.default_rng(6)
    for ie, e in enumerate(o.kpts):
        X = rng.standard_normal((3, e.npw)) + 1j * rng.standard_normal((3, e.npw))
        X = np.vstack([X, e.u[:2]])
        assert rel(hp.hp_apply_h(ctx(name), ie, X), o.h_apply(ie, X)) < 1e-13, f"entry {ie}"


def test_hub_apply_h_with_ortho_atomic_projectors():
    hp = _hp()
    gs = ground_state("duo_k221_afm_u")
    atw, hub_rows = synth.atomic_orbital_tables(gs)
    c = hp.hp_ground_state_load(gs, atwfc=atw, hub_rows=hub_rows)
    o = oracle.Oracle(gs, projectors="ortho-atomic")
    rng = np.random.default_rng(7)
    for ie in (0, 5, o.nk_spin + 3):
        e = o.kpts[ie]
        X = rng.standard_normal((3, e.npw)) + 1j * rng.standard_normal((3, e.npw))
        assert rel(hp.hp_apply_h(c, ie, X), o.h_apply(ie, X)) < 1e-13


@pytest.mark.parametrize("name,site,q", [("sc1_gamma_u", 0, (0, 0, 0)), ("duo_k221_afm_u", 1, (0, 0.5, 0))])
def test_hub_scf_matches_oracle(name, site, q):
    hp = _hp()
    ref = orc(name).scf(site, np.array(q, dtype=float), TIGHT_O)
    d64 = hp.hp_sternheimer_scf(ctx(name), site, q, tight_gpu())
    assert d64[3] == 0
    assert rel(d64[0], ref["dn0"]) < 1e-10 and rel(d64[1], ref["dn"]) < 1e-10
    d32 = hp.hp_sternheimer_scf(ctx(name), site, q, tight_gpu(1, 1, 1e-10))
    assert d32[3] == 0
    assert rel(d32[0], ref["dn0"]) < 1e-6 and rel(d32[1], ref["dn"]) < 1e-6


def test_hub_response_matrix_and_uv():
    hp = _hp()
    name = "duo_k221_afm_u"
    chi0, chi, mim, st, status = hp.hp_response_matrix(ctx(name), (1, 2, 1), tight_gpu())
    assert status == 0
    c0, c1, _, _, _ = orc(name).response_matrix(TIGHT_O)
    assert rel(chi0, c0) < 1e-10 and rel(chi, c1) < 1e-10
    uv = hp.hp_hubbard_params(chi0, chi)
    assert np.abs(uv - oracle.hubbard_params(c0, c1)).max() * HA_MEV < 1e-3


@pytest.mark.parametrize("name", ["sc1_super211", "duo_k221_afm"])
def test_site_occupations_and_classes(name):
    hp = _hp()
    tr, mo, cl = hp.hp_site_occupations(ctx(name))
    t_ref, m_ref = orc(name).site_traces()
    assert np.abs(tr - t_ref).max() < 1e-12 * np.abs(t_ref).max()
    assert np.abs(mo - m_ref).max() < 1e-12 * max(1.0, np.abs(m_ref).max())
    assert list(cl) == list(oracle.equivalent_sites(t_ref))


def test_reduced_response_matrix_equals_full():
    """Two sites related by a translation of the replica: perturbing one and rebuilding the
    other column gives the matrix of perturbing both, and the oracle's."""
    hp = _hp()
    name = "sc1_super211"
    full = hp.hp_response_matrix(ctx(name), (1, 1, 1), tight_gpu())
    red = hp.hp_response_matrix(ctx(name), (1, 1, 1), tight_gpu(find_atpert=1))
    assert full[4] == 0 and red[4] == 0
    assert red[3]["scf_iters"] < full[3]["scf_iters"]      # one (site, q) problem instead of two
    for i in (0, 1):
        assert rel(red[i], full[i]) < 1e-9
    o = orc(name)
    p = oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11)
    cols0, cols = [], []
    for sp in range(2):
        r = o.scf(sp, np.zeros(3), p)
        cols0.append(np.einsum("smm->s", r["dn0"]).real)
        cols.append(np.einsum("smm->s", r["dn"]).real)
    assert rel(red[0], np.array(cols0).T) < 1e-9 and rel(red[1], np.array(cols).T) < 1e-9


def test_reduced_response_matrix_inequivalent_sites_is_the_full_one():
    hp = _hp()
    name = "duo_k221"
    full = hp.hp_response_matrix(ctx(name), (1, 2, 1), tight_gpu())
    red = hp.hp_response_matrix(ctx(name), (1, 2, 1), tight_gpu(find_atpert=1))
    for i in (0, 1):
        assert np.array_equal(red[i], full[i])


# ------------------------------------------------------------------ full size

@functools.lru_cache(maxsize=None)
def gs_full():
    from synth import cache
    return cache.get("olivine28_u_gamma")  # DFT+U olivine-shaped cell at Gamma (+ (0, 1/2, 0))


@functools.lru_cache(maxsize=None)
def ctx_full():
    return _hp().hp_ground_state_load(gs_full())


@functools.lru_cache(maxsize=None)
def orc_full():
    return oracle.Oracle(gs_full(), cache_limit_bytes=1.0e9)


@pytest.mark.parametrize("entry", [0, 1])
def test_hub_fullsize_apply_h_sampled(entry):
    hp = _hp()
    e = gs_full().kpts[entry]
    rng = np.random.default_rng(entry)
    X = np.vstack([rng.standard_normal((2, e.npw)) + 1j * rng.standard_normal((2, e.npw)), e.u[[0, 111]]])
    assert rel(hp.hp_apply_h(ctx_full(), entry, X), orc_full().h_apply(entry, X)) < 1e-13


def test_hub_fullsize_first_order_solve():
    hp = _hp()
    o = orc_full()
    q = (0.0, 0.5, 0.0)
    ik = 0
    j, _ = o.kq_entry(ik, q)
    du, st = hp.hp_solve_first_order(ctx_full(), 3, q, ik, None, hp.ScfParams(cg_tol=1e-12, max_cg_iter=2000),
                                     gs_full().kpts[j].npw)
    assert st == 0
    b = o.rhs(ik, q, 3, None)
    r = o.sternheimer_op(ik, q, du) - b
    assert np.linalg.norm(r, axis=1).max() / np.linalg.norm(b, axis=1).max() < 1e-10


def test_q_points_equivalent_by_time_reversal():
    """q mesh 3x1x1: q = 2/3 is -1/3 modulo G, so only two of the three q points are solved and
    chi(-q) = conj chi(q); the result equals solving every q and the oracle's."""
    hp = _hp()
    name = "sc1_k311"
    red = hp.hp_response_matrix(ctx(name), (3, 1, 1), tight_gpu())
    full = hp.hp_response_matrix(ctx(name), (3, 1, 1), tight_gpu(skip_equivalence_q=1))
    assert red[4] == 0 and full[4] == 0
    assert red[3]["scf_iters"] < full[3]["scf_iters"]
    for i in (0, 1):
        assert rel(red[i], full[i]) < 1e-10
    c0, c1, _, _, _ = orc(name).response_matrix(TIGHT_O)
    assert rel(red[0], c0) < 1e-10 and rel(red[1], c1) < 1e-10
