"""Metallic ground states (cold smearing; the paper's generalization of Eq. 15 to fractional
occupations) on the GPU against the oracle: first-order solves at q != 0 with the
beta-weighted projection, the self-consistent response at q = 0 (where the Fermi level
shifts; one k point and k meshes) and at q != 0, the response matrix and U, the ground-state
site occupations; FP64 bar 1e-10, mixed 1e-6.
"""
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
    # the mixed form stops at the change of chi its FP32 inner solves resolve (as for insulators)
    thr = (1e-13, 1e-11) if precision == 0 else (1e-10, 1e-9)
    return _hp().ScfParams(conv_thr_chi=thr[0], conv_thr_v=thr[1], cg_tol=cg_tol, niter_max=100, max_cg_iter=3000,
                           precision=precision, lowp_gemm=lowp)


@functools.lru_cache(maxsize=None)
def ctx(name):
    return _hp().hp_ground_state_load(ground_state(name))


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


def test_metal_first_order_solve():
    hp = _hp()
    name = "sc1_k211_metal"
    o = orc(name)
    q = (0.5, 0, 0)
    rng = np.random.default_rng(8)
    dv = 0.05 * (rng.standard_normal(o.fft) + 1j * rng.standard_normal(o.fft))
    for ik in o.mesh:
        j, _ = o.kq_entry(ik, q)
        x_ref, _ = o.solve(ik, q, o.rhs(ik, q, 0, dv), None, oracle.ScfParams(cg_tol=1e-14))
        du, st = hp.hp_solve_first_order(ctx(name), 0, q, ik, dv, hp.ScfParams(cg_tol=1e-13, max_cg_iter=3000),
                                         o.kpts[j].npw)
        assert st == 0
        assert rel(du, x_ref) < 1e-10, ik


@pytest.mark.parametrize("name,q", [("sc1_gamma_metal", (0, 0, 0)), ("sc1_k211_metal", (0, 0, 0)),
                                    ("sc1_k211_metal", (0.5, 0, 0))])
def test_metal_scf_matches_oracle(name, q):
    hp = _hp()
    ref = orc(name).scf(0, np.array(q, dtype=float), TIGHT_O)
    d64 = hp.hp_sternheimer_scf(ctx(name), 0, q, tight_gpu())
    assert d64[3] == 0, d64[2]
    assert rel(d64[0], ref["dn0"]) < 1e-10 and rel(d64[1], ref["dn"]) < 1e-10
    d32 = hp.hp_sternheimer_scf(ctx(name), 0, q, tight_gpu(1, 0, 1e-10))
    assert d32[3] == 0, d32[2]
    assert rel(d32[0], ref["dn0"]) < 1e-6 and rel(d32[1], ref["dn"]) < 1e-6


def test_metal_response_matrix_and_u():
    hp = _hp()
    name = "sc1_k211_metal"
    chi0, chi, mim, st, status = hp.hp_response_matrix(ctx(name), (2, 1, 1), tight_gpu())
    assert status == 0
    c0, c1, _, _, _ = orc(name).response_matrix(TIGHT_O)
    assert rel(chi0, c0) < 1e-10 and rel(chi, c1) < 1e-10
    uv = hp.hp_hubbard_params(chi0, chi)
    assert np.abs(uv - oracle.hubbard_params(c0, c1)).max() * HA_MEV < 1e-3


def test_metal_site_occupations():
    """Ground-state occupation traces of a metal carry the band occupations (Eq. 3)."""
    hp = _hp()
    name = "sc1_k211_metal"
    tr, mo, cl = hp.hp_site_occupations(ctx(name))
    t_ref, _ = orc(name).site_traces()
    assert np.abs(tr - t_ref).max() < 1e-12 * np.abs(t_ref).max()
    assert np.all(mo == 0) and list(cl) == [0]


def test_metal_q0_on_a_k_mesh_matches_oracle():
    hp = _hp()
    name = "duo_k221_metal"
    ref = orc(name).scf(1, np.zeros(3), TIGHT_O)
    d = hp.hp_sternheimer_scf(ctx(name), 1, (0, 0, 0), tight_gpu())
    assert d[3] == 0, d[2]
    assert rel(d[0], ref["dn0"]) < 1e-10 and rel(d[1], ref["dn"]) < 1e-10


@functools.lru_cache(maxsize=None)
def _full():
    from synth import cache
    g = cache.get("olivine28_metal")
    return g, _hp().hp_ground_state_load(g)


def test_metal_fullsize_first_order_one_k():
    """Full olivine size, metallic (cold smearing, partially filled kept bands, 72x45x40):
    one mesh k of the first SCF iteration at q = (0, 1/2, 0), all kept bands.  The GPU
    solution satisfies the oracle's Sternheimer equation (the beta-weighted projection of the
    metallic right-hand side) and equals the oracle's own CG solution."""
    hp = _hp()
    g, c = _full()
    o = oracle.Oracle(g, cache_limit_bytes=1.0e9)
    q = (0.0, 0.5, 0.0)
    ik = 5
    j, _ = o.kq_entry(ik, q)
    du, st = hp.hp_solve_first_order(c, 1, q, ik, None, hp.ScfParams(cg_tol=1e-12, max_cg_iter=3000), g.kpts[j].npw)
    assert st == 0
    b = o.rhs(ik, q, 1, None)
    r = o.sternheimer_op(ik, q, du) - b
    assert np.linalg.norm(r, axis=1).max() / np.linalg.norm(b, axis=1).max() < 1e-10
    x_ref, _ = o.solve(ik, q, b, None, oracle.ScfParams(cg_tol=1e-12))
    assert rel(du, x_ref) < 1e-9


def test_metal_fullsize_q0_pair_mixed_vs_fp64():
    """Full olivine size, metallic, q = 0 (the Fermi-level shift enters): one (site, q) SCF in
    both precisions converges, and the mixed form's response occupations match FP64's to
    the mixed bar."""
    hp = _hp()
    g, c = _full()
    base = dict(conv_thr_chi=1e-10, conv_thr_v=1e-8, cg_tol=1e-10, niter_max=100, max_cg_iter=3000)
    d64 = hp.hp_sternheimer_scf(c, 0, (0.0, 0.0, 0.0), hp.ScfParams(**base, precision=hp.HP_FP64))
    d32 = hp.hp_sternheimer_scf(c, 0, (0.0, 0.0, 0.0), hp.ScfParams(**base, precision=hp.HP_MIXED))
    assert d64[3] == 0 and d32[3] == 0, (d64[2], d32[2])
    assert rel(d32[0], d64[0]) < 1e-6 and rel(d32[1], d64[1]) < 1e-6
