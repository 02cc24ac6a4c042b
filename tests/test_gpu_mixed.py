"""Mixed-precision path (FP32 FFTs and FP32 or BF16 MFMA projections inside the PCG,
FP64 residual refinement of every Sternheimer solve, FP64 orthogonalization, scalars,
chi assembly and inversion) against the FP64 oracle and the FP64 GPU path. Every test
runs with each projection number type: FP32, BF16 for the KB and P_v GEMMs, and BF16
for the KB GEMMs with P_v in FP32.

Bar (stated for this form): chi within 1e-6 relative and U/V within 5 meV of the
FP64 reference; with a tight solve tolerance the refinement reaches FP64 accuracy.
"""
import functools

import numpy as np
import pytest

import oracle
from conftest import ground_state

pytestmark = pytest.mark.gpu
HA_MEV = 27211.386245988


def _hp():
    from paper_2203_15684_amd import hp
    return hp


@functools.lru_cache(maxsize=None)
def ctx(name):
    return _hp().hp_ground_state_load(ground_state(name))


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(ground_state(name))


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


LOWP = [0, 1, 2]   # HP_GEMM_FP32, HP_GEMM_BF16, HP_GEMM_BF16_PV32


def mixed(cg_tol, thr=1e-12, lowp=0):
    hp = _hp()
    return hp.ScfParams(conv_thr_chi=thr, conv_thr_v=1e-10, cg_tol=cg_tol, niter_max=100, max_cg_iter=2000,
                        precision=hp.HP_MIXED, lowp_gemm=lowp)


@pytest.mark.parametrize("lowp", LOWP)
@pytest.mark.parametrize("name,q", [("sc1_gamma", (0, 0, 0)), ("duo_k221", (0, 0.5, 0))])
def test_mixed_first_order_solve_refines_to_fp64(name, q, lowp):
    hp = _hp()
    o = orc(name)
    rng = np.random.default_rng(3)
    dv = 0.05 * (rng.standard_normal(o.fft) + 1j * rng.standard_normal(o.fft))
    for ik in range(o.n_mesh):
        j, _ = o.kq_entry(ik, q)
        x_ref, _ = o.solve(ik, q, o.rhs(ik, q, 0, dv), None, oracle.ScfParams(cg_tol=1e-14))
        du, st = hp.hp_solve_first_order(ctx(name), 0, q, ik, dv, mixed(1e-12, lowp=lowp), o.kpts[j].npw)
        assert st == 0
        assert rel(du, x_ref) < 1e-10, f"k {ik}"


@pytest.mark.parametrize("lowp", LOWP)
@pytest.mark.parametrize("name,site,q", [("sc1_gamma", 0, (0, 0, 0)), ("duo_k221", 1, (0, 0.5, 0))])
def test_mixed_scf_matches_oracle(name, site, q, lowp):
    hp = _hp()
    ref = orc(name).scf(site, np.array(q), oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11))
    dn0, dn, st, status = hp.hp_sternheimer_scf(ctx(name), site, q, mixed(1e-10, 1e-10, lowp))
    assert status == 0
    assert st["h_applies_lowp"] > 0
    assert rel(dn0, ref["dn0"]) < 1e-6
    assert rel(dn, ref["dn"]) < 1e-6


@functools.lru_cache(maxsize=None)
def _orc_response(name):
    return orc(name).response_matrix(oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11))


@pytest.mark.parametrize("lowp", LOWP)
def test_mixed_response_matrix_and_uv(lowp):
    hp = _hp()
    name = "duo_k221"
    c0, c1, _, _, _ = _orc_response(name)
    c = hp.hp_ground_state_load(ground_state(name))
    hp.hp_profile_start(c)
    chi0, chi, mim, st, status = hp.hp_response_matrix(c, (1, 2, 1), mixed(1e-10, 1e-10, lowp))
    prof = hp.hp_profile_stop(c)
    assert status == 0
    # the whole-response entry point runs the requested projection type and tunes its shapes
    calls = {k: v[0] for k, v in prof.items()}
    assert (calls.get("zproj16", 0) > 0) == (lowp in (1, 2))
    assert (calls.get("zproj32", 0) > 0) == (lowp in (0, 2))
    rep = hp.hp_tuning_report(c)
    assert {g["prec"] for g in rep["gemm"]} == ({64, 32} if lowp == 0 else {64, 16} if lowp == 1 else {64, 32, 16})
    assert rel(chi0, c0) < 1e-6 and rel(chi, c1) < 1e-6
    uv = hp.hp_hubbard_params(chi0, chi)
    assert np.abs(uv - oracle.hubbard_params(c0, c1)).max() * HA_MEV < 5.0


@pytest.mark.parametrize("lowp,bar", [(0, 2e-6), (1, 2e-2), (2, 2e-2)])
def test_lowp_operator_accuracy(lowp, bar):
    """The inner solves' operator itself (hp_apply_h_lowp: FP32 transforms and V psi; FP32,
    BF16, or BF16 KB with FP32 P_v projections) against the FP64 oracle on every entry:
    FP32 to ~1e-6, BF16 to its 8-bit mantissa (~4e-3)."""
    hp = _hp()
    name = "duo_k221"
    o = oracle.Oracle(ground_state(name))
    rng = np.random.default_rng(9)
    worst = 0.0
    for ie, e in enumerate(o.kpts):
        X = rng.standard_normal((4, e.npw)) + 1j * rng.standard_normal((4, e.npw))
        Y = hp.hp_apply_h_lowp(ctx(name), ie, X, lowp)
        ref = o.h_apply(ie, X)
        worst = max(worst, np.abs(Y - ref).max() / np.abs(ref).max())
    assert worst < bar, worst


def test_trust_tolerance_ablation():
    """lowp_trust_tol: solves at or above it are finished in FP32 (no FP64 operator apply);
    1 refines every solve in FP64.  Both meet the oracle at the mixed bar; refining every
    solve performs more FP64 applies, and a negative value is rejected."""
    hp = _hp()
    name, site, q = "duo_k221", 1, (0, 0.5, 0)
    ref = orc(name).scf(site, np.array(q), oracle.ScfParams(cg_tol=1e-13, conv_thr_chi=1e-13, conv_thr_v=1e-11))
    applies = {}
    for trust in (1e-6, 1.0):
        p = mixed(1e-10, 1e-10)
        p.lowp_trust_tol = trust
        dn0, dn, st, status = hp.hp_sternheimer_scf(ctx(name), site, q, p)
        assert status == 0
        assert rel(dn0, ref["dn0"]) < 1e-6 and rel(dn, ref["dn"]) < 1e-6
        applies[trust] = st["h_applies_fp64"]
    assert applies[1.0] > applies[1e-6]
    p = mixed(1e-10, 1e-10)
    p.lowp_trust_tol = -1.0
    with pytest.raises(Exception, match="lowp_trust_tol"):
        hp.hp_sternheimer_scf(ctx(name), site, q, p)
