"""CG iterations replayed from captured hipGraphs against the same iterations launched one
by one. Converged items are skipped by every kernel and the reductions run in a fixed
order, so the two must agree bit for bit, with the same iteration and H-apply counts. Each
SCF replays its graphs many times with eager work (RHS, response density, mixing) and host
synchronisations in between, and a second SCF replays the graphs cached by the first."""
import numpy as np
import pytest

from conftest import ground_state

pytestmark = pytest.mark.gpu


def _ctx(name):
    from paper_2203_15684_amd import hp
    return hp.hp_ground_state_load(ground_state(name))


def _run(ctx, prec, chunk, site=0, q=(0.0, 0.5, 0.0), **kw):
    from paper_2203_15684_amd import hp
    p = hp.ScfParams(conv_thr_chi=1e-12, conv_thr_v=1e-10, cg_tol=1e-11, niter_max=60, max_cg_iter=2000,
                     precision=prec, graph_chunk=chunk, **kw)
    return hp.hp_sternheimer_scf(ctx, site, q, p)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,q", [("duo_k221", (0.0, 0.5, 0.0)), ("sc1_k221", (0.5, 0.5, 0.0))])
def test_graph_matches_eager_bitwise(name, q, prec):
    from paper_2203_15684_amd import hp
    pr = hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED
    ctx = _ctx(name)
    eager = _run(ctx, pr, 0, q=q)
    for chunk in (8, 3, 8):   # the third run replays the graphs cached by the first
        g = _run(ctx, pr, chunk, q=q)
        assert g[3] == eager[3] == 0
        assert np.array_equal(g[0], eager[0]) and np.array_equal(g[1], eager[1])
        for key in ("scf_iters", "cg_iters", "h_applies_fp64", "h_applies_lowp"):
            assert g[2][key] == eager[2][key], key


def test_graph_profiling_counts_match_eager():
    """Kernel times inside graphs (device-clock stamps around each timed kernel) against HIP
    events around the same kernels launched one by one: the same launches are counted
    (iterations past convergence are not) and the per-kernel totals agree."""
    from paper_2203_15684_amd import hp
    ctx = _ctx("duo_k221")
    prof = {}
    for chunk in (0, 8):
        hp.hp_profile_start(ctx)
        _run(ctx, hp.HP_MIXED, chunk)
        prof[chunk] = hp.hp_profile_stop(ctx)
    for name, (calls, ms) in prof[0].items():
        assert prof[8][name][0] == calls, name
        if ms > 2.0:
            assert 0.8 < prof[8][name][1] / ms < 1.25, (name, ms, prof[8][name][1])


def test_graph_first_order_solve_matches_eager():
    from paper_2203_15684_amd import hp
    ctx = _ctx("duo_k221")
    gs = ground_state("duo_k221")
    out = []
    for chunk in (0, 8, 8):
        p = hp.ScfParams(cg_tol=1e-12, max_cg_iter=2000, graph_chunk=chunk)
        du, st = hp.hp_solve_first_order(ctx, 1, (0.0, 0.5, 0.0), 2, None, p, _npw_kq(gs, (0.0, 0.5, 0.0), 2))
        assert st == 0
        out.append(du)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def _npw_kq(gs, q, ik):
    k = gs.kpts[ik].k_frac + np.asarray(q)
    for e in gs.kpts:
        d = k - e.k_frac
        if np.allclose(d, np.round(d)):
            return e.npw
    raise AssertionError("no k+q entry")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_matches_eager_fullsize_one_pair(prec):
    from paper_2203_15684_amd import hp
    from synth import cache
    pr = hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED
    ctx = hp.hp_ground_state_load(cache.get("olivine28"))
    base = dict(conv_thr_chi=1e-10, conv_thr_v=1e-8, cg_tol=1e-10, niter_max=100, max_cg_iter=2000, precision=pr)
    e = hp.hp_sternheimer_scf(ctx, 2, (0.0, 0.0, 0.5), hp.ScfParams(**base, graph_chunk=0))
    g = hp.hp_sternheimer_scf(ctx, 2, (0.0, 0.0, 0.5), hp.ScfParams(**base, graph_chunk=8))
    assert e[3] == g[3] == 0
    assert np.array_equal(e[0], g[0]) and np.array_equal(e[1], g[1])
    assert e[2]["cg_iters"] == g[2]["cg_iters"]
