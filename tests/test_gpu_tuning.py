"""The autotuner and the launch-shape variants it chooses among.

Projection tiles, expansion band tiles and plane-batch FFT variants compute the same sums
in the same order, so with the K split pinned every combination must give bit-identical
results (the default shapes are held to the oracle by the parity tests, so every variant
is too). The tuner keeps the fastest candidate, never slower than the default it timed,
and tuned runs (whose K split may differ) agree with untuned ones to rounding."""
import itertools

import numpy as np
import pytest

from conftest import ground_state

pytestmark = pytest.mark.gpu


def _scf(ctx, prec, autotune=1, site=1, q=(0.0, 0.5, 0.0)):
    from paper_2203_15684_amd import hp
    p = hp.ScfParams(conv_thr_chi=1e-12, conv_thr_v=1e-10, cg_tol=1e-11, niter_max=60, max_cg_iter=2000,
                     precision=prec, autotune=autotune)
    return hp.hp_sternheimer_scf(ctx, site, q, p)


def _pin(ctx, gs, prec_list, batch, tile, nsplit, bands, pv, sv=(0, 0)):
    from paper_2203_15684_amd import hp
    rows = gs.n_beta + gs.n_occ
    for prec in prec_list:
        for m in (rows, gs.n_occ, 5 * gs.n_hub, 5):
            hp.hp_set_gemm_shape(ctx, prec, m, batch, tile, nsplit, bands)
        hp.hp_set_plane_variant(ctx, prec, pv)
        hp.hp_set_stick_variant(ctx, prec, *sv)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_shape_variants_bitwise(prec):
    from paper_2203_15684_amd import hp
    gs = ground_state("duo_k221")
    ctx = hp.hp_ground_state_load(gs)
    pr = hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED
    precs = [64] if prec == "fp64" else [64, 32]
    ref = None
    for i, (tile, bands) in enumerate(itertools.product(range(4), (32, 64, 128))):
        # the 30x24 plane has four LDS variants; N3 = 24 all three z-transform variants
        _pin(ctx, gs, precs, gs.n_mesh, tile, 2, bands, i % 4, (i % 3, (i // 3) % 3))
        out = _scf(ctx, pr)
        assert out[3] == 0
        if ref is None:
            ref = out
            continue
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), (tile, bands)
        assert out[2]["cg_iters"] == ref[2]["cg_iters"]


def test_shape_variants_bitwise_fullsize_solve():
    """At the olivine size (72x45 planes, 224 projector rows, 112 bands) on one k-point."""
    from paper_2203_15684_amd import hp
    from synth import cache
    gs = cache.get("olivine28")
    ctx = hp.hp_ground_state_load(gs)
    q, ik = (0.0, 0.5, 0.5), 5
    k = gs.kpts[ik].k_frac + np.asarray(q)
    npw = next(e.npw for e in gs.kpts if np.allclose(k - e.k_frac, np.round(k - e.k_frac)))
    ref = None
    for tile, bands, pv, sv in [(0, 32, 0, (0, 0)), (3, 128, 1, (1, 1)), (1, 64, 2, (1, 0)), (2, 128, 3, (0, 1)),
                                (3, 32, 2, (2, 2)), (0, 64, 0, (2, 1))]:
        for prec in ("fp64", "mixed"):
            _pin(ctx, gs, [64, 32], 1, tile, 4, bands, pv, sv)
            p = hp.ScfParams(cg_tol=1e-11, max_cg_iter=2000, precision=hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED)
            du, st = hp.hp_solve_first_order(ctx, 3, q, ik, None, p, npw)
            assert st == 0
            if ref is None or prec not in ref:
                ref = (ref or {}) | {prec: du}
            else:
                assert np.array_equal(du, ref[prec]), (tile, bands, pv, prec)


def test_tuner_report_and_agreement():
    from paper_2203_15684_amd import hp
    gs = ground_state("duo_k221")
    tuned = hp.hp_ground_state_load(gs)
    plain = hp.hp_ground_state_load(gs)
    a = _scf(tuned, hp.HP_MIXED, autotune=1)
    b = _scf(plain, hp.HP_MIXED, autotune=0)
    assert a[3] == b[3] == 0
    assert np.abs(a[1] - b[1]).max() < 1e-12 * np.abs(b[1]).max()
    rep = hp.hp_tuning_report(tuned)
    rows = gs.n_beta + gs.n_occ
    shapes = {(g["prec"], g["rows"], g["batch"]) for g in rep["gemm"]}
    assert {(64, rows, gs.n_mesh), (64, gs.n_occ, gs.n_mesh), (32, rows, gs.n_mesh)} <= shapes
    for g in rep["gemm"]:
        assert g["proj_tile"] in ("32x32", "64x32", "32x64", "64x64") and g["expand_bands"] in (32, 64, 128)
        assert g["proj_ms"] <= g["proj_default_ms"] and g["expand_ms"] <= g["expand_default_ms"]
    assert {p["prec"] for p in rep["plane"]} == {64, 32}
    for p in rep["plane"]:   # -1: variant not available for this grid
        assert p["ms"][p["variant"]] == min(m for m in p["ms"] if m >= 0)
    assert {p["prec"] for p in rep["sticks"]} == {64, 32}
    for p in rep["sticks"]:   # -1: variant not available
        assert p["inverse_ms"][p["inverse_variant"]] == min(m for m in p["inverse_ms"] if m >= 0)
        assert p["forward_ms"][p["forward_variant"]] == min(m for m in p["forward_ms"] if m >= 0)
    assert hp.hp_tuning_report(plain) == {"gemm": [], "plane": [], "sticks": []}


def test_pinning_rejects_bad_shapes():
    from paper_2203_15684_amd import hp
    gs = ground_state("sc1_gamma")
    ctx = hp.hp_ground_state_load(gs)
    for args in [(8, 8, 1, 0, 1, 32), (64, 8, 1, 4, 1, 32), (64, 8, 1, 0, 0, 32), (64, 8, 1, 0, 1, 48),
                 (64, 8, 2, 0, 1, 32)]:
        with pytest.raises(hp.HpError):
            hp.hp_set_gemm_shape(ctx, *args)
    with pytest.raises(hp.HpError):
        hp.hp_set_plane_variant(ctx, 64, 1)   # 24x24 planes: only variant 0
    with pytest.raises(hp.HpError):
        hp.hp_set_stick_variant(ctx, 64, 3, 0)


@pytest.mark.parametrize("name", ["sc1_gamma", "duo_k221", "olivine28_gamma", "olivine56_gamma"])
def test_register_plane_variants(name):
    """The FP32 register-resident plane round trips (variants 4-6: a y column, then an x row
    or half of one, in a thread's registers; 144-point rows split over two lanes with a DPP
    exchange in the last radix-2 stage; planes kept in LDS compacted to the window of x
    columns that can hold sphere points, zero inputs outside the x and y windows not
    loaded), on the 24x24, 30x24, 72x45 and 144x45 planes: the
    reduced-precision H apply (FP32 transforms and projections) against the FP64 oracle to
    FP32 accuracy, against the LDS variant 0 to within the rounding of the FMA choices (the
    butterflies are the same, the compiler may contract them differently), and the
    mixed-precision solves they drive agree to the solve tolerance."""
    import oracle
    from paper_2203_15684_amd import hp
    if name.startswith("olivine"):
        from synth import cache
        gs = cache.get(name)
    else:
        gs = ground_state(name)
    ctx = hp.hp_ground_state_load(gs)
    o = oracle.Oracle(gs)
    rng = np.random.default_rng(4)
    entry = len(gs.kpts) - 1
    X = rng.standard_normal((6, gs.kpts[entry].npw)) + 1j * rng.standard_normal((6, gs.kpts[entry].npw))
    X = np.vstack([X, gs.kpts[entry].u[:3]])
    ref64 = o.h_apply(entry, X)
    o_q = (0.0, 0.5, 0.0) if name != "sc1_gamma" else (0.0, 0.0, 0.0)
    ik = 0
    k = gs.kpts[ik].k_frac + np.asarray(o_q)
    npw = next(e.npw for e in gs.kpts if np.allclose(k - e.k_frac, np.round(k - e.k_frac)))
    y0 = du0 = None
    for pv in (0, 4, 5, 6):
        _pin(ctx, gs, [64, 32], 1, 0, 2, 32, 0)
        hp.hp_set_plane_variant(ctx, 32, pv)
        y = hp.hp_apply_h_lowp(ctx, entry, X)
        err = np.abs(y - ref64).max() / np.abs(ref64).max()
        print(f"[fp32 apply] {name} variant {pv}: {err:.2e} from FP64", flush=True)
        assert err < 2e-6, (pv, err)
        p = hp.ScfParams(cg_tol=1e-11, max_cg_iter=2000, precision=hp.HP_MIXED)
        du, st = hp.hp_solve_first_order(ctx, 0, o_q, ik, None, p, npw)
        assert st == 0
        if y0 is None:
            y0, du0 = y, du
        else:
            assert np.abs(y - y0).max() < 5e-7 * np.abs(y0).max(), pv
            assert np.abs(du - du0).max() < 1e-9 * np.abs(du0).max(), pv
    ctx.close()


def test_register_window_guard():
    """A sphere wider than the register variants' window (|m| up to 8 on 24-point x and y
    axes, whose window [0, 8) u [16, 24) holds m = -8..7): variants 4-6 are refused for it,
    and the FP32 apply of the variants that remain still meets the FP64 oracle."""
    import dataclasses
    import oracle
    import synth
    from paper_2203_15684_amd import hp
    spec = dataclasses.replace(synth.SPECS["sc1_gamma"], name="sc1_gamma_wide", ecut=20.0)
    gs = synth.build_ground_state(spec, device="cuda")
    assert max(int(np.abs(e.miller[:, 0]).max()) for e in gs.kpts) >= 8
    ctx = hp.hp_ground_state_load(gs)
    for v in (4, 5, 6):
        with pytest.raises(hp.HpError, match="not available"):
            hp.hp_set_plane_variant(ctx, 32, v)
    o = oracle.Oracle(gs)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((4, gs.kpts[0].npw)) + 1j * rng.standard_normal((4, gs.kpts[0].npw))
    ref = o.h_apply(0, X)
    hp.hp_set_plane_variant(ctx, 32, 0)
    y = hp.hp_apply_h_lowp(ctx, 0, X)
    assert np.abs(y - ref).max() / np.abs(ref).max() < 2e-6
