"""Full-size parity against stored oracle references.

tests/golden/*.json hold Delta_q n0 (the chi0 column) and Delta_q n (the chi column) of one
(site, q) self-consistent response, computed by the FP64 oracle alone
(tests/golden/make_golden.py) at the full-size grids, spheres and band counts:
olivine28_gamma (FFT 72x45x40, ~10^4 plane waves, 112 bands; q = (0, 1/2, 0) leaves the k
mesh, N2 = 45 is odd) and olivine56_gamma (144x45x40, ~2x10^4 plane waves, 224 bands), and
olivine28 itself (k 2x3x4 + 24 k+q entries) where its reference exists.  The GPU runs the
same pair in the launch configuration of the benchmark (every mesh k and band in one
batch), in FP64 (bar 1e-10 relative, element by element) and in the mixed form (1e-6).

The ground state is rebuilt here by the seeded generator (on the GPU when present); its
fingerprint (seed, sphere sizes, occupied energies, density integral) must match the one
stored with the reference, which holds when both builds converge their eigenpairs to a
residual far below the parity bar (1e-12 for these cells).
"""
import glob
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = sorted(glob.glob(os.path.join(HERE, "golden", "*.json")))


def _load(path):
    with open(path) as fh:
        g = json.load(fh)
    c = lambda a: np.asarray(a)[..., 0] + 1j * np.asarray(a)[..., 1]
    return g, c(g["dn0"]), c(g["dn"])


def _gs(name):
    from synth import cache
    return cache.get(name)


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-5] for p in GOLDEN])
def test_golden_reference(path):
    from paper_2203_15684_amd import hp
    g, dn0, dn = _load(path)
    gs = _gs(g["workload"])
    fp = g["fingerprint"]
    print(f"[golden] {g['workload']} site {g['site']} q {g['q']}", flush=True)
    assert int(gs.seed_used) == fp["seed_used"]
    assert [e.npw for e in gs.kpts] == fp["npw"]
    eps = np.array([e.eps for e in gs.kpts])
    assert np.abs(eps - np.array(fp["eps"])).max() < 1e-10
    assert abs(float(np.sum(gs.rho0)) - fp["rho0_sum"]) < 1e-10 * abs(fp["rho0_sum"])
    ctx = hp.hp_ground_state_load(gs)
    base = dict(conv_thr_chi=1e-12, conv_thr_v=1e-10, cg_tol=1e-12, niter_max=100, max_cg_iter=3000)
    d64 = hp.hp_sternheimer_scf(ctx, g["site"], g["q"], hp.ScfParams(**base, precision=hp.HP_FP64))
    assert d64[3] == 0, d64[2]
    e0, e1 = rel(d64[0], dn0), rel(d64[1], dn)
    print(f"[golden] FP64 dn0 {e0:.2e} dn {e1:.2e}", flush=True)
    assert e0 < 1e-10 and e1 < 1e-10
    mixed = dict(base, conv_thr_chi=1e-10, conv_thr_v=1e-8, cg_tol=1e-10)
    d32 = hp.hp_sternheimer_scf(ctx, g["site"], g["q"], hp.ScfParams(**mixed, precision=hp.HP_MIXED))
    assert d32[3] == 0, d32[2]
    e0, e1 = rel(d32[0], dn0), rel(d32[1], dn)
    print(f"[golden] mixed dn0 {e0:.2e} dn {e1:.2e}", flush=True)
    assert e0 < 1e-6 and e1 < 1e-6
    ctx.close()
