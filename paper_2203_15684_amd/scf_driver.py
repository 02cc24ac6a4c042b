"""Command-line driver: one self-consistent Sternheimer solve (one Hubbard site,
one q) on a synthetic workload, with the same launch configuration as the
full response (every mesh k and band in one batch).  Prints the statistics and
the per-kernel GPU times as JSON.

  python -m paper_2203_15684_amd.scf_driver --config olivine28 --site 0 --q 0 0.5 0
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="olivine28")
    ap.add_argument("--site", type=int, default=0)
    ap.add_argument("--q", type=float, nargs=3, default=[0.0, 0.5, 0.0])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cg-tol", type=float, default=1e-10)
    ap.add_argument("--conv-thr-chi", type=float, default=1e-10)
    ap.add_argument("--conv-thr-v", type=float, default=1e-8)
    ap.add_argument("--niter-max", type=int, default=100)
    ap.add_argument("--alpha-mix", type=float, default=0.3)
    ap.add_argument("--nmix", type=int, default=4)
    ap.add_argument("--verbosity", type=int, default=0)
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--max-refine", type=int, default=12)
    ap.add_argument("--graph-chunk", type=int, default=8)
    ap.add_argument("--lowp-gemm", type=int, default=0, help="0 FP32, 1 BF16, 2 BF16 with P_v in FP32")
    ap.add_argument("--lowp-trust-tol", type=float, default=1e-6,
                    help="mixed: solves at or above this tolerance skip FP64 refinement (1: refine every solve)")
    ap.add_argument("--plane-variant32", type=int, default=-1,
                    help="pin the FP32 plane-FFT variant (hp_set_plane_variant) instead of the tuner's choice")
    ap.add_argument("--stick-variant32", type=int, default=-1,
                    help="pin both FP32 z-transform variants (hp_set_stick_variant)")
    a = ap.parse_args()
    from synth import cache
    from paper_2203_15684_amd import hp
    gs = cache.get(a.config)
    ctx = hp.hp_ground_state_load(gs)
    p = hp.ScfParams(conv_thr_chi=a.conv_thr_chi, conv_thr_v=a.conv_thr_v, cg_tol=a.cg_tol,
                     niter_max=a.niter_max, alpha_mix=a.alpha_mix, nmix=a.nmix, max_cg_iter=2000,
                     verbosity=a.verbosity,
                     precision=hp.HP_FP64 if a.precision == "fp64" else hp.HP_MIXED,
                     inner_tol=a.inner_tol, max_refine=a.max_refine, graph_chunk=a.graph_chunk,
                     lowp_gemm=a.lowp_gemm, lowp_trust_tol=a.lowp_trust_tol)
    if a.plane_variant32 >= 0:
        hp.hp_set_plane_variant(ctx, 32, a.plane_variant32)
    if a.stick_variant32 >= 0:
        hp.hp_set_stick_variant(ctx, 32, a.stick_variant32, a.stick_variant32)
    hp.hp_profile_start(ctx)
    dn0, dn, st, status = hp.hp_sternheimer_scf(ctx, a.site, a.q, p)
    prof = hp.hp_profile_stop(ctx)
    chi0 = [complex(x) for x in dn0.trace(axis1=1, axis2=2)]
    chi = [complex(x) for x in dn.trace(axis1=1, axis2=2)]
    print(json.dumps({"config": a.config, "site": a.site, "q": a.q, "status": status, "stats": st,
                      "chi0_q": [[c.real, c.imag] for c in chi0], "chi_q": [[c.real, c.imag] for c in chi],
                      "kernel_ms": prof}))
    hp.hp_destroy(ctx)


if __name__ == "__main__":
    main()
