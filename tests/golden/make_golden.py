"""Write the stored full-size references of the GPU parity tests.

For one workload and one (perturbed site J, q) pair this runs the FP64 oracle alone
(the self-consistent Sternheimer response of Eqs. 12-18, in oracle/) and stores
Delta_q n0 (first SCF iteration: the chi0 column) and Delta_q n (self-consistent: the
chi column), [n_hub][5][5] complex, with the oracle's parameters, its wall time and core
count, and a fingerprint of the synthetic ground state it ran on (seed, sphere sizes,
every occupied energy, the density's integral), so that a test can check it is comparing
on the same inputs.  Nothing here calls the GPU library; the ground state comes from the
seeded input generator (synth/), built on the CPU.

    python tests/golden/make_golden.py olivine28_gamma --site 0 --q 0 0.5 0
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.hp_oracle import _workers  # noqa: E402


def fingerprint(gs):
    return {"seed_used": int(gs.seed_used), "npw": [int(e.npw) for e in gs.kpts],
            "k_frac": [[float(x) for x in e.k_frac] for e in gs.kpts],
            "eps": [[float(x) for x in e.eps] for e in gs.kpts],
            "rho0_sum": float(np.sum(gs.rho0)), "fft": [int(x) for x in gs.fft], "n_occ": int(gs.n_occ)}


def cplx(a):
    a = np.asarray(a)
    return np.stack([a.real, a.imag], axis=-1).tolist()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--site", type=int, default=0)
    ap.add_argument("--q", type=float, nargs=3, default=(0.0, 0.5, 0.0))
    ap.add_argument("--cg-tol", type=float, default=1e-13)
    ap.add_argument("--conv-thr-chi", type=float, default=1e-13)
    ap.add_argument("--conv-thr-v", type=float, default=1e-11)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    from synth import cache
    t0 = time.time()
    gs = cache.get(args.name, device="cpu", verbose=True)
    t_gs = time.time() - t0
    p = oracle.ScfParams(cg_tol=args.cg_tol, conv_thr_chi=args.conv_thr_chi, conv_thr_v=args.conv_thr_v)
    o = oracle.Oracle(gs, cache_limit_bytes=8e9)
    t0 = time.time()
    r = o.scf(args.site, np.array(args.q, dtype=float), p, verbose=True)
    wall = time.time() - t0
    out = {"workload": args.name, "site": args.site, "q": [float(x) for x in args.q],
           "oracle_params": {"cg_tol": args.cg_tol, "conv_thr_chi": args.conv_thr_chi,
                             "conv_thr_v": args.conv_thr_v, "niter_max": p.niter_max,
                             "alpha_mix": p.alpha_mix, "nmix": p.nmix},
           "converged": bool(r["converged"]), "scf_iters": int(r["iters"]), "cg_iters": int(r["cg_iters"]),
           "oracle_wall_s": round(wall, 1), "ground_state_build_s": round(t_gs, 1), "cores": _workers(),
           "fingerprint": fingerprint(gs), "dn0": cplx(r["dn0"]), "dn": cplx(r["dn"]),
           "made_by": "tests/golden/make_golden.py (oracle only)"}
    if not r["converged"]:
        raise SystemExit(f"the oracle did not converge in {r['iters']} iterations; nothing written")
    path = args.out or os.path.join(HERE, f"{args.name}_site{args.site}_q{'_'.join(f'{x:g}' for x in args.q)}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: {r['iters']} SCF iterations, {wall:.0f} s on {_workers()} cores", flush=True)


if __name__ == "__main__":
    main()
