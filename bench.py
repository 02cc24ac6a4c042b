"""Benchmark of the DFPT Hubbard-response Sternheimer path on one MI355X.

One step = one self-consistent Sternheimer solve of one (perturbed site J, q) pair
(hp_sternheimer_scf): every SCF iteration builds the right-hand sides of Eq. 15 for all
occupied bands of all mesh k, solves them in one batched PCG launch sequence (H applies:
kinetic term, FFT round trip for V_loc, projector GEMMs on the matrix cores), rebuilds
the response density and the Hartree + LDA response potential, mixes, and contracts the
response occupations of Eq. 13.  Steps cycle through the N_hub x N_q pairs of the q mesh
(site fastest).  The chi(q) column of each pair (Eq. 12's input) is the trace of its
response occupations; the full response matrix, U and V need every pair, so the whole
job's time is the per-pair time times the number of pairs (reported as extrapolated).

Default workload: the 2x1x1 supercell of the olivine-shaped cell (56 atoms, 8 d sites,
~2x10^4 plane waves, FFT 144x45x40, 224 bands, k 2x3x4, q 1x2x2: 32 pairs, 5,376 band
solves per launch), the largest single-GPU configuration.  Inputs are generated once and
resident in HBM before timing.

Forms, all on the same resident inputs and the same pairs:
  mixed          FP32 FFTs / V psi / projection GEMMs inside the PCG, FP64 residual
                 refinement, FP64 orthogonalization, scalars and occupations (headline);
  fp64           plain FP64 at the configured tolerances;
  fp64_relaxed   FP64 with the loosest tolerances that keep every chi column within 1e-6
                 of the fp64 form (the precision-vs-tolerance control);
  mixed_relaxed  the mixed form at the same relaxed tolerances;
  mixed_bf16, mixed_bf16_pv32, mixed_graphs  (optional) BF16 projections, BF16 KB with
                 FP32 P_v, and CG iterations replayed from captured hipGraphs;
  mixed_refine_all  (optional ablation) the mixed form with every solve FP64-refined
                 (lowp_trust_tol 1: no solve finished in FP32 alone);
  any form as "<form>@cg_tol:conv_thr_chi:conv_thr_v[:inner_tol]" for tolerance sweeps.
The mixed form is timed over --steps pairs after --warmup pairs; every other form over
the first --ref-steps of those pairs.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Sternheimer SCF wall time + Hψ applies/s, mixed-batched vs FP64, at χ err"
HA_EV = 27.211386245988
PEAK = {"fp64_vector": 78.6e12, "fp64_mfma": 78.6e12, "fp32_vector": 157.3e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}
# The relaxed forms: the loosest of the swept tolerances whose chi columns stay within
# 1e-6 of the FP64 form at the configured tolerance (cg_tol, conv_thr_chi, conv_thr_v).
RELAXED = (1e-5, 1e-7, 1e-4)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ref-steps", type=int, default=3, help="timed pairs of every form other than --precision")
    ap.add_argument("--config", default="olivine56_sc211")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--projectors", default="atomic", choices=["atomic", "ortho-atomic"],
                    help="Hubbard projectors: the atomic d orbitals, or Loewdin ortho-atomic ones built at load")
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--cg-tol", type=float, default=1e-10)
    ap.add_argument("--conv-thr-chi", type=float, default=1e-10)
    ap.add_argument("--conv-thr-v", type=float, default=1e-8)
    ap.add_argument("--niter-max", type=int, default=100, help="SCF iteration limit (the paper's niter_max)")
    ap.add_argument("--alpha-mix", type=float, default=0.3, help="mixing factor (the paper's alpha_mix)")
    ap.add_argument("--nmix", type=int, default=4, help="mixing history length (the paper's nmix), 1..8")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="mixed,fp64,fp64_relaxed,mixed_relaxed,mixed_graphs",
                    help="comma-separated forms (must include fp64 and --precision)")
    ap.add_argument("--graph-chunk", type=int, default=0,
                    help="CG iterations per captured hipGraph launch in the main forms (0: launch kernels one by "
                         "one, timed with HIP events)")
    ap.add_argument("--verbosity", type=int, default=0, help="1: one line per SCF iteration on stderr")
    ap.add_argument("--cache-ground-state", action="store_true",
                    help="write a newly built ground state to the on-disk cache for later runs")
    ap.add_argument("--full-response", action="store_true",
                    help="also run the whole response (hp_response_matrix over every pair, then U/V) once per form "
                         "and report its wall time, status and the chi and U/V differences from the FP64 form")
    return ap.parse_args()


def fft_flops(n):
    return 5.0 * n * math.log2(n)


def plane_flops(gs, entry):
    """Algorithmic flops of one xy-plane round trip for the local potential on the sphere of
    `entry`: radix FFTs along y on the columns that hold sticks and along x on every row,
    both directions, plus the real x complex product (5 N log2 N per complex FFT)."""
    n1, n2, _ = gs.fft
    m1 = set(int(m) % n1 for m in gs.kpts[entry].miller[:, 0])
    return 2.0 * (len(m1) * fft_flops(n2) + n2 * fft_flops(n1)) + 2.0 * n1 * n2


def kq_entries(gs, q):
    import numpy as np
    out = []
    for ik in range(gs.n_mesh):
        kq = gs.kpts[ik].k_frac + q
        for j, e in enumerate(gs.kpts):
            d = kq - e.k_frac
            if np.all(np.abs(d - np.round(d)) < 1e-9):
                out.append(j)
                break
    return out


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2203_15684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def roofline(gs, prof, q_list, h_applies):
    """Roofline record of the kernel with the largest measured GPU time.

    Every H apply of the batched CG launches the operator kernels once over all (mesh k,
    band) items of one (site, q) problem; converged items exit at once, so the work of a
    launch is counted per performed single-band apply:
    achieved = (single-band applies) x (algorithmic work per band) / (summed launch time).
    h_applies: single-band applies of the precision the dominant kernel runs in."""
    import numpy as np
    name, (calls, ms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_s = ms / max(calls, 1) * 1e-3
    n3 = gs.fft[2]
    items_per_launch = h_applies / max(calls, 1)
    ej_all = [j for q in q_list for j in kq_entries(gs, np.array(q))]
    lowp = name.endswith("32")
    base = name[:-2] if lowp else name
    bytes_c = 8.0 if lowp else 16.0
    if base == "plane_vloc":
        per_item = float(np.mean([plane_flops(gs, j) for j in ej_all])) * n3
        peak = PEAK["fp32_vector" if lowp else "fp64_vector"]
        rec = {"bound": "alu", "achieved": per_item * items_per_launch / avg_s / 1e12, "peak": peak / 1e12,
               "unit": "TFLOP/s"}
    elif base in ("zproj", "zexpand"):
        m = gs.n_beta + gs.n_occ
        per_item = float(np.mean([8.0 * m * gs.kpts[j].npw for j in ej_all]))
        peak = PEAK["fp32_mfma" if lowp else "fp64_mfma"]
        rec = {"bound": "mfma", "achieved": per_item * items_per_launch / avg_s / 1e12, "peak": peak / 1e12,
               "unit": "TFLOP/s"}
    else:
        per_item = float(np.mean([bytes_c * 3 * gs.kpts[j].npw for j in ej_all]))
        rec = {"bound": "hbm", "achieved": per_item * items_per_launch / avg_s / 1e9,
               "peak": PEAK["hbm"] / 1e9, "unit": "GB/s"}
    rec["frac"] = rec["achieved"] / rec["peak"]
    rec["kernel"] = name
    rec["avg_launch_ms"] = avg_s * 1e3
    rec["launches"] = calls
    rec["items_per_launch"] = items_per_launch
    rec["work_per_item"] = per_item
    rec["traffic"] = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{name}_{gs.spec.name}.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        if t.get("source_hash") == source_hash(t.get("source_files", [])):
            rec["traffic"] = t["bytes_per_item"] * items_per_launch
            rec["traffic_unit"] = "bytes per launch (HBM, measured, calibrated)"
    return rec


def cpu_baseline(gs, seconds, q, applies_per_pair_fp64, n_pairs):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload: the
    Sternheimer operator of Eq. 15 (H apply with the FFT local potential and the KB
    projectors, the alpha P_v shift, minus eps) on every occupied band of one mesh k of
    the timed (site, q) pair, repeated for about `seconds`.  Its rate, divided into the
    single-band applies the FP64 GPU form performs per (site, q) SCF solve, gives the
    oracle's seconds per solve (extrapolated, not run)."""
    import numpy as np
    import oracle
    from oracle.hp_oracle import _workers
    o = oracle.Oracle(gs, cache_limit_bytes=0)
    ik = 0
    X = gs.kpts[ik].u
    o.sternheimer_op(ik, q, X)  # plan caches
    t0 = time.perf_counter()
    reps = 0
    while True:
        o.sternheimer_op(ik, q, X)
        reps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    rate = reps * X.shape[0] / dt
    j, _ = o.kq_entry(ik, q)
    per_pair = applies_per_pair_fp64 / rate
    return {"value": rate, "unit": "Hpsi/s", "cores": _workers(), "kind": "oracle",
            "sample": f"oracle Sternheimer operator (Eq. 15 LHS: FFT local potential, KB projectors, alpha P_v) on "
                      f"{X.shape[0]} bands x {reps} repetitions at mesh k 0 -> k+q entry {j} "
                      f"({gs.kpts[j].npw} plane waves) of {gs.spec.name}, {dt:.1f} s",
            "s_per_site_q_scf_extrapolated": per_pair,
            "s_full_response_extrapolated": per_pair * n_pairs,
            "extrapolation": "single-band applies of the FP64 GPU form per (site, q) SCF solve / oracle rate"}


def gemm_rates(gs, prof, q_list, a64, a32):
    """MFMA rate of the projection GEMMs averaged over the timed run: the flops of the H
    applies' projection (or expansion) over the stacked table (n_beta KB rows and n_occ
    alpha P_v rows, 8 flops per complex multiply-add) per performed single-band apply,
    divided by the summed time of every launch of that kernel.  The FP32 kernels run only
    inside H applies; the FP64 ones also serve P_c, the Hubbard terms and Eq. 13, whose
    flops are not counted, so their rate is a lower bound."""
    import numpy as np
    ej_all = [j for q in q_list for j in kq_entries(gs, np.array(q))]
    per_item = float(np.mean([8.0 * (gs.n_beta + gs.n_occ) * gs.kpts[j].npw for j in ej_all]))
    out = {}
    for name, n, peak in (("zproj32", a32, PEAK["fp32_mfma"]), ("zexpand32", a32, PEAK["fp32_mfma"]),
                          ("zproj", a64, PEAK["fp64_mfma"]), ("zexpand", a64, PEAK["fp64_mfma"])):
        calls, ms = prof.get(name, (0, 0.0))
        if calls and ms > 0 and n:
            tf = per_item * n / (ms * 1e-3) / 1e12
            out[name] = {"achieved_tflops": round(tf, 2), "peak": peak / 1e12, "frac": round(tf * 1e12 / peak, 3),
                         "launches": calls, "ms": round(ms, 1)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the (site, q) problems would be "
              "sharded across GPUs with no collective, see the design notes.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from synth import cache
    from paper_2203_15684_amd import hp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    gs = cache.get(args.config, save_built=args.cache_ground_state)
    t_gen = time.time() - t0
    print(f"[bench] ground state {gs.spec.name} ready ({t_gen:.1f} s)", file=sys.stderr, flush=True)
    load_kw = {}
    if args.projectors == "ortho-atomic":
        import synth
        t0 = time.time()
        atw, hub_rows = synth.atomic_orbital_tables(gs)
        t_gen += time.time() - t0
        load_kw = {"atwfc": atw, "hub_rows": hub_rows}
    free_before_load = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    ctx = hp.hp_ground_state_load(gs, **load_kw)
    load_kw = None
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    free_loaded = torch.cuda.mem_get_info()[0]
    q_list = [tuple(float(x) for x in q) for q in gs.qpoints()]
    pairs = [(s, q) for q in q_list for s in range(gs.n_hub)]

    g = args.graph_chunk
    base_tol = (args.cg_tol, args.conv_thr_chi, args.conv_thr_v)
    # (precision, tolerances, low-precision GEMMs, graph chunk, lowp_trust_tol)
    named = {"mixed": ("mixed", base_tol, hp.HP_GEMM_FP32, g, 1e-6), "fp64": ("fp64", base_tol, 0, g, 1e-6),
             "fp64_relaxed": ("fp64", RELAXED, 0, g, 1e-6),
             "mixed_relaxed": ("mixed", RELAXED, hp.HP_GEMM_FP32, g, 1e-6),
             "mixed_bf16": ("mixed", base_tol, hp.HP_GEMM_BF16, g, 1e-6),
             "mixed_bf16_pv32": ("mixed", base_tol, hp.HP_GEMM_BF16_PV32, g, 1e-6),
             "mixed_graphs": ("mixed", base_tol, hp.HP_GEMM_FP32, 8, 1e-6),
             "mixed_refine_all": ("mixed", base_tol, hp.HP_GEMM_FP32, g, 1.0)}
    form_def = {}
    for f in args.forms.split(","):
        if "@" in f:
            b, tl = f.split("@")
            if b not in named:
                raise SystemExit(f"unknown form {b}")
            t = tuple(float(x) for x in tl.split(":"))
            if len(t) not in (3, 4):
                raise SystemExit(f"{f}: want <form>@cg_tol:conv_thr_chi:conv_thr_v[:inner_tol]")
            form_def[f] = (named[b][0], t) + named[b][2:]
        elif f in named:
            form_def[f] = named[f]
        else:
            raise SystemExit(f"unknown form {f}; choose from {', '.join(named)}")
    if args.precision not in form_def or "fp64" not in form_def:
        raise SystemExit("--forms must include fp64 and the --precision form")

    def params(form):
        prec, tols, lowp, chunk, trust = form_def[form]
        tol, thr_chi, thr_v = tols[:3]
        inner = tols[3] if len(tols) > 3 else args.inner_tol
        return hp.ScfParams(conv_thr_chi=thr_chi, conv_thr_v=thr_v, cg_tol=tol, niter_max=args.niter_max,
                            alpha_mix=args.alpha_mix, nmix=args.nmix, max_cg_iter=2000,
                            inner_tol=inner, graph_chunk=chunk, lowp_trust_tol=trust,
                            precision=hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED, lowp_gemm=lowp,
                            verbosity=args.verbosity)

    def pair(i):
        return pairs[i % len(pairs)]

    for i in range(args.warmup):
        s, q = pair(i)
        r = hp.hp_sternheimer_scf(ctx, s, q, params(args.precision))
        print(f"[bench] warm-up pair {i} (site {s}, q {q}): status {r[3]}, {r[2]['scf_iters']} SCF iterations",
              file=sys.stderr, flush=True)

    def timed(form, first, n):
        p = params(form)
        torch.cuda.synchronize()
        hp.hp_profile_start(ctx)
        t_start = time.perf_counter()
        res = []
        for i in range(first, first + n):
            s, q = pair(i)
            t1 = time.perf_counter()
            dn0, dn, st, status = hp.hp_sternheimer_scf(ctx, s, q, p)  # returns after the library synchronized
            res.append({"pair": i % len(pairs), "site": s, "q": q, "dn0": dn0, "dn": dn, "st": st, "status": status,
                        "wall": time.perf_counter() - t1})
        torch.cuda.synchronize()
        t = time.perf_counter() - t_start
        prof = hp.hp_profile_stop(ctx)
        return t, res, prof

    forms = [args.precision] + [f for f in form_def if f != args.precision]
    runs = {}
    first = args.warmup
    for f in forms:
        n = args.steps if f == args.precision else min(args.ref_steps, args.steps)
        runs[f] = timed(f, first, n)
        print(f"[bench] form {f}: {runs[f][0]:.2f} s over {n} pairs", file=sys.stderr, flush=True)
    full = {}
    if args.full_response:
        for f in forms:
            p = params(f)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            chi0, chi, mim, st, status = hp.hp_response_matrix(ctx, gs.qmesh, p)
            uv = hp.hp_hubbard_params(chi0, chi)
            full[f] = {"wall_s": time.perf_counter() - t1, "status": status, "scf_iters": st["scf_iters"],
                       "h_applies_fp64": st["h_applies_fp64"], "h_applies_lowp": st["h_applies_lowp"],
                       "chi0": chi0, "chi": chi, "uv": uv}
            print(f"[bench] full response {f}: {full[f]['wall_s']:.2f} s, status {status}", file=sys.stderr,
                  flush=True)
    hbm_used = free_before_load - torch.cuda.mem_get_info()[0]

    def column(r, key):
        """chi(q) column of the pair: chi_s = sum_m dn[s][m][m] (Eq. 12's input), complex."""
        return np.einsum("smm->s", r[key])

    ref = {r["pair"]: r for r in runs["fp64"][1]}
    summary = {}
    for f, (t, res, pr) in runs.items():
        a64 = sum(r["st"]["h_applies_fp64"] for r in res)
        a32 = sum(r["st"]["h_applies_lowp"] for r in res)
        pcg = sum(r["st"]["stage_s"][1] for r in res)
        d = max(pr.items(), key=lambda kv: kv[1][1])[0]
        prec, tols, lowp, chunk, trust = form_def[f]
        errs = []
        for r in res:
            if r["pair"] in ref:
                for key in ("dn0", "dn"):
                    c, c64 = column(r, key), column(ref[r["pair"]], key)
                    errs.append(float(np.abs(c - c64).max() / np.abs(c64).max()))
        same = [r for r in res if r["pair"] in ref]
        t_same = sum(r["wall"] for r in same)
        t_ref_same = sum(ref[r["pair"]]["wall"] for r in same)
        summary[f] = {"precision": prec, "cg_tol": tols[0], "conv_thr_chi": tols[1], "conv_thr_v": tols[2],
                      "inner_tol": (tols[3] if len(tols) > 3 else args.inner_tol) if prec == "mixed" else None,
                      "graph_chunk": chunk,
                      "lowp_trust_tol": trust if prec == "mixed" and lowp == 0 else None,
                      "kernel_timing": "device-clock stamps in graphs" if chunk else "hip events",
                      "projection_gemms": {0: "fp32", 1: "bf16", 2: "bf16 (KB), fp32 (P_v)"}[lowp]
                      if prec == "mixed" else "fp64",
                      "steps": len(res), "pairs": [r["pair"] for r in res],
                      "s_per_site_q_scf": t / len(res),
                      "s_per_site_q_scf_median": float(np.median([r["wall"] for r in res])),
                      "s_full_response_extrapolated": t / len(res) * len(pairs),
                      "hpsi_per_s": (a64 + a32) / t,
                      "pcg_s_per_step": pcg / len(res),
                      "hpsi_per_s_in_pcg": {"fp64": a64 / max(pcg, 1e-30), "lowp": a32 / max(pcg, 1e-30)},
                      "ms_per_scf_iteration": t / sum(r["st"]["scf_iters"] for r in res) * 1e3,
                      "h_applies_fp64_per_step": a64 / len(res), "h_applies_lowp_per_step": a32 / len(res),
                      "scf_iters": [r["st"]["scf_iters"] for r in res],
                      "cg_iters": [r["st"]["cg_iters"] for r in res],
                      "status": [r["status"] for r in res],
                      "chi_column_rel_err_vs_fp64": max(errs) if errs else None,
                      "speedup_vs_fp64_same_pairs": t_ref_same / t_same if t_same > 0 else None,
                      "kernel_ms": {k: round(v[1], 1) for k, v in pr.items() if v[0]},
                      "roofline": roofline(gs, pr, q_list, a32 if d.endswith("32") else a64),
                      "projection_gemm_mfma": gemm_rates(gs, pr, q_list, a64, a32)}
    t_total, res, prof = runs[args.precision]
    h64 = sum(r["st"]["h_applies_fp64"] for r in res)
    h32 = sum(r["st"]["h_applies_lowp"] for r in res)
    value = (h64 + h32) / t_total
    npws = [e.npw for e in gs.kpts]
    main_form = summary[args.precision]
    out = {
        "metric": METRIC, "value": value, "unit": "Hpsi/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_total / args.steps * 1e3,
        "ms_per_step_median": main_form["s_per_site_q_scf_median"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{gs.spec.name}: olivine-shaped cell {gs.spec.cell} bohr, {gs.spec.n_atoms} atoms, "
                               f"{gs.n_hub} d sites, {gs.n_occ} bands, FFT {'x'.join(map(str, gs.fft))}, "
                               f"k {'x'.join(map(str, gs.kmesh))}, q {'x'.join(map(str, gs.qmesh))}; "
                               f"a step is one (site, q) self-consistent Sternheimer solve, "
                               f"{gs.n_mesh * gs.n_occ} band solves per launch",
                   "npw_min": min(npws), "npw_max": max(npws), "k_entries": len(npws),
                   "site_q_pairs": len(pairs), "precision": args.precision, "cg_tol": args.cg_tol,
                   "conv_thr_chi": args.conv_thr_chi, "conv_thr_v": args.conv_thr_v, "inner_tol": args.inner_tol,
                   "niter_max": args.niter_max, "alpha_mix": args.alpha_mix, "nmix": args.nmix,
                   "projectors": args.projectors},
        "chi_column_rel_err_mixed_vs_fp64": summary["mixed"]["chi_column_rel_err_vs_fp64"]
        if "mixed" in summary else None,
        "speedup_mixed_vs_fp64_same_pairs": summary["mixed"]["speedup_vs_fp64_same_pairs"]
        if "mixed" in summary else None,
        "full_response_s_extrapolated": {f: s["s_full_response_extrapolated"] for f, s in summary.items()},
        "forms": summary,
        "roofline": main_form["roofline"],
        "roofline_fp64": summary["fp64"]["roofline"],
        "setup_s": {"ground_state": round(t_gen, 1), "load_from_host": round(t_load, 2)},
        # the boundary takes host arrays here: throughput with the one-time host-to-device load included
        "value_including_load": (h64 + h32) / (t_total + t_load),
        "autotune": hp.hp_tuning_report(ctx),
        "hbm_footprint_gb": {"context_after_all_forms": round(hbm_used / 1e9, 2),
                             "loaded_ground_state": round((free_before_load - free_loaded) / 1e9, 2)},
    }
    if full:
        r64 = full["fp64"]
        out["full_response"] = {
            f: {"wall_s": v["wall_s"], "status": v["status"], "scf_iters": v["scf_iters"],
                "h_applies_fp64": v["h_applies_fp64"], "h_applies_lowp": v["h_applies_lowp"],
                "speedup_vs_fp64": r64["wall_s"] / v["wall_s"],
                "chi_rel_err_vs_fp64": max(float(np.abs(v["chi0"] - r64["chi0"]).max() / np.abs(r64["chi0"]).max()),
                                           float(np.abs(v["chi"] - r64["chi"]).max() / np.abs(r64["chi"]).max())),
                "uv_err_meV_vs_fp64": float(np.abs(v["uv"] - r64["uv"]).max() * HA_EV * 1e3),
                "U_eV": [float(x) * HA_EV for x in np.diag(v["uv"])[:gs.n_hub]]}
            for f, v in full.items()}
    if not args.no_cpu_baseline:
        s0, q0 = pair(first)
        out["cpu_baseline"] = cpu_baseline(gs, args.cpu_baseline_seconds, np.array(q0),
                                           summary["fp64"]["h_applies_fp64_per_step"], len(pairs))
    print(json.dumps(out), flush=True)
    hp.hp_destroy(ctx)


if __name__ == "__main__":
    main()
