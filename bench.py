"""Benchmark of the DFPT Hubbard-response Sternheimer path on one MI355X.

One step = the whole hot path over one synthetic workload: the self-consistent
Sternheimer solves (Eq. 15) for every Hubbard site and every q of the q-mesh
(hp_response_matrix: RHS, batched PCG with H applies, response density,
Hartree + LDA kernel, mixing, response occupations, the q-sum of Eq. 12) and the
U/V inversion (Eqs. 8-9).  The default workload is the olivine-shaped cell
(28 atoms, 4 d sites, ~10^4 plane waves, FFT 72x45x40, 112 bands, k 2x3x4,
q 1x2x2).  Inputs are generated once and are resident in HBM before timing.

Both forms run in the same invocation on the same resident inputs: the
mixed-precision batched form (FP32 FFTs and FP32 MFMA projections inside the PCG,
FP64 residual refinement, FP64 orthogonalization, scalars, chi and inversion) and
the plain FP64 form.  Prints one JSON line: value = single-band H applications per
second of the --precision form over its timed steps (whole job), ms_per_step = its
Sternheimer SCF wall time per step; "forms" holds both forms, and the chi / U,V
difference of the mixed form against the FP64 form is reported.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="olivine28")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--projectors", default="atomic", choices=["atomic", "ortho-atomic"],
                    help="Hubbard projectors: the atomic d orbitals, or Loewdin ortho-atomic ones built at load")
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--cg-tol", type=float, default=1e-10)
    ap.add_argument("--conv-thr-chi", type=float, default=1e-10)
    ap.add_argument("--conv-thr-v", type=float, default=1e-8)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--relaxed-cg-tol", type=float, default=1e-7,
                    help="cg_tol of the relaxed FP64 / mixed forms")
    ap.add_argument("--forms", default="mixed,fp64,fp64_relaxed",
                    help="comma-separated forms to time (must include fp64 and --precision); also available: "
                         "mixed_relaxed, mixed_bf16, mixed_bf16_pv32, mixed_graphs")
    ap.add_argument("--verbosity", type=int, default=0, help="1: one line per SCF iteration on stderr")
    ap.add_argument("--graph-chunk", type=int, default=0,
                    help="CG iterations per captured hipGraph launch in the main forms (0: launch kernels one by "
                         "one, timed with HIP events)")
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


def roofline(gs, prof, nq_list, h_applies):
    """h_applies: single-band applies of the precision the dominant kernel runs in."""
    """Roofline record of the kernel with the largest measured GPU time.

    Every H apply of the batched CG launches the operator kernels once over all
    (mesh k, band) items of one (site, q) problem; converged items exit at once, so
    the work of a launch is counted per performed single-band apply:
    achieved = (single-band applies) x (algorithmic work per band) / (summed launch time)."""
    import numpy as np
    name, (calls, ms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_s = ms / max(calls, 1) * 1e-3
    n3 = gs.fft[2]
    nb = gs.n_occ
    items_per_launch = h_applies / max(calls, 1)
    ej_all = [j for q in nq_list for j in kq_entries(gs, np.array(q))]
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


def cpu_baseline(gs, seconds):
    """The FP64 oracle's H apply timed on the host cores on a bounded sample."""
    import numpy as np
    import oracle
    from oracle.hp_oracle import _workers
    o = oracle.Oracle(gs, cache_limit_bytes=0)
    e = gs.kpts[0]
    X = e.u
    o.h_apply(0, X[:2])  # plan caches
    t0 = time.perf_counter()
    reps = 0
    while True:
        o.h_apply(0, X)
        reps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": reps * X.shape[0] / dt, "unit": "Hpsi/s", "cores": _workers(), "kind": "oracle",
            "sample": f"oracle H apply (FFT local potential + KB projectors), {X.shape[0]} bands x {reps} "
                      f"repetitions at one k-point of {gs.spec.name} ({e.npw} plane waves), {dt:.1f} s"}


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
    gs = cache.get(args.config)
    t_gen = time.time() - t0
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
    nq = gs.qmesh
    nq_list = [tuple(q) for q in gs.qpoints()]

    # forms: name -> (precision, cg_tol). The relaxed forms separate the gain of the precision
    # from the gain of a looser Sternheimer tolerance: the loosest cg_tol that still keeps chi
    # within 1e-6 of the FP64 form at the configured tolerance.
    # (the BF16 forms put the KB and P_v projections of the inner solves on BF16 MFMA, or
    # only the KB ones with P_v kept in FP32)
    # (mixed_graphs replays the CG iterations from captured hipGraphs; its per-kernel times
    # come from device-clock stamps, every other form's from HIP events)
    g = args.graph_chunk
    form_def = {"mixed": ("mixed", args.cg_tol, hp.HP_GEMM_FP32, g), "fp64": ("fp64", args.cg_tol, 0, g),
                "fp64_relaxed": ("fp64", args.relaxed_cg_tol, 0, g),
                "mixed_relaxed": ("mixed", args.relaxed_cg_tol, hp.HP_GEMM_FP32, g),
                "mixed_bf16": ("mixed", args.cg_tol, hp.HP_GEMM_BF16, g),
                "mixed_bf16_pv32": ("mixed", args.cg_tol, hp.HP_GEMM_BF16_PV32, g),
                "mixed_graphs": ("mixed", args.cg_tol, hp.HP_GEMM_FP32, 8)}
    wanted = args.forms.split(",")
    for f in wanted:
        if f not in form_def:
            raise SystemExit(f"unknown form {f}; choose from {', '.join(form_def)}")
    if args.precision not in wanted or "fp64" not in wanted:
        raise SystemExit("--forms must include fp64 and the --precision form")
    form_def = {f: form_def[f] for f in wanted}

    def params(form):
        prec, tol, lowp, chunk = form_def[form]
        return hp.ScfParams(conv_thr_chi=args.conv_thr_chi, conv_thr_v=args.conv_thr_v, cg_tol=tol,
                            niter_max=100, max_cg_iter=2000, inner_tol=args.inner_tol, graph_chunk=chunk,
                            precision=hp.HP_FP64 if prec == "fp64" else hp.HP_MIXED, lowp_gemm=lowp,
                            verbosity=args.verbosity)

    def step(p):
        chi0, chi, mim, st, status = hp.hp_response_matrix(ctx, nq, p)
        uv = hp.hp_hubbard_params(chi0, chi)
        return chi0, chi, uv, st, status

    def timed(prec, steps):
        p = params(prec)
        torch.cuda.synchronize()
        hp.hp_profile_start(ctx)
        t_start = time.perf_counter()
        res, per_step = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            res.append(step(p))   # step() returns after the library has synchronized
            per_step.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        t = time.perf_counter() - t_start
        prof = hp.hp_profile_stop(ctx)
        timed.per_step[prec] = per_step
        return t, res, prof
    timed.per_step = {}

    forms = [args.precision] + [f for f in form_def if f != args.precision]
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(args.warmup):
        step(params(args.precision))
        print(f"[bench] warm-up step done", file=sys.stderr, flush=True)
    runs = {}
    for f in forms:
        runs[f] = timed(f, args.steps if f == args.precision else 1)
        print(f"[bench] form {f}: {runs[f][0]:.2f} s", file=sys.stderr, flush=True)
    hbm_used = free_before_load - torch.cuda.mem_get_info()[0]
    t_total, results, prof = runs[args.precision]
    chi0, chi, uv, st, status = results[-1]
    h64 = sum(r[3]["h_applies_fp64"] for r in results)
    h32 = sum(r[3]["h_applies_lowp"] for r in results)
    value = (h64 + h32) / t_total
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    rec = roofline(gs, prof, nq_list, h32 if dom.endswith("32") else h64)
    summary = {}
    for f, (t, res, pr) in runs.items():
        c0, c1, u, s_, stat = res[-1]
        a64 = sum(r[3]["h_applies_fp64"] for r in res)
        a32 = sum(r[3]["h_applies_lowp"] for r in res)
        d = max(pr.items(), key=lambda kv: kv[1][1])[0]
        summary[f] = {"precision": form_def[f][0], "cg_tol": form_def[f][1], "graph_chunk": form_def[f][3],
                      "kernel_timing": "device-clock stamps in graphs" if form_def[f][3] else "hip events",
                      "projection_gemms": {0: "fp32", 1: "bf16", 2: "bf16 (KB), fp32 (P_v)"}[form_def[f][2]]
                      if form_def[f][0] == "mixed" else "fp64",
                      "scf_wall_s_per_step": t / len(res), "hpsi_per_s": (a64 + a32) / t,
                      "scf_wall_s_median_step": float(np.median(timed.per_step[f])),
                      "steps": len(res),
                      # single-band applies per second of PCG time (stage 1 of the library's
                      # per-stage GPU timing), FP64 and low precision separately
                      "pcg_s_per_step": sum(r[3]["stage_s"][1] for r in res) / len(res),
                      "hpsi_per_s_in_pcg": {"fp64": a64 / max(sum(r[3]["stage_s"][1] for r in res), 1e-30),
                                            "lowp": a32 / max(sum(r[3]["stage_s"][1] for r in res), 1e-30)},
                      "ms_per_scf_iteration": t / sum(r[3]["scf_iters"] for r in res) * 1e3,
                      "h_applies_fp64": a64 / len(res), "h_applies_fp32": a32 / len(res),
                      "scf_iters": s_["scf_iters"], "cg_iters": s_["cg_iters"], "status": stat,
                      "kernel_ms": {k: round(v[1], 1) for k, v in pr.items() if v[0]},
                      "roofline": roofline(gs, pr, nq_list, a32 if d.endswith("32") else a64)}
    r64 = runs["fp64"][1][-1]
    for f, (t, res, pr) in runs.items():
        r = res[-1]
        summary[f]["chi_rel_err_vs_fp64"] = max(float(np.abs(r[0] - r64[0]).max() / np.abs(r64[0]).max()),
                                                float(np.abs(r[1] - r64[1]).max() / np.abs(r64[1]).max()))
        summary[f]["uv_err_meV_vs_fp64"] = float(np.abs(r[2] - r64[2]).max() * HA_EV * 1e3)
        summary[f]["speedup_vs_fp64"] = (runs["fp64"][0] / len(runs["fp64"][1])) / (t / len(res))
    chi_err = summary["mixed"]["chi_rel_err_vs_fp64"]
    uv_err_mev = summary["mixed"]["uv_err_meV_vs_fp64"]
    npws = [e.npw for e in gs.kpts]
    out = {
        "metric": METRIC, "value": value, "unit": "Hpsi/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_total / args.steps * 1e3,
        "ms_per_step_median": summary[args.precision]["scf_wall_s_median_step"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{gs.spec.name}: olivine-shaped cell {gs.spec.cell} bohr, {gs.spec.n_atoms} atoms, "
                               f"{gs.n_hub} d sites, {gs.n_occ} bands, FFT {'x'.join(map(str, gs.fft))}, "
                               f"k {'x'.join(map(str, gs.kmesh))}, q {'x'.join(map(str, gs.qmesh))}",
                   "npw_min": min(npws), "npw_max": max(npws), "k_entries": len(npws),
                   "precision": args.precision, "cg_tol": args.cg_tol, "conv_thr_chi": args.conv_thr_chi,
                   "conv_thr_v": args.conv_thr_v, "inner_tol": args.inner_tol,
                   "site_q_pairs": gs.n_hub * len(nq_list), "projectors": args.projectors},
        "chi_rel_err_mixed_vs_fp64": chi_err, "uv_err_meV_mixed_vs_fp64": uv_err_mev,
        "speedup_mixed_vs_fp64": summary["mixed"]["speedup_vs_fp64"],
        "forms": summary,
        "chi0_diag": [float(x) for x in np.diag(chi0)[:gs.n_hub]],
        "chi_diag": [float(x) for x in np.diag(chi)[:gs.n_hub]],
        "U_eV": [float(x) * HA_EV for x in np.diag(uv)[:gs.n_hub]],
        "V_nearest_neighbours_eV": [{"I": i, "J": j, "d_bohr": round(d, 4), "V": float(uv[i, j]) * HA_EV}
                                    for i, j, d in hp.hp_neighbours(gs.cell, gs.hub_tau, gs.qmesh)],
        "roofline": rec,
        "setup_s": {"ground_state": round(t_gen, 1), "load_from_host": round(t_load, 2)},
        # the boundary takes host arrays: throughput with the one-time host-to-device load included
        "value_including_load": (h64 + h32) / (t_total + t_load),
        "autotune": hp.hp_tuning_report(ctx),
        "hbm_footprint_gb": {"context_after_all_forms": round(hbm_used / 1e9, 2),
                             "loaded_ground_state": round((free_before_load - free0) / 1e9, 2)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(gs, args.cpu_baseline_seconds)
    print(json.dumps(out), flush=True)
    hp.hp_destroy(ctx)


if __name__ == "__main__":
    main()
