"""On-disk cache of generated ground states (within one machine session).

Generating the olivine-shaped systems takes minutes on the host; the cache keeps
the occupied states, energies and grids of a built system in an .npz file under
$HP_SYNTH_CACHE (default /tmp/hp_synth_cache) and rebuilds the projector tables
from their closed forms on load.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

from . import system as S


def cache_dir() -> str:
    d = os.environ.get("HP_SYNTH_CACHE", "/tmp/hp_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _path(name: str) -> str:
    return os.path.join(cache_dir(), f"{name}.npz")


def save(gs: S.GroundState) -> str:
    p = _path(gs.spec.name)
    arrs = {"vloc": gs.vloc, "rho0": gs.rho0, "tau": gs.tau, "hub_atoms": gs.hub_atoms, "hub_zeta": gs.hub_zeta,
            "kb_s": gs.kb_s, "kb_d": gs.kb_d, "d_kb": gs.d_kb, "cell": gs.cell,
            "meta": np.array([gs.seed_used, gs.n_mesh, len(gs.kpts), gs.gap, gs.nspin], dtype=np.float64)}
    if gs.hub_pot is not None:
        arrs["hub_pot"] = gs.hub_pot
    for i, e in enumerate(gs.kpts):
        arrs[f"k{i}_kfrac"] = e.k_frac
        arrs[f"k{i}_scal"] = np.array([e.weight, e.ecut, e.eps_next, e.resid])
        arrs[f"k{i}_miller"] = e.miller
        arrs[f"k{i}_eps"] = e.eps
        arrs[f"k{i}_u"] = e.u
    tmp = p + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, p)
    return p


def load(name: str):
    p = _path(name)
    if not os.path.exists(p):
        return None
    spec = S.SPECS[name]
    z = np.load(p, allow_pickle=False)
    meta = z["meta"]
    seed, n_mesh, nk, gap = int(meta[0]), int(meta[1]), int(meta[2]), float(meta[3])
    nspin = int(meta[4]) if meta.shape[0] > 4 else 1
    shell = S._Shell(z["cell"], z["tau"], z["hub_atoms"], z["hub_zeta"], z["kb_s"], z["kb_d"])
    kpts = []
    for i in range(nk):
        kf = z[f"k{i}_kfrac"]
        w, ecut, en, rs = z[f"k{i}_scal"]
        mil = z[f"k{i}_miller"]
        beta, phi = S.projector_tables(shell, kf, mil)
        kpts.append(S.KEntry(k_frac=kf, weight=float(w), ecut=float(ecut), miller=mil, eps=z[f"k{i}_eps"],
                             u=z[f"k{i}_u"], beta=beta, phi=phi, eps_next=float(en), resid=float(rs)))
    return S.GroundState(spec=spec, seed_used=seed, cell=z["cell"], fft=tuple(spec.fft), vloc=z["vloc"],
                         rho0=z["rho0"], tau=z["tau"], hub_atoms=z["hub_atoms"], hub_zeta=z["hub_zeta"],
                         kb_s=z["kb_s"], kb_d=z["kb_d"], d_kb=z["d_kb"], n_occ=spec.n_occ, kmesh=tuple(spec.kmesh),
                         qmesh=tuple(spec.qmesh), kpts=kpts, n_mesh=n_mesh, gap=gap,
                         spin_factor=2 if nspin == 1 else 1, nspin=nspin,
                         hub_pot=z["hub_pot"] if "hub_pot" in z.files else None)


def get(name: str, device: str = "auto", verbose: bool = None, save_built: bool = True):
    """Cached ground state of a named workload, generated on first use (progress on stderr
    for the large systems); save_built=False skips writing a newly built one to disk."""
    gs = load(name)
    if gs is not None:
        return gs
    if verbose is None:
        verbose = S.SPECS[name].n_occ >= 100
    if device == "auto":
        try:
            import torch
            device = "cuda" if torch.cuda.is_available() else "cpu"
        except Exception:
            device = "cpu"
    t = time.time()
    if verbose:
        _stdout = sys.stdout
        sys.stdout = sys.stderr  # progress lines go to stderr
    try:
        gs = S.build_ground_state(name, device=device, verbose=verbose)
    finally:
        if verbose:
            sys.stdout = _stdout
    if verbose:
        print(f"[synth] built {name} on {device} in {time.time() - t:.1f} s", file=sys.stderr, flush=True)
    if save_built:
        save(gs)
    return gs
