"""Python binding of the C ABI in include/hp.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  All arithmetic
runs in the HIP library libhp.so; this module only converts numpy arrays to the
C structs and pointers and raises HpError on error statuses.  Importing it
without a built library raises immediately: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhp.so")

HP_OK = 0
HP_WARN_NOT_CONVERGED = 1
HP_ERR_ARG, HP_ERR_SHAPE, HP_ERR_HIP, HP_ERR_OOM, HP_ERR_STATE, HP_ERR_SINGULAR, HP_ERR_NUMERIC = -1, -2, -3, -4, -5, -6, -7
HP_FP64, HP_MIXED = 0, 1
HP_GEMM_FP32, HP_GEMM_BF16, HP_GEMM_BF16_PV32 = 0, 1, 2
HP_XC_LDA_PZ81 = 1
HP_PROJ_ATOMIC, HP_PROJ_ORTHO_ATOMIC = 0, 1


class HpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hp status {status}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2203_15684_amd/build.py (hipcc, gfx950)")
# One HIP runtime per process: PyTorch ships its own libamdhip64.so.7.  Loading it
# first makes the library's dependency resolve to that same copy, so device memory
# and streams from torch and from this library share one runtime.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class HpKpoint(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("k_frac", C.c_double * 3), ("weight", C.c_double),
                ("npw", C.c_int32), ("miller", _ip), ("eps", _dp), ("u", _dp), ("beta", _dp), ("phi", _dp),
                ("atwfc", _dp)]


class HpGroundState(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("cell", (C.c_double * 3) * 3), ("fft", C.c_int32 * 3),
                ("v_loc", _dp), ("rho0", _dp), ("n_occ", C.c_int32), ("n_beta", C.c_int32), ("n_hub", C.c_int32),
                ("d_kb", _dp), ("hub_tau", _dp), ("spin_factor", C.c_int32), ("n_mesh", C.c_int32),
                ("n_kpts", C.c_int32), ("kpts", C.POINTER(HpKpoint)), ("xc", C.c_int32), ("inputs_on_device", C.c_int32),
                ("stream", C.c_void_p), ("projectors", C.c_int32), ("n_atwfc", C.c_int32), ("hub_rows", _ip),
                ("nspin", C.c_int32), ("hub_pot", _dp), ("degauss", C.c_double), ("efermi", C.c_double)]


class HpScfParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("conv_thr_chi", C.c_double), ("conv_thr_v", C.c_double),
                ("cg_tol", C.c_double), ("niter_max", C.c_int32), ("alpha_mix", C.c_double), ("nmix", C.c_int32),
                ("max_cg_iter", C.c_int32), ("precision", C.c_int32), ("verbosity", C.c_int32),
                ("inner_tol", C.c_double), ("max_refine", C.c_int32), ("graph_chunk", C.c_int32),
                ("autotune", C.c_int32), ("lowp_gemm", C.c_int32), ("find_atpert", C.c_int32),
                ("docc_thr", C.c_double), ("dist_thr", C.c_double), ("skip_equivalence_q", C.c_int32),
                ("lowp_trust_tol", C.c_double)]


class HpScfStats(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("scf_iters", C.c_int32), ("converged", C.c_int32),
                ("cg_iters", C.c_int32), ("h_applies_fp64", C.c_int64), ("h_applies_lowp", C.c_int64),
                ("wall_s", C.c_double), ("chi_change", C.c_double), ("v_residual", C.c_double),
                ("max_rel_resid", C.c_double), ("stage_s", C.c_double * 8)]

    def as_dict(self):
        return {f: (list(getattr(self, f)) if f == "stage_s" else getattr(self, f)) for f, _ in self._fields_
                if f != "struct_size"}


_lib.hp_ground_state_load.argtypes = [C.POINTER(HpGroundState), C.POINTER(C.c_void_p)]
_lib.hp_ground_state_load.restype = C.c_int32
_lib.hp_sternheimer_scf.argtypes = [C.c_void_p, C.c_int32, _dp, C.POINTER(HpScfParams), _dp, _dp,
                                    C.POINTER(HpScfStats)]
_lib.hp_sternheimer_scf.restype = C.c_int32
_lib.hp_response_matrix.argtypes = [C.c_void_p, _ip, C.POINTER(HpScfParams), _dp, _dp, _dp, C.POINTER(HpScfStats)]
_lib.hp_response_matrix.restype = C.c_int32
_lib.hp_hubbard_params.argtypes = [C.c_int32, _dp, _dp, _dp]
_lib.hp_hubbard_params.restype = C.c_int32
_lib.hp_destroy.argtypes = [C.c_void_p]
_lib.hp_destroy.restype = None
_lib.hp_last_error.argtypes = []
_lib.hp_last_error.restype = C.c_char_p
_lib.hp_apply_h.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp]
_lib.hp_apply_h.restype = C.c_int32
_lib.hp_solve_first_order.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_int32, _dp, C.POINTER(HpScfParams), _dp]
_lib.hp_solve_first_order.restype = C.c_int32
_lib.hp_xc_kernel.argtypes = [C.c_int32, C.c_int64, _dp, _dp]
_lib.hp_xc_kernel.restype = C.c_int32
_lib.hp_apply_h_lowp.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _dp, _dp]
_lib.hp_apply_h_lowp.restype = C.c_int32
_lib.hp_apply_h_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp]
_lib.hp_apply_h_noalloc.restype = C.c_int32



class HpKernelTime(C.Structure):
    _fields_ = [("name", C.c_char_p), ("calls", C.c_int64), ("total_ms", C.c_double)]


_lib.hp_profile_start.argtypes = [C.c_void_p]
_lib.hp_profile_start.restype = C.c_int32
_lib.hp_profile_stop.argtypes = [C.c_void_p, C.POINTER(HpKernelTime), C.c_int32, C.POINTER(C.c_int32)]
_lib.hp_profile_stop.restype = C.c_int32
_lib.hp_neighbours.argtypes = [_dp, C.c_int32, _dp, _ip, C.c_double, C.c_int32, _ip, _ip, _dp, _ip]
_lib.hp_neighbours.restype = C.c_int32
_lib.hp_tuning_report.argtypes = [C.c_void_p, C.c_char_p, C.c_int32]
_lib.hp_site_occupations.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _ip]
_lib.hp_site_occupations.restype = C.c_int32
_lib.hp_tuning_report.restype = C.c_int32
_lib.hp_set_gemm_shape.argtypes = [C.c_void_p] + [C.c_int32] * 6
_lib.hp_set_gemm_shape.restype = C.c_int32
_lib.hp_set_plane_variant.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
_lib.hp_set_plane_variant.restype = C.c_int32
_lib.hp_set_stick_variant.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
_lib.hp_set_stick_variant.restype = C.c_int32

EXPORTED = ["hp_ground_state_load", "hp_sternheimer_scf", "hp_response_matrix", "hp_hubbard_params",
            "hp_destroy", "hp_last_error", "hp_apply_h", "hp_solve_first_order", "hp_profile_start",
            "hp_profile_stop", "hp_tuning_report", "hp_set_gemm_shape", "hp_set_plane_variant",
            "hp_neighbours", "hp_set_stick_variant", "hp_site_occupations", "hp_xc_kernel",
            "hp_apply_h_lowp", "hp_apply_h_noalloc"]


def hp_last_error() -> str:
    return _lib.hp_last_error().decode()


def _check(status: int, allow_warn: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_warn):
        raise HpError(status, hp_last_error())
    return status


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128_as_f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128).view(np.float64)


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _is_device(a) -> bool:
    """A torch tensor in GPU memory (the bulk inputs of hp_ground_state_load may be)."""
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


def _dev_ptr(t, dtype_name: str, count: int):
    """Device address of a contiguous torch tensor of `count` elements of torch.<dtype_name>."""
    import torch
    if t.dtype != getattr(torch, dtype_name) or not t.is_contiguous() or t.numel() != count:
        raise ValueError(f"device array must be a contiguous {dtype_name} tensor of {count} elements, got "
                         f"{t.dtype} {tuple(t.shape)}")
    return C.cast(C.c_void_p(t.data_ptr()), _dp)


@dataclass
class ScfParams:
    """Mirror of hp_scf_params (the paper's conv_thr_chi, niter_max, alpha_mix, nmix)."""
    conv_thr_chi: float = 1e-5 * 27.211386245988  # the paper's default 1e-5 eV^-1, in Ha^-1
    conv_thr_v: float = 1e-8
    cg_tol: float = 1e-10
    niter_max: int = 100
    alpha_mix: float = 0.3
    nmix: int = 4
    max_cg_iter: int = 1000
    precision: int = HP_FP64
    verbosity: int = 0
    inner_tol: float = 1e-4
    max_refine: int = 12
    graph_chunk: int = 8   # CG iterations per captured hipGraph launch; 0 launches kernels one by one
    autotune: int = 1      # time candidate GEMM tiles / FFT plane batches on first use of a shape
    lowp_gemm: int = 0     # HP_MIXED: HP_GEMM_FP32, HP_GEMM_BF16 or HP_GEMM_BF16_PV32
    find_atpert: int = 4   # hp_response_matrix: 4 perturbs every site, 1 one per occupation class
    docc_thr: float = 5e-5
    dist_thr: float = 6e-4
    skip_equivalence_q: int = 0   # 0: chi(-q) = conj chi(q) for the -q partners of the mesh
    lowp_trust_tol: float = 1e-6  # mixed, FP32 GEMMs: solves this loose or looser skip FP64 refinement

    def c(self) -> HpScfParams:
        return HpScfParams(C.sizeof(HpScfParams), self.conv_thr_chi, self.conv_thr_v, self.cg_tol, self.niter_max,
                           self.alpha_mix, self.nmix, self.max_cg_iter, self.precision, self.verbosity,
                           self.inner_tol, self.max_refine, self.graph_chunk, self.autotune,
                           self.lowp_gemm, self.find_atpert, self.docc_thr, self.dist_thr,
                           self.skip_equivalence_q, self.lowp_trust_tol)


class Context:
    """Owns an hp_ctx; hp_destroy runs on close() or garbage collection."""

    def __init__(self, handle: int, gs):
        self.handle = C.c_void_p(handle)
        self.n_occ = int(gs.n_occ)
        self.n_hub = int(gs.n_hub)
        self.npw = [int(e.miller.shape[0]) for e in gs.kpts]
        self.fft = tuple(int(x) for x in gs.fft)
        self.nspin = int(getattr(gs, "nspin", 1))

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.hp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hp_ground_state_load(gs, stream: Optional[int] = None, atwfc: Optional[Sequence[np.ndarray]] = None,
                         hub_rows: Optional[np.ndarray] = None) -> Context:
    """gs: an object with cell, fft, vloc, rho0, n_occ, d_kb, hub_tau, n_hub, n_mesh, kpts
    (each k-entry with k_frac, weight, miller, eps, u, beta, phi), optionally nspin = 2
    (kpts: a spin-up then a spin-down block; vloc, rho0: (2, N1, N2, N3)).  With atwfc (one
    (n_atwfc, npw) complex array per k-entry: every atomic orbital) and hub_rows (the row of
    d orbital m of Hubbard site s at 5 s + m) the library builds ortho-atomic projectors and
    the entries' phi are not read.

    The bulk arrays (vloc, rho0 and every entry's u, beta, phi, atwfc) may all be torch
    tensors in GPU memory (contiguous float64 / complex128): they are then passed as device
    pointers (inputs_on_device = 1) and copied device to device on `stream` (torch's
    current stream when None).  Mixing host and device bulk arrays is an error."""
    ortho = atwfc is not None
    if ortho and (hub_rows is None or len(atwfc) != len(gs.kpts)):
        raise ValueError("ortho-atomic projectors need one atwfc table per k-entry and hub_rows")
    bulk = [gs.vloc, gs.rho0] + [a for e in gs.kpts for a in (e.u, e.beta)]
    bulk += list(atwfc) if ortho else [e.phi for e in gs.kpts]
    flags = {_is_device(a) for a in bulk}
    if len(flags) != 1:
        raise ValueError("the bulk arrays must be all host arrays or all GPU tensors")
    on_dev = flags.pop()
    if on_dev and stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream

    def table(a, rows, npw, what):
        """Pointer to a [>= rows][npw] complex table (host array or GPU tensor); the library
        reads the first `rows` rows."""
        if len(a.shape) != 2 or int(a.shape[1]) != npw or int(a.shape[0]) < rows:
            raise ValueError(f"{what} has shape {tuple(a.shape)}, want ({rows}, {npw})")
        if on_dev:
            return a, _dev_ptr(a, "complex128", int(a.shape[0]) * npw)
        h = _c128_as_f64(a)
        return h, _ptr(h)

    keep = []
    kp = (HpKpoint * len(gs.kpts))()
    n_atwfc = 0
    n_occ, n_beta, nh5 = int(gs.n_occ), int(np.asarray(gs.d_kb).shape[0]), 5 * int(gs.n_hub)
    for i, e in enumerate(gs.kpts):
        mil = np.ascontiguousarray(e.miller, dtype=np.int32)
        npw = int(mil.shape[0])
        eps = _f64(e.eps)
        u, up = table(e.u, n_occ, npw, f"kpts[{i}].u")
        beta, bp = table(e.beta, n_beta, npw, f"kpts[{i}].beta")
        phi, pp = (None, None) if ortho else table(e.phi, nh5, npw, f"kpts[{i}].phi")
        at, ap = None, None
        if ortho:
            a = atwfc[i]
            n_a = int(a.shape[0])
            if len(a.shape) != 2 or int(a.shape[1]) != npw or (i and n_a != n_atwfc):
                raise ValueError(f"atwfc[{i}] has shape {tuple(a.shape)}, entry {i} has {npw} plane waves")
            n_atwfc = n_a
            at, ap = table(a, n_a, npw, f"atwfc[{i}]")
        keep += [mil, eps, u, beta, phi, at]
        kp[i] = HpKpoint(C.sizeof(HpKpoint), (C.c_double * 3)(*[float(x) for x in e.k_frac]), float(e.weight),
                         npw, _ptr(mil, _ip), _ptr(eps), up, bp, pp, ap)
    nspin = int(getattr(gs, "nspin", 1))
    nr = int(np.prod([int(x) for x in gs.fft])) * nspin
    if on_dev:
        vloc, rho0 = gs.vloc, gs.rho0
        vloc_p, rho0_p = _dev_ptr(vloc, "float64", nr), _dev_ptr(rho0, "float64", nr)
    else:
        vloc = _f64(gs.vloc)
        rho0 = _f64(gs.rho0)
        if vloc.size != nr or rho0.size != nr:
            raise ValueError(f"v_loc/rho0 hold {vloc.size}/{rho0.size} values, {nspin} spin(s) of the grid "
                             f"{tuple(gs.fft)} hold {nr}")
        vloc_p, rho0_p = _ptr(vloc), _ptr(rho0)
    dkb = _f64(gs.d_kb)
    htau = _f64(gs.hub_tau)
    hrows = np.ascontiguousarray(hub_rows, dtype=np.int32) if ortho else None
    hpot = getattr(gs, "hub_pot", None)
    if hpot is not None:
        hpot = np.ascontiguousarray(hpot, dtype=np.complex128)
        if hpot.shape != (nspin, int(gs.n_hub), 5, 5):
            raise ValueError(f"hub_pot has shape {hpot.shape}, want {(nspin, int(gs.n_hub), 5, 5)}")
        hpot = hpot.view(np.float64)
    keep += [vloc, rho0, dkb, htau, hrows, hpot]
    cell = ((C.c_double * 3) * 3)(*[(C.c_double * 3)(*[float(x) for x in row]) for row in np.asarray(gs.cell)])
    g = HpGroundState()
    g.struct_size = C.sizeof(HpGroundState)
    g.cell = cell
    g.fft = (C.c_int32 * 3)(*[int(x) for x in gs.fft])
    g.v_loc = vloc_p
    g.rho0 = rho0_p
    g.n_occ = int(gs.n_occ)
    g.n_beta = int(dkb.shape[0])
    g.n_hub = int(gs.n_hub)
    g.d_kb = _ptr(dkb)
    g.hub_tau = _ptr(htau)
    g.spin_factor = int(getattr(gs, "spin_factor", 2))
    g.n_mesh = int(gs.n_mesh)
    g.n_kpts = len(gs.kpts)
    g.kpts = kp
    g.xc = HP_XC_LDA_PZ81
    g.inputs_on_device = 1 if on_dev else 0
    g.stream = C.c_void_p(stream) if stream else None
    g.projectors = HP_PROJ_ORTHO_ATOMIC if ortho else HP_PROJ_ATOMIC
    g.n_atwfc = n_atwfc
    g.hub_rows = _ptr(hrows, _ip) if ortho else None
    g.nspin = nspin
    g.hub_pot = _ptr(hpot) if hpot is not None else None
    g.degauss = float(getattr(gs, "degauss", 0.0) or 0.0)
    g.efermi = float(getattr(gs, "efermi", 0.0) or 0.0)
    h = C.c_void_p()
    _check(_lib.hp_ground_state_load(C.byref(g), C.byref(h)), allow_warn=False)
    del keep
    return Context(h.value, gs)


def hp_site_occupations(ctx: Context, docc_thr: float = 5e-5):
    """(trace, moment, class) per Hubbard site: sum over spins of Tr n^I (Eq. 3), the moment
    Tr n^I_up - Tr n^I_dn, and the representative site of I's class of equal traces."""
    tr = np.zeros(ctx.n_hub)
    mo = np.zeros(ctx.n_hub)
    cl = np.zeros(ctx.n_hub, dtype=np.int32)
    _check(_lib.hp_site_occupations(ctx.handle, float(docc_thr), _ptr(tr), _ptr(mo), _ptr(cl, _ip)), allow_warn=False)
    return tr, mo, cl


def hp_sternheimer_scf(ctx: Context, pert_site: int, q_frac: Sequence[float], params: ScfParams):
    """Returns (dn0, dn, stats, status); dn0/dn are complex (n_hub, 5, 5)."""
    q = _f64(q_frac)
    dn0 = np.zeros(ctx.n_hub * 50)
    dn = np.zeros(ctx.n_hub * 50)
    st = HpScfStats()
    st.struct_size = C.sizeof(HpScfStats)
    p = params.c()
    s = _check(_lib.hp_sternheimer_scf(ctx.handle, int(pert_site), _ptr(q), C.byref(p), _ptr(dn0), _ptr(dn),
                                       C.byref(st)))
    return (dn0.view(np.complex128).reshape(ctx.n_hub, 5, 5), dn.view(np.complex128).reshape(ctx.n_hub, 5, 5),
            st.as_dict(), s)


def hp_response_matrix(ctx: Context, nq: Sequence[int], params: ScfParams):
    """Returns (chi0, chi, max_imag, stats, status), chi0/chi real (n, n) with n = n_hub * prod(nq)."""
    nqa = np.ascontiguousarray(nq, dtype=np.int32)
    n = ctx.n_hub * int(np.prod(nqa))
    chi0 = np.zeros((n, n))
    chi = np.zeros((n, n))
    mim = np.zeros(1)
    st = HpScfStats()
    st.struct_size = C.sizeof(HpScfStats)
    p = params.c()
    s = _check(_lib.hp_response_matrix(ctx.handle, _ptr(nqa, _ip), C.byref(p), _ptr(chi0), _ptr(chi), _ptr(mim),
                                       C.byref(st)))
    return chi0, chi, float(mim[0]), st.as_dict(), s


def hp_hubbard_params(chi0: np.ndarray, chi: np.ndarray) -> np.ndarray:
    a = _f64(chi0)
    b = _f64(chi)
    n = a.shape[0]
    if a.shape != (n, n) or b.shape != (n, n):
        raise ValueError("chi0 and chi must be square and of the same size")
    out = np.zeros((n, n))
    _check(_lib.hp_hubbard_params(n, _ptr(a), _ptr(b), _ptr(out)), allow_warn=False)
    return out


def hp_destroy(ctx: Context) -> None:
    ctx.close()


def hp_apply_h(ctx: Context, entry: int, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    y = np.zeros_like(x)
    _check(_lib.hp_apply_h(ctx.handle, int(entry), x.shape[0], _ptr(x.view(np.float64)), _ptr(y.view(np.float64))),
           allow_warn=False)
    return y


def hp_solve_first_order(ctx: Context, pert_site: int, q_frac, mesh_k: int, dv: Optional[np.ndarray],
                         params: ScfParams, npw_kq: int):
    q = _f64(q_frac)
    out = np.zeros((ctx.n_occ, npw_kq), dtype=np.complex128)
    p = params.c()
    dvp = None
    if dv is not None:
        dva = np.ascontiguousarray(dv, dtype=np.complex128)
        want = ctx.fft if ctx.nspin == 1 else (ctx.nspin,) + ctx.fft
        if dva.shape != want:
            raise ValueError(f"dv must have the shape {want}")
        dvp = _ptr(dva.view(np.float64))
    s = _check(_lib.hp_solve_first_order(ctx.handle, int(pert_site), _ptr(q), int(mesh_k), dvp, C.byref(p),
                                         _ptr(out.view(np.float64))))
    return out, s


def hp_apply_h_lowp(ctx: Context, entry: int, x: np.ndarray, lowp_gemm: int = HP_GEMM_FP32) -> np.ndarray:
    """H_k x with the mixed form's reduced-precision operator (FP32 FFTs, FP32 or BF16
    projections), returned in FP64."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    y = np.zeros_like(x)
    _check(_lib.hp_apply_h_lowp(ctx.handle, int(entry), x.shape[0], int(lowp_gemm), _ptr(x.view(np.float64)),
                                _ptr(y.view(np.float64))), allow_warn=False)
    return y


def hp_apply_h_noalloc(ctx: Context, entry: int, x, y) -> None:
    """y = H_k x on device arrays with no allocation: x, y contiguous complex128 GPU tensors
    of shape (n, npw) (entry's plane-wave order).  Enqueued on the context's stream; returns
    without waiting (synchronize before reading y)."""
    if not (_is_device(x) and _is_device(y)):
        raise ValueError("x and y must be GPU tensors")
    n = int(x.shape[0])
    npw = ctx.npw[entry] if 0 <= entry < len(ctx.npw) else 0
    if tuple(x.shape) != (n, npw) or tuple(y.shape) != (n, npw):
        raise ValueError(f"x and y must have the shape (n, {npw})")
    xp = _dev_ptr(x, "complex128", n * npw)
    yp = _dev_ptr(y, "complex128", n * npw)
    _check(_lib.hp_apply_h_noalloc(ctx.handle, int(entry), n, xp, yp), allow_warn=False)


def hp_xc_kernel(rho: np.ndarray) -> np.ndarray:
    """The library's LDA kernel at the densities rho: shape (n,) -> (n,) unpolarized, or
    (2, n) (up, down) -> (3, n) (f_uu, f_ud, f_dd)."""
    r = _f64(rho)
    nspin = 2 if r.ndim == 2 else 1
    if r.ndim not in (1, 2) or (nspin == 2 and r.shape[0] != 2):
        raise ValueError("rho must have the shape (n,) or (2, n)")
    n = r.shape[-1]
    out = np.zeros((3, n) if nspin == 2 else (n,))
    _check(_lib.hp_xc_kernel(nspin, n, _ptr(r), _ptr(out)), allow_warn=False)
    return out


def hp_profile_start(ctx: Context) -> None:
    _check(_lib.hp_profile_start(ctx.handle), allow_warn=False)


def hp_profile_stop(ctx: Context) -> dict:
    """{kernel name: (launches, summed GPU ms)} since hp_profile_start."""
    out = (HpKernelTime * 32)()
    n = C.c_int32(0)
    _check(_lib.hp_profile_stop(ctx.handle, out, 32, C.byref(n)), allow_warn=False)
    return {out[i].name.decode(): (int(out[i].calls), float(out[i].total_ms)) for i in range(n.value)}


def hp_tuning_report(ctx: Context) -> dict:
    """Launch shapes the autotuner chose in this context, with measured and default times."""
    import json
    buf = C.create_string_buffer(1 << 16)
    _check(_lib.hp_tuning_report(ctx.handle, buf, len(buf)), allow_warn=False)
    return json.loads(buf.value.decode())


def hp_set_gemm_shape(ctx: Context, prec: int, rows: int, batch: int, tile: int, nsplit: int, expand_bands: int):
    _check(_lib.hp_set_gemm_shape(ctx.handle, prec, rows, batch, tile, nsplit, expand_bands), allow_warn=False)


def hp_set_plane_variant(ctx: Context, prec: int, variant: int):
    _check(_lib.hp_set_plane_variant(ctx.handle, prec, variant), allow_warn=False)


def hp_neighbours(cell, hub_tau, nq, dist_thr: float = 6e-4):
    """Nearest-neighbour (I, J, distance) triples of the q-supercell (see hp.h); V_IJ = uv[I, J]."""
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    tau = np.ascontiguousarray(hub_tau, dtype=np.float64)
    nqa = np.ascontiguousarray(nq, dtype=np.int32)
    n_hub = tau.shape[0]
    cap = 64 * n_hub
    pi, pj = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    d = np.zeros(cap)
    n = C.c_int32(0)
    _check(_lib.hp_neighbours(_ptr(cell), n_hub, _ptr(tau), _ptr(nqa, _ip), float(dist_thr), cap, _ptr(pi, _ip),
                              _ptr(pj, _ip), _ptr(d), C.byref(n)), allow_warn=False)
    k = n.value
    return [(int(pi[i]), int(pj[i]), float(d[i])) for i in range(k)]


def hp_set_stick_variant(ctx: Context, prec: int, inverse_variant: int, forward_variant: int):
    _check(_lib.hp_set_stick_variant(ctx.handle, prec, inverse_variant, forward_variant), allow_warn=False)
