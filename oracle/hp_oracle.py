"""Plain FP64 CPU oracle of the q-resolved DFPT Hubbard response.
TEST INFRASTRUCTURE ONLY (see the package header).

Conventions (the paper defers these to its Ref. Timrov 2018; the readings
are listed in the design notes of the repository):

* lattice-periodic functions: u(r) = Omega^{-1/2} sum_G c(G) e^{iG.r};
  on grid point r_j the dimensionless field psi(r_j) = sum_G c(G) e^{iG.r_j}
  is N_r * ifftn of the coefficients scattered to (m mod N);
* the local potential acts on the grid: (V c)(G) = fftn(V psi)/N_r at G, which
  equals the matrix V_hat[(m - m') mod N] with V_hat = fftn(V)/N_r;
* spin-unpolarized closed shell: occupations and densities carry a factor 2;
* collinear spin-polarized ground states (nspin = 2; the paper's formalism is
  written for spin-resolved states, Eqs. 3, 10-15): the k-entries come in two
  blocks (spin up, then spin down, the same k list in each), every state holds one
  electron, V_loc and rho0 carry a leading spin index, the response density is
  spin-resolved and the Hxc response uses the 2 x 2 LSDA kernel; the perturbation of
  Eq. 16 acts on both spins and the occupation response is summed over spins;
* metallic ground states (the paper's generalization to fractional occupations): cold
  (Marzari-Vanderbilt) smearing of width sigma, occupations f_i = occ((e_F - e_i)/sigma);
  splitting the sum over pairs of states with a smooth step theta (theta_ij + theta_ji = 1)
  keeps Eq. 15 with the right-hand side -(f_i - sum_j beta_ij |u_j><u_j|) dV u_i and
  beta_ij = f_i theta_ij + f_j theta_ji + alpha theta_ji (f_i - f_j)/(e_i - e_j); at q = 0
  the Fermi level shifts to keep the electron count (an extra density and occupation
  term).  Unpolarized only;
* time reversal folds the -q partner into the +q term (paper, text after
  Eq. 14), giving the factor 4 = 2 (spin) x 2 (time reversal) in the response
  density (2 per spin channel when polarized) and the two-term form of Eq. 13.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import scipy.fft as sfft

from . import pz81

FOUR_PI = 4.0 * math.pi


def _workers() -> int:
    """Host threads for the oracle's FFTs: HP_ORACLE_WORKERS, else the CPUs this process may use."""
    import os
    v = os.environ.get("HP_ORACLE_WORKERS")
    if v:
        return max(1, int(v))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


@dataclass
class ScfParams:
    """Controls of the self-consistent Sternheimer loop (the paper's inputhp
    convergence keywords: conv_thr_chi, niter_max, alpha_mix, nmix)."""
    cg_tol: float = 1e-12            # per band ||r|| / ||b||
    conv_thr_chi: float = 1e-12      # max |chi(q)_it - chi(q)_it-1| (Ha^-1)
    conv_thr_v: float = 1e-10        # ||dV_out - dV_in|| / ||dV_out||
    niter_max: int = 100
    alpha_mix: float = 0.3
    nmix: int = 4
    max_cg_iter: int = 2000
    method: str = "cg"               # "cg" or "direct" (dense solve per band)
    hxc: bool = True                 # False: frozen Hxc (then chi = chi0)
    alpha_shift: Optional[float] = None   # override of the Eq. 15 shift


def _fftfreq_int(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.where(j < (n + 1) // 2, j, j - n)


class Oracle:
    """One ground state (synth.GroundState-like object) and the linear-response
    machinery of Eqs. 12-18 on top of it."""

    def __init__(self, gs, cache_limit_bytes: float = 2e9, projectors: str = "atomic"):
        """projectors: "atomic" (the d orbitals as given) or "ortho-atomic" (Loewdin-orthogonalized
        over every atomic orbital of the system, Eq. 6)."""
        self.gs = gs
        if projectors == "atomic":
            self.phi = [e.phi for e in gs.kpts]
        elif projectors == "ortho-atomic":
            self.phi = [ortho_atomic_phi(gs, e) for e in gs.kpts]
        else:
            raise ValueError(projectors)
        self.fft = tuple(int(x) for x in gs.fft)
        self.nr = int(np.prod(self.fft))
        self.cell = np.asarray(gs.cell, dtype=np.float64)
        self.omega = float(abs(np.linalg.det(self.cell)))
        self.bvec = 2.0 * math.pi * np.linalg.inv(self.cell).T
        self.n_occ = int(gs.n_occ)
        self.n_hub = int(gs.n_hub)
        self.kpts = gs.kpts
        self.n_mesh = int(gs.n_mesh)
        self.nspin = int(getattr(gs, "nspin", 1))
        if self.nspin not in (1, 2) or len(self.kpts) % self.nspin:
            raise ValueError("nspin must be 1 or 2, with one block of k-entries per spin")
        self.nk_spin = len(self.kpts) // self.nspin          # entries per spin block
        self.occ = 2.0 / self.nspin                            # electrons per state
        # mesh entries of every spin (entry index = spin * nk_spin + mesh index)
        self.mesh = [s * self.nk_spin + i for s in range(self.nspin) for i in range(self.n_mesh)]
        if self.nspin == 1:
            self.vloc = np.asarray(gs.vloc, dtype=np.float64)
            self.fxc = pz81.f_xc(gs.rho0)
        else:
            self.vloc = np.asarray(gs.vloc, dtype=np.float64).reshape((2,) + self.fft)
            rho = np.asarray(gs.rho0, dtype=np.float64).reshape((2,) + self.fft)
            self.fxc = pz81.f_xc_spin(rho[0], rho[1])          # (2, 2) + grid
        # ground-state Hubbard potential (Eq. 5, on-site part): per spin and site the 5 x 5
        # matrix M with V_Hub = sum_I sum_{m1 m2} M^I_{m1 m2} |phi^I_{m1}><phi^I_{m2}|, or None
        hpot = getattr(gs, "hub_pot", None)
        self.hub_pot = (None if hpot is None else
                        np.asarray(hpot, dtype=np.complex128).reshape(self.nspin, self.n_hub, 5, 5))
        # metallic occupations (cold smearing) of the kept bands
        self.degauss = float(getattr(gs, "degauss", 0.0) or 0.0)
        self.metal = self.degauss > 0.0
        if self.metal:
            if self.nspin != 1:
                raise NotImplementedError("metallic ground states are unpolarized here")
            self.efermi = float(gs.efermi)
            self.f = [cold_occupation((self.efermi - e.eps) / self.degauss) for e in self.kpts]
            self.dlt = [cold_delta((self.efermi - e.eps) / self.degauss) for e in self.kpts]
        # alpha = 2 (max - min) over the occupied energies of every loaded entry
        # (paper, text after Eq. 18); floor 0.01 Ha.
        emax = max(float(e.eps.max()) for e in self.kpts)
        emin = min(float(e.eps.min()) for e in self.kpts)
        self.alpha = max(2.0 * (emax - emin), 0.01)
        self._psi_cache: Dict[int, np.ndarray] = {}
        self._cache_bytes = 0.0
        self._cache_limit = cache_limit_bytes
        self._dense: Dict[int, np.ndarray] = {}
        self._kin: Dict[int, np.ndarray] = {}

    def spin_of(self, ie: int) -> int:
        return ie // self.nk_spin

    def v_of(self, ie: int) -> np.ndarray:
        """Local potential seen by entry ie (its spin's)."""
        return self.vloc if self.nspin == 1 else self.vloc[self.spin_of(ie)]

    # ------------------------------------------------------------------ grids
    def grid_index(self, ie: int, g0=(0, 0, 0)) -> np.ndarray:
        """Linear grid index of each plane wave of entry ie, Miller indices shifted by -g0."""
        m = (self.kpts[ie].miller - np.asarray(g0, dtype=np.int64)[None, :]) % np.array(self.fft)
        return np.ravel_multi_index(tuple(m.T), self.fft)

    def to_real(self, c: np.ndarray, idx: np.ndarray) -> np.ndarray:
        """psi(r_j) = sum_G c(G) e^{iG.r_j} for each row of c; returns (nb, N1, N2, N3)."""
        c = np.atleast_2d(c)
        g = np.zeros((c.shape[0], self.nr), dtype=np.complex128)
        g[:, idx] = c
        return sfft.ifftn(g.reshape((c.shape[0],) + self.fft), axes=(1, 2, 3), workers=_workers()) * self.nr

    def to_recip(self, f: np.ndarray, idx: np.ndarray) -> np.ndarray:
        """c(G) = (1/N_r) sum_j f(r_j) e^{-iG.r_j} at the plane waves idx; f is (nb, N1, N2, N3)."""
        g = sfft.fftn(f, axes=(1, 2, 3), workers=_workers()).reshape(f.shape[0], self.nr) / self.nr
        return g[:, idx]

    def psi_r(self, ie: int) -> np.ndarray:
        if ie in self._psi_cache:
            return self._psi_cache[ie]
        p = self.to_real(self.kpts[ie].u, self.grid_index(ie))
        if self._cache_bytes + p.nbytes <= self._cache_limit:
            self._psi_cache[ie] = p
            self._cache_bytes += p.nbytes
        return p

    def kinetic(self, ie: int) -> np.ndarray:
        if ie not in self._kin:
            e = self.kpts[ie]
            p = (e.miller + e.k_frac[None, :]) @ self.bvec
            self._kin[ie] = 0.5 * np.einsum("ij,ij->i", p, p)
        return self._kin[ie]

    # ----------------------------------------------------- Hamiltonian (Eq. 15)
    def h_apply(self, ie: int, X: np.ndarray) -> np.ndarray:
        """H_k X for rows X on entry ie: kinetic + V_loc on the grid + sum_i D_i |beta_i><beta_i|
        (norm-conserving pseudopotentials; the Hubbard potential is zero in the
        unperturbed state used here)."""
        e = self.kpts[ie]
        idx = self.grid_index(ie)
        out = self.kinetic(ie)[None, :] * X
        out = out + self.to_recip(self.to_real(X, idx) * self.v_of(ie)[None], idx)
        proj = X @ e.beta.conj().T            # <beta_i|x> for every row
        out = out + (proj * self.gs.d_kb[None, :]) @ e.beta
        if self.hub_pot is not None:
            out = out + self.vhub_apply(ie, X)
        return out

    def vhub_apply(self, ie: int, X: np.ndarray) -> np.ndarray:
        """Ground-state Hubbard potential on rows X (Eq. 5, on-site):
        sum_s sum_{m1 m2} M^s_{m1 m2} |phi_{m1}> <phi_{m2}|x>."""
        P = self.phi[ie]
        M = self.hub_pot[self.spin_of(ie)]
        proj = X @ P.conj().T                 # proj[v, m] = <phi_m|x_v>
        out = np.zeros_like(X)
        for s in range(self.n_hub):
            sl = slice(5 * s, 5 * s + 5)
            out += (proj[:, sl] @ M[s].T) @ P[sl]
        return out

    def h_dense(self, ie: int) -> np.ndarray:
        """Dense H_k built element by element from the same definition."""
        if ie in self._dense:
            return self._dense[ie]
        e = self.kpts[ie]
        vhat = np.fft.fftn(self.v_of(ie)) / self.nr
        dm = (e.miller[:, None, :] - e.miller[None, :, :]) % np.array(self.fft)
        H = vhat[dm[..., 0], dm[..., 1], dm[..., 2]].astype(np.complex128)
        H += np.diag(self.kinetic(ie))
        H += (e.beta.T * self.gs.d_kb[None, :]) @ e.beta.conj()
        if self.hub_pot is not None:
            P = self.phi[ie]
            for s in range(self.n_hub):
                sl = slice(5 * s, 5 * s + 5)
                H += P[sl].T @ self.hub_pot[self.spin_of(ie)][s] @ P[sl].conj()
        self._dense[ie] = H
        return H

    # ------------------------------------------------------------ q mapping
    def kq_entry(self, ik: int, q) -> Tuple[int, np.ndarray]:
        """Entry j (of the same spin) holding k+q and the integer shift g0 with k + q = k_j + g0."""
        kq = self.kpts[ik].k_frac + np.asarray(q, dtype=np.float64)
        j0 = self.spin_of(ik) * self.nk_spin
        for j in range(j0, j0 + self.nk_spin):
            e = self.kpts[j]
            d = kq - e.k_frac
            if np.all(np.abs(d - np.round(d)) < 1e-9):
                return j, np.round(d).astype(np.int64)
        raise KeyError(f"no entry for k+q = {kq}")

    # ----------------------------------------------- Sternheimer, Eqs. 15-18
    def rhs(self, ik: int, q, site: int, dv: Optional[np.ndarray]) -> np.ndarray:
        """-P_c,k+q (dV_Hxc u_vk + V_pert u_vk) for every occupied v (Eq. 15 RHS,
        V_pert from Eq. 16, P_c from Eq. 18); for metals -(f_v - sum_j beta_vj |u_j><u_j|)
        applied to the same vectors."""
        j, g0 = self.kq_entry(ik, q)
        ek, ej = self.kpts[ik], self.kpts[j]
        b = np.zeros((self.n_occ, ej.npw), dtype=np.complex128)
        if dv is not None:  # dv: the grid field, (2,) + grid when spin-polarized
            dvs = dv if self.nspin == 1 else dv[self.spin_of(ik)]
            b += self.to_recip(dvs[None] * self.psi_r(ik), self.grid_index(j, g0))
        sl = slice(5 * site, 5 * site + 5)
        A = self.phi[ik][sl].conj() @ ek.u.T    # A[m, v] = <phi_{m,k}|u_vk>
        b += A.T @ self.phi[j][sl]              # sum_m |phi_{m,k+q}> A[m, v]
        if self.metal:                          # -(f_i - sum_j beta_ij |u_j><u_j|) b_i
            C = b @ ej.u.conj().T               # C[i, j] = <u_j,k+q|b_i>
            return -(self.f[ik][:, None] * b - (self.beta_matrix(ik, j) * C) @ ej.u)
        b -= (b @ ej.u.conj().T) @ ej.u         # P_c = 1 - sum_v' |u_v',k+q><u_v',k+q|
        return -b

    def beta_matrix(self, ik: int, j: int) -> np.ndarray:
        """beta_ij = f_i theta_ij + f_j theta_ji + alpha theta_ji (f_i - f_j)/(e_i - e_j) for band
        i at entry ik and band j at entry j; theta_ji = step((e_j - e_i)/sigma); equal energies
        take the derivative of the occupation."""
        ei, ej = self.kpts[ik].eps, self.kpts[j].eps
        fi, fj = self.f[ik], self.f[j]
        sig = self.degauss
        d = ei[:, None] - ej[None, :]
        th_ji = smooth_step(-d / sig)
        close = np.abs(d) < 1e-9
        mid = 0.5 * (ei[:, None] + ej[None, :])
        F = np.where(close, -cold_delta((self.efermi - mid) / sig) / sig,
                     (fi[:, None] - fj[None, :]) / np.where(close, 1.0, d))
        return fi[:, None] * (1.0 - th_ji) + fj[None, :] * th_ji + self.alpha * th_ji * F

    def fermi_shift(self, X: Dict[int, np.ndarray]) -> complex:
        """Shift of the Fermi level at q = 0 that keeps the electron count:
        sum_k w sum_i delta_i <u_i|dV|u_i> / sum_k w sum_i delta_i (X[ik] = dV u rows).
        Kept complex: the response is linear over the complex numbers (the iterates of the
        response potential are complex), and for a physical perturbation the sum over
        time-reversed k points makes it real."""
        num, den = 0.0 + 0.0j, 0.0
        for ik in self.mesh:
            e = self.kpts[ik]
            m = np.einsum("ig,ig->i", e.u.conj(), X[ik])
            num += e.weight * np.dot(self.dlt[ik], m)
            den += e.weight * self.dlt[ik].sum()
        return num / den if den != 0.0 else 0.0

    def perturbed_vectors(self, ik: int, q, site: int, dv: Optional[np.ndarray]) -> np.ndarray:
        """dV_Hxc u_vk + V_pert u_vk in the k+q basis (the right-hand side before projection)."""
        j, g0 = self.kq_entry(ik, q)
        ek, ej = self.kpts[ik], self.kpts[j]
        b = np.zeros((self.n_occ, ej.npw), dtype=np.complex128)
        if dv is not None:
            dvs = dv if self.nspin == 1 else dv[self.spin_of(ik)]
            b += self.to_recip(dvs[None] * self.psi_r(ik), self.grid_index(j, g0))
        sl = slice(5 * site, 5 * site + 5)
        A = self.phi[ik][sl].conj() @ ek.u.T
        b += A.T @ self.phi[j][sl]
        return b

    def sternheimer_op(self, ik: int, q, X: np.ndarray, alpha: Optional[float] = None) -> np.ndarray:
        """(H_k+q + alpha O_k+q - eps_vk) X, row v paired with eps_vk (Eq. 15 LHS, O from Eq. 17)."""
        j, _ = self.kq_entry(ik, q)
        ej = self.kpts[j]
        a = self.alpha if alpha is None else alpha
        out = self.h_apply(j, X)
        out += a * (X @ ej.u.conj().T) @ ej.u
        out -= self.kpts[ik].eps[:, None] * X
        return out

    def solve(self, ik: int, q, b: np.ndarray, x0: Optional[np.ndarray], p: ScfParams):
        """Solve Eq. 15 for every occupied band of mesh point ik.  Returns (x, iterations)."""
        a = self.alpha if p.alpha_shift is None else p.alpha_shift
        if p.method == "direct":
            j, _ = self.kq_entry(ik, q)
            ej = self.kpts[j]
            M0 = self.h_dense(j) + a * ej.u.T @ ej.u.conj()
            x = np.empty_like(b)
            for v in range(self.n_occ):
                M = M0 - self.kpts[ik].eps[v] * np.eye(M0.shape[0])
                x[v] = np.linalg.solve(M, b[v])
            return x, 0
        # preconditioned conjugate gradients, one independent recursion per band (rows),
        # Jacobi preconditioner: the exact diagonal of the (positive definite) operator
        j, _ = self.kq_entry(ik, q)
        ej = self.kpts[j]
        vhat0 = float(np.mean(self.v_of(j)))
        diag = (self.kinetic(j) + vhat0 + (np.abs(ej.beta) ** 2 * self.gs.d_kb[:, None]).sum(0)
                + a * (np.abs(ej.u) ** 2).sum(0))
        if self.hub_pot is not None:
            P = self.phi[j]
            for s in range(self.n_hub):
                sl = slice(5 * s, 5 * s + 5)
                diag = diag + np.einsum("mg,mn,ng->g", P[sl], self.hub_pot[self.spin_of(j)][s],
                                        P[sl].conj()).real
        dinv = 1.0 / (diag[None, :] - self.kpts[ik].eps[:, None])
        x = np.zeros_like(b) if x0 is None else x0.copy()
        r = b - self.sternheimer_op(ik, q, x, a)
        bn = np.linalg.norm(b, axis=1)
        bn = np.where(bn > 0, bn, 1.0)
        z = dinv * r
        pdir = z.copy()
        rz = np.einsum("ij,ij->i", r.conj(), z).real
        active = np.linalg.norm(r, axis=1) / bn > p.cg_tol
        it = 0
        while active.any() and it < p.max_cg_iter:
            it += 1
            Ap = self.sternheimer_op(ik, q, pdir, a)
            pAp = np.einsum("ij,ij->i", pdir.conj(), Ap).real
            step = np.where(active, rz / np.where(pAp != 0, pAp, 1.0), 0.0)
            x += step[:, None] * pdir
            r -= step[:, None] * Ap
            z = dinv * r
            rz_new = np.einsum("ij,ij->i", r.conj(), z).real
            beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
            pdir = np.where(active[:, None], z + beta[:, None] * pdir, pdir)
            rz = np.where(active, rz_new, rz)
            active = active & (np.linalg.norm(r, axis=1) / bn > p.cg_tol)
        if active.any():
            raise RuntimeError(f"CG did not converge at k-entry {ik} after {it} iterations")
        return x, it

    # ------------------------------------------------ response density and Hxc
    def drho_k(self, ik: int, q, du: np.ndarray) -> np.ndarray:
        """Contribution of mesh entry ik to the response density at q (of ik's spin):
        (2 occ w_k / Omega) sum_v conj(psi_vk(r)) dpsi_vk+q(r), occ electrons per state
        times 2 for time reversal."""
        j, g0 = self.kq_entry(ik, q)
        dpsi = self.to_real(du, self.grid_index(j, g0))
        w = self.kpts[ik].weight
        return (2.0 * self.occ * w / self.omega) * np.einsum("vxyz,vxyz->xyz", self.psi_r(ik).conj(), dpsi)

    def gvec_q(self, q) -> np.ndarray:
        """|q+G|^2 over the FFT grid (G from the centred integer frequencies)."""
        m = [_fftfreq_int(n) for n in self.fft]
        M = np.stack(np.meshgrid(*m, indexing="ij"), -1).astype(np.float64)
        p = (M + np.asarray(q, dtype=np.float64)) @ self.bvec
        return np.einsum("...i,...i->...", p, p)

    def dv_hxc(self, drho: np.ndarray, q, hxc: bool = True) -> np.ndarray:
        """Response Hxc potential: Hartree 4 pi drho(G)/|q+G|^2 (zero at q+G = 0) of the
        total response density plus the local LDA kernel, f_xc(r) drho(r), or per spin
        sum_t f_xc^{st}(r) drho_t(r) when spin-polarized (drho then (2,) + grid)."""
        if not hxc:
            return np.zeros_like(drho)
        g2 = self.gvec_q(q)
        tot = drho if self.nspin == 1 else drho.sum(axis=0)
        dg = np.fft.fftn(tot) / self.nr
        vh = np.where(g2 > 1e-12, FOUR_PI * dg / np.where(g2 > 1e-12, g2, 1.0), 0.0)
        vh = np.fft.ifftn(vh) * self.nr
        if self.nspin == 1:
            return vh + self.fxc * drho
        return np.stack([vh + self.fxc[s, 0] * drho[0] + self.fxc[s, 1] * drho[1] for s in range(2)])

    # ----------------------------------------------------- occupations, Eq. 13
    def dn_k(self, ik: int, q, du: np.ndarray) -> np.ndarray:
        """Contribution of mesh entry ik to Delta_q n^s_{m1 m2} for every site s (summed over
        spins by the caller): occ w_k sum_v [<u|phi_{m2,k}><phi_{m1,k+q}|du>
        + <u|phi_{m1,k}><phi_{m2,k+q}|du>]."""
        j, _ = self.kq_entry(ik, q)
        ek, ej = self.kpts[ik], self.kpts[j]
        A = self.phi[ik].conj() @ ek.u.T         # (n_hub*5, n_occ)
        B = self.phi[j].conj() @ du.T            # (n_hub*5, n_occ)
        out = np.zeros((self.n_hub, 5, 5), dtype=np.complex128)
        for s in range(self.n_hub):
            sl = slice(5 * s, 5 * s + 5)
            T = B[sl] @ A[sl].conj().T           # T[m1, m2] = sum_v B[m1,v] conj(A[m2,v])
            out[s] = self.occ * ek.weight * (T + T.T)
        return out

    def occupations(self) -> np.ndarray:
        """Ground-state n^s_{m1 m2} = (occ/N_k) sum_kv f_v <u|phi_{m2}><phi_{m1}|u> (Eq. 3, on-site,
        summed over spins; f_v = 1 for insulators)."""
        out = np.zeros((self.n_hub, 5, 5), dtype=np.complex128)
        for ik in self.mesh:
            e = self.kpts[ik]
            A = self.phi[ik].conj() @ e.u.T
            if self.metal:
                A = A * np.sqrt(self.f[ik])[None, :]
            for s in range(self.n_hub):
                sl = slice(5 * s, 5 * s + 5)
                out[s] += self.occ * e.weight * A[sl] @ A[sl].conj().T
        return out

    def site_traces(self) -> Tuple[np.ndarray, np.ndarray]:
        """Per Hubbard site: the occupation trace summed over spins, sum_s Tr n^{I s} (Eq. 3),
        and the moment Tr n^{I up} - Tr n^{I dn} (zero when unpolarized)."""
        tr = np.zeros((self.nspin, self.n_hub))
        for ik in self.mesh:
            e = self.kpts[ik]
            A = self.phi[ik].conj() @ e.u.T
            f = self.f[ik] if self.metal else np.ones(self.n_occ)   # occupations of the bands
            w = self.occ * e.weight * (np.abs(A) ** 2 @ f)
            tr[self.spin_of(ik)] += w.reshape(self.n_hub, 5).sum(axis=1)
        mom = tr[0] - tr[1] if self.nspin == 2 else np.zeros(self.n_hub)
        return tr.sum(axis=0), mom

    # ------------------------------------------------------------ SCF loop
    def scf(self, site: int, q, p: ScfParams = ScfParams(), verbose: bool = False):
        """Self-consistent solution of Eq. 15 for the perturbation of Hubbard site
        `site` at wavevector q.  Returns a dict with dn0 (first iteration, Hxc
        response not yet built up: the chi0 column, paper's linear-response
        calculation section) and dn (self-consistent), each (n_hub, 5, 5)."""
        q = np.asarray(q, dtype=np.float64)
        shape = self.fft if self.nspin == 1 else (2,) + self.fft
        dv_in = np.zeros(shape, dtype=np.complex128)
        du = {}
        hist_df: List[np.ndarray] = []
        hist_dv: List[np.ndarray] = []
        prev = None
        chi_prev = None
        dn0 = None
        dn = None
        it_total = 0
        converged = False
        for it in range(1, p.niter_max + 1):
            drho = np.zeros(shape, dtype=np.complex128)
            dn = np.zeros((self.n_hub, 5, 5), dtype=np.complex128)
            for ik in self.mesh:
                b = self.rhs(ik, q, site, dv_in if it > 1 else None)
                du[ik], nit = self.solve(ik, q, b, du.get(ik), p)
                it_total += nit
                if self.nspin == 1:
                    drho += self.drho_k(ik, q, du[ik])
                else:
                    drho[self.spin_of(ik)] += self.drho_k(ik, q, du[ik])
                dn += self.dn_k(ik, q, du[ik])
            if self.metal and np.all(np.abs(q - np.round(q)) < 1e-12):
                # Fermi-level shift: density and occupations of the states at the Fermi level
                X = {ik: self.perturbed_vectors(ik, q, site, dv_in if it > 1 else None) for ik in self.mesh}
                def_ = self.fermi_shift(X)
                for ik in self.mesh:
                    e = self.kpts[ik]
                    g = 2.0 * e.weight * self.dlt[ik] / self.degauss * def_   # occupation change per band
                    drho += np.einsum("i,ixyz->xyz", g, np.abs(self.psi_r(ik)) ** 2) / self.omega
                    A = self.phi[ik].conj() @ e.u.T
                    for s2 in range(self.n_hub):
                        a = A[5 * s2:5 * s2 + 5]
                        dn[s2] += (a * g[None, :]) @ a.conj().T
            chi = np.einsum("smm->s", dn)
            if it == 1:
                dn0 = dn.copy()
            dv_out = self.dv_hxc(drho, q, p.hxc)
            f = dv_out - dv_in
            fn = np.linalg.norm(f)
            vn = max(np.linalg.norm(dv_out), 1e-300)
            if verbose:
                dchi = np.nan if chi_prev is None else np.abs(chi - chi_prev).max()
                print(f"  scf it {it}: |dchi| {dchi:.3e}  |f|/|v| {fn / vn:.3e}", flush=True)
            if not p.hxc or fn == 0.0:
                converged = True
                break
            if chi_prev is not None and np.abs(chi - chi_prev).max() < p.conv_thr_chi and fn / vn < p.conv_thr_v:
                converged = True
                break
            chi_prev = chi
            dv_new = self._mix(dv_in, f, prev, hist_df, hist_dv, p)
            prev = (dv_in, f)
            dv_in = dv_new
        return {"dn0": dn0, "dn": dn, "iters": it, "cg_iters": it_total, "converged": converged}

    def _mix(self, vin, f, prev, hist_df, hist_dv, p: ScfParams):
        """Modified Broyden mixing of the response potential (Johnson 1988, with
        unit weights and no w0 term, i.e. the Anderson form): the new input is
        vin + a f - sum_i g_i (a df_i + dv_i), g = inv(<df_i|df_j>) <df_j|f>."""
        if prev is not None:
            vin_prev, f_prev = prev
            df = f - f_prev
            nrm = np.linalg.norm(df)
            hist_df.append(df / nrm)
            hist_dv.append((vin - vin_prev) / nrm)
            if len(hist_df) > p.nmix:
                hist_df.pop(0)
                hist_dv.pop(0)
        a = p.alpha_mix
        if not hist_df:
            return vin + a * f
        n = len(hist_df)
        G = np.array([[np.vdot(hist_df[i], hist_df[j]) for j in range(n)] for i in range(n)])
        rhs = np.array([np.vdot(hist_df[i], f) for i in range(n)])
        g = np.linalg.solve(G, rhs)
        out = vin + a * f
        for i in range(n):
            out = out - g[i] * (a * hist_df[i] + hist_dv[i])
        return out

    # -------------------------------------------------------- full response
    def response_matrix(self, p: ScfParams = ScfParams(), verbose: bool = False):
        """chi0, chi over the N_H N_q sites of the q-supercell (Eq. 12 with Eq. 7)."""
        qs = self.gs.qpoints()
        chi0_q = np.zeros((len(qs), self.n_hub, self.n_hub), dtype=np.complex128)
        chi_q = np.zeros_like(chi0_q)
        for iq, q in enumerate(qs):
            for sp in range(self.n_hub):
                r = self.scf(sp, q, p, verbose=verbose)
                chi0_q[iq, :, sp] = np.einsum("smm->s", r["dn0"])
                chi_q[iq, :, sp] = np.einsum("smm->s", r["dn"])
        chi0, im0 = assemble_chi(chi0_q, qs, self.gs.qmesh)
        chi, im1 = assemble_chi(chi_q, qs, self.gs.qmesh)
        return chi0, chi, max(im0, im1), chi0_q, chi_q

    # ------------------------------------------------- independent references
    def sos_solve(self, ik: int, q, b: np.ndarray) -> np.ndarray:
        """Sum over all empty states of the full dense spectrum at k+q:
        du_v = sum_c u_c <u_c|b_v> / (eps_c - eps_vk)  (Eq. 15 with P_c b = b)."""
        j, _ = self.kq_entry(ik, q)
        w, V = np.linalg.eigh(self.h_dense(j))
        C = V[:, self.n_occ:]
        coef = C.conj().T @ b.T                      # (n_c, n_v)
        den = w[self.n_occ:, None] - self.kpts[ik].eps[None, :]
        return (C @ (coef / den)).T

    def fd_occupation_response(self, site: int, lam: float, hxc: bool = True, tol: float = 1e-13,
                               maxit: int = 200) -> np.ndarray:
        """Central finite difference [n^I(+lam) - n^I(-lam)] / 2 lam of the self-consistent
        ground state under lam sum_m |phi^J_m><phi^J_m| on every spin (Eq. 7 by its
        definition).  Gamma-only systems; with hxc=False the Hxc potential is frozen (chi0)."""
        assert self.nk_spin == 1 and np.allclose(self.kpts[0].k_frac, 0.0)
        res = []
        for sgn in (+1.0, -1.0):
            res.append(self._perturbed_ground_state(site, sgn * lam, hxc, tol, maxit))
        return (res[0] - res[1]) / (2.0 * lam)

    def _perturbed_ground_state(self, site, lam, hxc, tol, maxit):
        ns = self.nspin
        sl = slice(5 * site, 5 * site + 5)
        Pj = self.phi[0][sl].T @ self.phi[0][sl].conj()   # sum_m |phi_m><phi_m|
        rho0 = np.asarray(self.gs.rho0, dtype=np.float64).reshape((ns,) + self.fft)

        def vxc(r):  # per-spin xc potential of spin densities r, (ns,) + grid
            return pz81.v_xc(r[0])[None] if ns == 1 else pz81.v_xc_spin(r[0], r[1])

        vxc0 = vxc(rho0)
        g2 = self.gvec_q(np.zeros(3))
        e = self.kpts[0]
        idx = self.grid_index(0)
        dm = (e.miller[:, None, :] - e.miller[None, :, :]) % np.array(self.fft)
        rho_in = rho0.copy()
        hist_r, hist_f = [], []
        for it in range(maxit):
            if hxc:
                dg = np.fft.fftn(rho_in.sum(0) - rho0.sum(0)) / self.nr
                vh = np.where(g2 > 1e-12, FOUR_PI * dg / np.where(g2 > 1e-12, g2, 1.0), 0.0)
                v = (np.fft.ifftn(vh) * self.nr).real[None] + vxc(rho_in) - vxc0
            else:
                v = np.zeros((ns,) + self.fft)
            rho_out = np.zeros_like(rho_in)
            Us = []
            for sp in range(ns):
                ie = sp * self.nk_spin
                vhat = np.fft.fftn(v[sp]) / self.nr
                H = self.h_dense(ie) + lam * Pj + vhat[dm[..., 0], dm[..., 1], dm[..., 2]]
                w, V = np.linalg.eigh(0.5 * (H + H.conj().T))
                if self.metal:  # Fermi level of the unperturbed electron count, all bands
                    f = self._occupations_for(w)
                    keep = f > 1e-15
                    U, fw = V[:, keep].T, f[keep]
                else:
                    U, fw = V[:, :self.n_occ].T, np.ones(self.n_occ)
                Us.append((U, fw))
                psi = self.to_real(U, idx)
                rho_out[sp] = self.occ * np.einsum("i,ixyz->xyz", fw, np.abs(psi) ** 2) / self.omega
            f = rho_out - rho_in
            if not hxc or np.abs(f).max() < tol:
                break
            # Anderson mixing of the (spin) densities
            hist_r.append(rho_in.copy())
            hist_f.append(f.copy())
            if len(hist_r) > 6:
                hist_r.pop(0)
                hist_f.pop(0)
            n = len(hist_f)
            if n > 1:
                dF = [hist_f[i + 1] - hist_f[i] for i in range(n - 1)]
                dR = [hist_r[i + 1] - hist_r[i] for i in range(n - 1)]
                Gm = np.array([[np.vdot(a, b2).real for b2 in dF] for a in dF])
                rh = np.array([np.vdot(a, f).real for a in dF])
                g = np.linalg.lstsq(Gm, rh, rcond=None)[0]
                r_opt = rho_in - sum(g[i] * dR[i] for i in range(n - 1))
                f_opt = f - sum(g[i] * dF[i] for i in range(n - 1))
                rho_in = r_opt + 0.3 * f_opt
            else:
                rho_in = rho_in + 0.3 * f
        else:
            raise RuntimeError("perturbed ground state did not converge")
        n = np.zeros(self.n_hub)
        for U, fw in Us:
            A = self.phi[0].conj() @ U.T
            n += np.array([self.occ * np.sum(fw[None, :] * np.abs(A[5 * s:5 * s + 5]) ** 2)
                           for s in range(self.n_hub)])
        return n

    def _occupations_for(self, w: np.ndarray) -> np.ndarray:
        """Cold-smearing occupations of the Gamma-only eigenvalues w with the Fermi level that
        keeps the ground state's electron count (bisection)."""
        n_el = sum(2.0 * self.kpts[ik].weight * self.f[ik].sum() for ik in self.mesh)
        lo, hi = w.min() - 20 * self.degauss, w.max() + 20 * self.degauss
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if 2.0 * cold_occupation((mid - w) / self.degauss).sum() < n_el:
                lo = mid
            else:
                hi = mid
        return cold_occupation((0.5 * (lo + hi) - w) / self.degauss)


def loewdin(rows: np.ndarray) -> np.ndarray:
    """Symmetric (Loewdin) orthonormalization of a set of plane-wave rows (Eq. 6):
    phi~_i = sum_j (O^-1/2)_ji phi_j with O_ij = <phi_i|phi_j>."""
    O = rows.conj() @ rows.T
    w, U = np.linalg.eigh(O)
    X = (U * w ** -0.5) @ U.conj().T
    return X.T @ rows


def ortho_atomic_phi(gs, e) -> np.ndarray:
    """Ortho-atomic Hubbard projectors of k-entry e (Eq. 6): every atomic orbital of the system
    (synth.atomic_orbitals, an input) Loewdin-orthogonalized, then the Hubbard d rows."""
    from synth.system import atomic_orbitals
    rows, hub_rows = atomic_orbitals(gs, e.k_frac, e.miller)
    return loewdin(rows)[hub_rows]


def supercell_cells(qmesh) -> np.ndarray:
    """Integer cell offsets l of the q-supercell, lexicographic with the last index fastest."""
    n1, n2, n3 = qmesh
    return np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)], dtype=np.float64)


def assemble_chi(chi_q: np.ndarray, qs: np.ndarray, qmesh) -> Tuple[np.ndarray, float]:
    """Eq. 12 traced over m: chi_{(s,l),(s',l')} = (1/N_q) sum_q e^{iq.(R_l - R_l')} chi(q)_{s s'}.
    Site index = l * n_hub + s.  Returns the real part and max |imaginary part|."""
    nq, nh, _ = chi_q.shape
    cells = supercell_cells(qmesh)
    nc = cells.shape[0]
    out = np.zeros((nc * nh, nc * nh), dtype=np.complex128)
    for l in range(nc):
        for lp in range(nc):
            ph = np.exp(2j * math.pi * (qs @ (cells[l] - cells[lp])))
            blk = np.einsum("q,qab->ab", ph, chi_q) / nq
            out[l * nh:(l + 1) * nh, lp * nh:(lp + 1) * nh] = blk
    return out.real.copy(), float(np.abs(out.imag).max())


def nearest_neighbours(cell, hub_tau, qmesh, dist_thr: float = 6e-4):
    """Nearest-neighbour pairs for the inter-site V of Eq. 9 in the q-supercell of Eq. 12
    (site index l * n_hub + s as in assemble_chi): for each primitive site I, every other
    supercell site at I's smallest minimum-image distance (within dist_thr, bohr).
    Brute force over all sites and supercell images two shells out.  Returns (I, J, d)."""
    A = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    tau = np.asarray(hub_tau, dtype=np.float64).reshape(-1, 3)
    nh = tau.shape[0]
    cells = supercell_cells(qmesh)
    pos = (cells @ A)[:, None, :] + tau[None, :, :]
    pos = pos.reshape(-1, 3)
    a_sc = np.diag(np.asarray(qmesh, dtype=np.float64)) @ A
    rng = np.arange(-2, 3)
    shifts = np.array(np.meshgrid(rng, rng, rng, indexing="ij")).reshape(3, -1).T @ a_sc
    out = []
    for i in range(nh):
        d = np.linalg.norm(pos[None, :, :] - pos[i][None, None, :] + shifts[:, None, :], axis=2).min(axis=0)
        d[i] = np.inf
        dmin = d.min()
        if not np.isfinite(dmin):  # a lone site in a one-cell supercell has no neighbours
            continue
        for j in np.nonzero(d <= dmin + dist_thr)[0]:
            out.append((i, int(j), float(d[j])))
    return out


def cold_occupation(x):
    """Marzari-Vanderbilt (cold) smearing occupation of x = (e_F - e)/sigma: the integral from
    -infinity to x of (1/sqrt(pi)) exp(-u^2) (1 - sqrt(2) u), u = t - 1/sqrt(2)."""
    from scipy.special import erf
    u = np.asarray(x, dtype=np.float64) - 1.0 / math.sqrt(2.0)
    return 0.5 * (1.0 + erf(u)) + np.exp(-u * u) / math.sqrt(2.0 * math.pi)


def cold_delta(x):
    """Derivative of cold_occupation: (1/sqrt(pi)) exp(-u^2) (1 - sqrt(2) u), u = x - 1/sqrt(2)."""
    u = np.asarray(x, dtype=np.float64) - 1.0 / math.sqrt(2.0)
    return np.exp(-u * u) * (1.0 - math.sqrt(2.0) * u) / math.sqrt(math.pi)


def smooth_step(x):
    """The step that splits pairs of states, (1 + erf(x))/2; step(x) + step(-x) = 1."""
    from scipy.special import erf
    return 0.5 * (1.0 + erf(np.asarray(x, dtype=np.float64)))


def equivalent_sites(traces, docc_thr: float = 5e-5) -> np.ndarray:
    """Perturbation classes from the ground-state occupations (the paper's default search for
    the atoms to perturb, with its docc_thr): site s joins the class of the first earlier
    representative whose spin-summed occupation trace differs by less than docc_thr, else it
    represents a class of its own.  Returns the representative of every site."""
    rep = []
    for s, t in enumerate(traces):
        r = s
        for u in range(s):
            if rep[u] == u and abs(traces[u] - t) < docc_thr:
                r = u
                break
        rep.append(r)
    return np.array(rep, dtype=np.int64)


def supercell_distances(cell, hub_tau, qmesh) -> np.ndarray:
    """Minimum-image distances between all sites of the q-supercell (index l * n_hub + s)."""
    A = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    tau = np.asarray(hub_tau, dtype=np.float64).reshape(-1, 3)
    pos = ((supercell_cells(qmesh) @ A)[:, None, :] + tau[None, :, :]).reshape(-1, 3)
    a_sc = np.diag(np.asarray(qmesh, dtype=np.float64)) @ A
    rng = np.arange(-2, 3)
    shifts = np.array(np.meshgrid(rng, rng, rng, indexing="ij")).reshape(3, -1).T @ a_sc
    d = pos[:, None, None, :] - pos[None, :, None, :] + shifts[None, None, :, :]
    return np.linalg.norm(d, axis=3).min(axis=2)


def reconstruct_chi(chi, site_rep, cell, hub_tau, qmesh, moments=None, dist_thr: float = 6e-4):
    """Fill the columns of the q-supercell response matrix whose primitive site was not
    perturbed (site_rep[s] != s), by comparing inter-site distances, classes and the relative
    orientation of the moments (paper, post-processing of the response matrices): chi[I][J]
    is taken from the first computed chi[I2][J2] (J2 scanned before I2, both ascending) with
    rep(J2) = rep(J), rep(I2) = rep(I), the same sign of m_I m_J, and |d(I2,J2) - d(I,J)|
    <= dist_thr.  Raises if an element has no match."""
    nh = len(site_rep)
    n = chi.shape[0]
    D = supercell_distances(cell, hub_tau, qmesh)
    rep = np.array([site_rep[i % nh] for i in range(n)])
    m = np.zeros(nh) if moments is None else np.asarray(moments, dtype=np.float64)
    sg = np.array([0 if abs(m[i % nh]) <= 1e-6 else (1 if m[i % nh] > 0 else -1) for i in range(n)])
    computed = np.array([site_rep[j % nh] == j % nh for j in range(n)])
    out = chi.copy()
    for J in range(n):
        if computed[J]:
            continue
        for I in range(n):
            found = False
            for J2 in range(n):
                if not computed[J2] or rep[J2] != rep[J]:
                    continue
                for I2 in range(n):
                    if rep[I2] == rep[I] and sg[I2] * sg[J2] == sg[I] * sg[J] and \
                            abs(D[I2, J2] - D[I, J]) <= dist_thr:
                        out[I, J] = chi[I2, J2]
                        found = True
                        break
                if found:
                    break
            if not found:
                raise ValueError(f"no equivalent computed element for chi[{I}][{J}]")
    return out


def hubbard_params(chi0: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """U on the diagonal, V off the diagonal: chi0^-1 - chi^-1 (Eqs. 8-9)."""
    return np.linalg.inv(chi0) - np.linalg.inv(chi)
