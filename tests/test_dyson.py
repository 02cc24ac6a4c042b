"""Dyson pin of the oracle's self-consistent response (Eq. 15 iterated with the Hxc response,
mixing, the response density and Eq. 13) on the one-site Gamma system, by a route that
shares none of that machinery: the full spectrum of the dense Hamiltonian, the bare
density response chi0_rr(G, G') on the density sphere (sum over all empty states), the
Hxc kernel K as a dense matrix in the same basis (Hartree diagonal plus the grid
convolution with f_xc), the exact solve drho = (1 - chi0_rr K)^-1 drho0, and the
occupation response to the total potential by a sum over states.

The response is the linear map the oracle defines (time reversal folded into the factor
4; the grid-defined local operators); at Gamma it equals the physical response.  Variants:
the ground-state Hubbard potential, ortho-atomic projectors, a spin-polarized system, and a
metal (full pair sum with fractional occupations plus the Fermi-level shift).
"""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle
from oracle import pz81
from conftest import ground_state


@pytest.mark.parametrize("name,projectors", [("sc1_gamma", "atomic"), ("sc1_gamma_u", "atomic"),
                                             ("sc1_gamma", "ortho-atomic")])
def test_dyson_solve_equals_self_consistent_sternheimer(name, projectors):
    """Plain, with the ground-state Hubbard potential in H (Eq. 5), and with ortho-atomic
    projectors (Eq. 6) for the perturbation and the occupations."""
    gs = ground_state(name)
    o = oracle.Oracle(gs, projectors=projectors)
    e = gs.kpts[0]
    fft, nr, omega = o.fft, o.nr, o.omega
    nocc = gs.n_occ
    # full spectrum at Gamma
    w, V = np.linalg.eigh(o.h_dense(0))
    U = V.T                                               # rows: all states, plane-wave coefficients
    idx = o.grid_index(0)
    psi = np.zeros((U.shape[0], nr), dtype=np.complex128)
    psi[:, idx] = U
    psi = (sfft.ifftn(psi.reshape((-1,) + fft), axes=(1, 2, 3)) * nr).reshape(U.shape[0], nr)
    # density sphere: every G of a product of two states (alias-free on this grid)
    freq = [np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n) for n in fft]
    M = np.stack(np.meshgrid(*freq, indexing="ij"), -1).reshape(-1, 3)
    gvec = M @ o.bvec
    gmax = np.sqrt(np.einsum("ij,ij->i", (e.miller @ o.bvec), (e.miller @ o.bvec)).max())
    S = np.nonzero(np.einsum("ij,ij->i", gvec, gvec) <= (2 * gmax) ** 2 + 1e-9)[0]
    # P[v, c, G] = (1/N) sum_r exp(-iGr) conj(psi_v) psi_c
    ne = U.shape[0] - nocc
    P = np.empty((nocc, ne, S.size), dtype=np.complex128)
    for v in range(nocc):
        prod = np.conj(psi[v])[None, :] * psi[nocc:]
        P[v] = (sfft.fftn(prod.reshape((-1,) + fft), axes=(1, 2, 3)).reshape(ne, nr) / nr)[:, S]
    den = w[:nocc, None] - w[None, nocc:]                 # e_v - e_c
    Pw = (P / den[:, :, None]).reshape(-1, S.size)
    chi0_rr = (4.0 / omega) * Pw.T @ np.conj(P.reshape(-1, S.size))      # (G, G')
    # Hxc kernel on the sphere: 4 pi / |G|^2 (0 at G = 0) + fhat(G - G') on the grid
    g2 = np.einsum("ij,ij->i", gvec[S], gvec[S])
    fhat = sfft.fftn(pz81.f_xc(gs.rho0)) / nr
    d = (M[S][:, None, :] - M[S][None, :, :]) % np.array(fft)
    K = fhat[d[..., 0], d[..., 1], d[..., 2]].astype(np.complex128)
    K[np.diag_indices(S.size)] += np.where(g2 > 1e-12, 4.0 * np.pi / np.where(g2 > 1e-12, g2, 1.0), 0.0)
    # bare response to the Hubbard projector of site 0 (Eq. 16)
    phi = o.phi[0][0:5]
    Vp = (U[nocc:].conj() @ phi.T) @ (phi.conj() @ U[:nocc].T)      # <c|V_pert|v>
    drho0 = (4.0 / omega) * np.einsum("vcg,cv->g", P / den[:, :, None], Vp)
    drho = np.linalg.solve(np.eye(S.size) - chi0_rr @ K, drho0)
    dv_hxc = K @ drho                                     # Fourier components on the sphere
    # <c|dV_Hxc|v> = sum_G' dv(G') <c|e^{iG'r}|v> = sum_G' dv(G') conj(P[v, c, G'])
    Vt = Vp + np.einsum("vcg,g->cv", np.conj(P), dv_hxc)
    dpsi = ((Vt / den.T).T @ U[nocc:])                    # rows v: sum_c u_c <c|dV|v>/(e_v - e_c)
    A = phi.conj() @ U[:nocc].T                           # <phi_m|u_v>
    B = phi.conj() @ dpsi.T                               # <phi_m|du_v>
    T = B @ A.conj().T
    dn = 2.0 * (T + T.T)                                  # Eq. 13, two-term form, weight 1
    ref = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-14, conv_thr_chi=1e-14, conv_thr_v=1e-12))
    assert np.abs(dn - ref["dn"][0]).max() < 1e-12 * np.abs(ref["dn"][0]).max()     # measured 1.1e-14
    chi, chi_ref = np.trace(dn).real, np.trace(ref["dn"][0]).real
    assert abs(chi - chi_ref) < 1e-12 * abs(chi_ref)                                  # measured 6.6e-15
    # and without the Hxc response the same route gives chi0
    B0 = phi.conj() @ ((Vp / den.T).T @ U[nocc:]).T
    T0 = B0 @ A.conj().T
    assert np.abs(2.0 * (T0 + T0.T) - ref["dn0"][0]).max() < 1e-12 * np.abs(ref["dn0"][0]).max()


def test_dyson_solve_spin_polarized():
    """The same construction for the polarized one-site system: per-spin bare responses
    (one electron per state, time reversal 2), the 2 x 2 LSDA kernel and the Hartree
    kernel of the total density, one joint solve for (drho_up, drho_dn)."""
    gs = ground_state("sc1_gamma_spin")
    o = oracle.Oracle(gs)
    fft, nr, omega = o.fft, o.nr, o.omega
    nocc = gs.n_occ
    freq = [np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n) for n in fft]
    M = np.stack(np.meshgrid(*freq, indexing="ij"), -1).reshape(-1, 3)
    gvec = M @ o.bvec
    e0 = gs.kpts[0]
    gmax = np.sqrt(np.einsum("ij,ij->i", (e0.miller @ o.bvec), (e0.miller @ o.bvec)).max())
    S = np.nonzero(np.einsum("ij,ij->i", gvec, gvec) <= (2 * gmax) ** 2 + 1e-9)[0]
    ns = S.size
    blocks = []
    for sp in range(2):
        e = gs.kpts[sp]
        w, V = np.linalg.eigh(o.h_dense(sp))
        U = V.T
        psi = np.zeros((U.shape[0], nr), dtype=np.complex128)
        psi[:, o.grid_index(sp)] = U
        psi = (sfft.ifftn(psi.reshape((-1,) + fft), axes=(1, 2, 3)) * nr).reshape(U.shape[0], nr)
        ne = U.shape[0] - nocc
        P = np.empty((nocc, ne, ns), dtype=np.complex128)
        for v in range(nocc):
            prod = np.conj(psi[v])[None, :] * psi[nocc:]
            P[v] = (sfft.fftn(prod.reshape((-1,) + fft), axes=(1, 2, 3)).reshape(ne, nr) / nr)[:, S]
        den = w[:nocc, None] - w[None, nocc:]
        chi0 = (2.0 / omega) * (P / den[:, :, None]).reshape(-1, ns).T @ np.conj(P.reshape(-1, ns))
        phi = e.phi[0:5]
        Vp = (U[nocc:].conj() @ phi.T) @ (phi.conj() @ U[:nocc].T)
        drho0 = (2.0 / omega) * np.einsum("vcg,cv->g", P / den[:, :, None], Vp)
        blocks.append((U, P, den, chi0, Vp, drho0, phi))
    g2 = np.einsum("ij,ij->i", gvec[S], gvec[S])
    vh = np.where(g2 > 1e-12, 4.0 * np.pi / np.where(g2 > 1e-12, g2, 1.0), 0.0)
    rho = np.asarray(gs.rho0).reshape((2,) + fft)
    f = pz81.f_xc_spin(rho[0], rho[1])
    d = (M[S][:, None, :] - M[S][None, :, :]) % np.array(fft)
    K = np.zeros((2 * ns, 2 * ns), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            fh = sfft.fftn(f[a, b]) / nr
            blk = fh[d[..., 0], d[..., 1], d[..., 2]].astype(np.complex128)
            blk[np.diag_indices(ns)] += vh
            K[a * ns:(a + 1) * ns, b * ns:(b + 1) * ns] = blk
    chi0 = np.zeros((2 * ns, 2 * ns), dtype=np.complex128)
    chi0[:ns, :ns], chi0[ns:, ns:] = blocks[0][3], blocks[1][3]
    drho0 = np.concatenate([blocks[0][5], blocks[1][5]])
    drho = np.linalg.solve(np.eye(2 * ns) - chi0 @ K, drho0)
    dv = K @ drho
    dn = np.zeros((5, 5), dtype=np.complex128)
    for sp, (U, P, den, _, Vp, _, phi) in enumerate(blocks):
        Vt = Vp + np.einsum("vcg,g->cv", np.conj(P), dv[sp * ns:(sp + 1) * ns])
        dpsi = (Vt / den.T).T @ U[nocc:]
        A = phi.conj() @ U[:nocc].T
        T = (phi.conj() @ dpsi.T) @ A.conj().T
        dn += T + T.T                                     # one electron per state, summed over spins
    ref = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-14, conv_thr_chi=1e-14, conv_thr_v=1e-12))
    assert np.abs(dn - ref["dn"][0]).max() < 1e-12 * np.abs(ref["dn"][0]).max()


def test_dyson_solve_metal_at_gamma():
    """Metallic one-site system at Gamma: the bare response is the full pair sum
    4/Omega sum_{i kept, j all} F_ij theta_ji conj(u_i) u_j <u_j|dV|u_i> (F_ij = (f_i - f_j) /
    (e_i - e_j), the occupation derivative at equal energies) plus the Fermi-level term
    (2/Omega) sum_i (d_i/sigma) |u_i|^2 * sum_i d_i <u_i|dV|u_i> / sum_i d_i, inverted
    exactly with the Hxc kernel, against the self-consistent Sternheimer response."""
    from oracle.hp_oracle import cold_delta, cold_occupation, smooth_step
    gs = ground_state("sc1_gamma_metal")
    o = oracle.Oracle(gs)
    e = gs.kpts[0]
    fft, nr, omega, sig = o.fft, o.nr, o.omega, gs.degauss
    nk = gs.n_occ                                          # kept bands
    w, V = np.linalg.eigh(o.h_dense(0))
    U = V.T
    psi = np.zeros((U.shape[0], nr), dtype=np.complex128)
    psi[:, o.grid_index(0)] = U
    psi = (sfft.ifftn(psi.reshape((-1,) + fft), axes=(1, 2, 3)) * nr).reshape(U.shape[0], nr)
    freq = [np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n) for n in fft]
    M = np.stack(np.meshgrid(*freq, indexing="ij"), -1).reshape(-1, 3)
    gvec = M @ o.bvec
    gmax = np.sqrt(np.einsum("ij,ij->i", (e.miller @ o.bvec), (e.miller @ o.bvec)).max())
    S = np.nonzero(np.einsum("ij,ij->i", gvec, gvec) <= (2 * gmax) ** 2 + 1e-9)[0]
    nall = U.shape[0]
    P = np.empty((nk, nall, S.size), dtype=np.complex128)
    for i in range(nk):
        prod = np.conj(psi[i])[None, :] * psi
        P[i] = (sfft.fftn(prod.reshape((-1,) + fft), axes=(1, 2, 3)).reshape(nall, nr) / nr)[:, S]
    f = cold_occupation((gs.efermi - w) / sig)
    dl = cold_delta((gs.efermi - w[:nk]) / sig)
    dd = w[:nk, None] - w[None, :]
    close = np.abs(dd) < 1e-9
    mid = 0.5 * (w[:nk, None] + w[None, :])
    F = np.where(close, -cold_delta((gs.efermi - mid) / sig) / sig, (f[:nk, None] - f[None, :]) / np.where(close, 1, dd))
    W = F * smooth_step(-dd / sig)                         # (i, j)
    chi0 = (4.0 / omega) * (P * W[:, :, None]).reshape(-1, S.size).T @ np.conj(P.reshape(-1, S.size))
    Pd = np.einsum("iig->ig", P[:, :nk])                   # FT of |u_i|^2
    rhoF = (2.0 / omega) * (dl / sig) @ Pd
    chi0 += np.outer(rhoF, (dl @ np.conj(Pd)) / dl.sum())  # Fermi-level shift, linear in dV
    g2 = np.einsum("ij,ij->i", gvec[S], gvec[S])
    fhat = sfft.fftn(pz81.f_xc(gs.rho0)) / nr
    d = (M[S][:, None, :] - M[S][None, :, :]) % np.array(fft)
    K = fhat[d[..., 0], d[..., 1], d[..., 2]].astype(np.complex128)
    K[np.diag_indices(S.size)] += np.where(g2 > 1e-12, 4.0 * np.pi / np.where(g2 > 1e-12, g2, 1.0), 0.0)
    phi = e.phi[0:5]
    Vp = (U.conj() @ phi.T) @ (phi.conj() @ U[:nk].T)      # <j|V_pert|i>, (j all, i kept)
    drho0 = (4.0 / omega) * np.einsum("ijg,ji->g", P * W[:, :, None], Vp)
    drho0 += rhoF * (dl @ np.diag(Vp[:nk])) / dl.sum()
    drho = np.linalg.solve(np.eye(S.size) - chi0 @ K, drho0)
    dv = K @ drho
    Vt = Vp + np.einsum("ijg,g->ji", np.conj(P), dv)       # <j|dV_total|i>
    dpsi = (W.T * Vt).T @ U                                # rows i: sum_j F theta u_j <j|dV|i>
    A = phi.conj() @ U[:nk].T
    T = (phi.conj() @ dpsi.T) @ A.conj().T
    dn = 2.0 * (T + T.T)
    shift = (dl @ np.diag(Vt[:nk])) / dl.sum()
    dn += (A * (2.0 * dl / sig * shift)[None, :]) @ A.conj().T
    ref = o.scf(0, np.zeros(3), oracle.ScfParams(cg_tol=1e-14, conv_thr_chi=1e-14, conv_thr_v=1e-12))
    assert np.abs(dn - ref["dn"][0]).max() < 1e-12 * np.abs(ref["dn"][0]).max()     # measured 8.5e-14
