"""LDA exchange-correlation (Perdew-Zunger 1981 fit of Ceperley-Alder), spin
unpolarized, Hartree units.  TEST INFRASTRUCTURE ONLY (see the package header).

The paper restricts HP to local and semi-local xc kernels (its statement of
scope); the response Hxc potential needs the LDA kernel f_xc = d v_xc / d rho
evaluated at the ground-state density.  Perdew & Zunger's correlation fit:

  r_s >= 1 : eps_c = gamma / (1 + beta1 sqrt(r_s) + beta2 r_s)
  r_s <  1 : eps_c = A ln r_s + B + C r_s ln r_s + D r_s

with gamma = -0.1423, beta1 = 1.0529, beta2 = 0.3334, A = 0.0311, B = -0.048,
C = 0.0020, D = -0.0116.  Exchange: eps_x = -(3/4) (3 rho / pi)^(1/3).
"""
import numpy as np

GAMMA, BETA1, BETA2 = -0.1423, 1.0529, 0.3334
A_, B_, C_, D_ = 0.0311, -0.048, 0.0020, -0.0116
RHO_MIN = 1e-10


def rs_of(rho):
    return (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)


def eps_xc(rho):
    """Energy per electron (Ha)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    m = rho > RHO_MIN
    r = rs_of(rho[m])
    ex = -0.75 * (3.0 * rho[m] / np.pi) ** (1.0 / 3.0)
    sq = np.sqrt(r)
    ec = np.where(r >= 1.0, GAMMA / (1.0 + BETA1 * sq + BETA2 * r),
                  A_ * np.log(r) + B_ + C_ * r * np.log(r) + D_ * r)
    out[m] = ex + ec
    return out


def v_xc(rho):
    """Potential d(rho eps_xc)/d rho (Ha)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    m = rho > RHO_MIN
    r = rs_of(rho[m])
    vx = -(3.0 * rho[m] / np.pi) ** (1.0 / 3.0)
    sq = np.sqrt(r)
    den = 1.0 + BETA1 * sq + BETA2 * r
    vc_hi = GAMMA * (1.0 + 7.0 / 6.0 * BETA1 * sq + 4.0 / 3.0 * BETA2 * r) / den ** 2
    vc_lo = A_ * np.log(r) + (B_ - A_ / 3.0) + 2.0 / 3.0 * C_ * r * np.log(r) + (2.0 * D_ - C_) * r / 3.0
    out[m] = vx + np.where(r >= 1.0, vc_hi, vc_lo)
    return out


def f_xc(rho):
    """Kernel d v_xc / d rho (Ha bohr^3); zero where rho < 1e-10."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    m = rho > RHO_MIN
    rr = rho[m]
    r = rs_of(rr)
    fx = -(1.0 / 3.0) * (3.0 / np.pi) ** (1.0 / 3.0) * rr ** (-2.0 / 3.0)
    sq = np.sqrt(r)
    num = 1.0 + 7.0 / 6.0 * BETA1 * sq + 4.0 / 3.0 * BETA2 * r
    den = 1.0 + BETA1 * sq + BETA2 * r
    dnum = 7.0 / 12.0 * BETA1 / sq + 4.0 / 3.0 * BETA2
    dden = 0.5 * BETA1 / sq + BETA2
    dv_hi = GAMMA * (dnum * den - 2.0 * num * dden) / den ** 3
    dv_lo = A_ / r + 2.0 / 3.0 * C_ * (np.log(r) + 1.0) + (2.0 * D_ - C_) / 3.0
    dv_drs = np.where(r >= 1.0, dv_hi, dv_lo)
    out[m] = fx + dv_drs * (-r / (3.0 * rr))
    return out
