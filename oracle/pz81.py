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


# ---------------------------------------------------------------------------
# Collinear spin-polarized form (LSDA).  Exchange from the spin-scaling relation
# E_x[rho_up, rho_dn] = (E_x[2 rho_up] + E_x[2 rho_dn]) / 2, i.e. the energy density
# -(3/4) (6/pi)^(1/3) (rho_up^(4/3) + rho_dn^(4/3)).  Correlation: Perdew & Zunger's
# interpolation between their unpolarized (U) and fully polarized (P) fits,
#   eps_c(r_s, zeta) = eps_U(r_s) + f(zeta) (eps_P(r_s) - eps_U(r_s)),
#   f(zeta) = ((1+zeta)^(4/3) + (1-zeta)^(4/3) - 2) / (2^(4/3) - 2),
# with the polarized parameters gamma = -0.0843, beta1 = 1.3981, beta2 = 0.2611,
# A = 0.01555, B = -0.0269, C = 0.0007, D = -0.0048.
# Readings: every output is zero where rho_up + rho_dn <= 1e-10; zeta is clipped to
# |zeta| <= 1 - 1e-12 (the kernel diverges at full polarization).
# ---------------------------------------------------------------------------

U_PARAMS = (GAMMA, BETA1, BETA2, A_, B_, C_, D_)
P_PARAMS = (-0.0843, 1.3981, 0.2611, 0.01555, -0.0269, 0.0007, -0.0048)
ZETA_MAX = 1.0 - 1e-12
_F_DEN = 2.0 ** (4.0 / 3.0) - 2.0


def _ec_rs(r, prm):
    """eps_c of one fit and its first two r_s derivatives."""
    g, b1, b2, a, b, c, d = prm
    sq = np.sqrt(r)
    den = 1.0 + b1 * sq + b2 * r
    den1 = 0.5 * b1 / sq + b2
    den2 = -0.25 * b1 / (r * sq)
    hi = (g / den, -g * den1 / den ** 2, g * (2.0 * den1 ** 2 / den ** 3 - den2 / den ** 2))
    lr = np.log(r)
    lo = (a * lr + b + c * r * lr + d * r, a / r + c * (lr + 1.0) + d, -a / r ** 2 + c / r)
    return tuple(np.where(r >= 1.0, h, l) for h, l in zip(hi, lo))


def _fz(z):
    """f(zeta) and its first two derivatives."""
    p, m = 1.0 + z, 1.0 - z
    f = (p ** (4.0 / 3.0) + m ** (4.0 / 3.0) - 2.0) / _F_DEN
    f1 = (4.0 / 3.0) * (p ** (1.0 / 3.0) - m ** (1.0 / 3.0)) / _F_DEN
    f2 = (4.0 / 9.0) * (p ** (-2.0 / 3.0) + m ** (-2.0 / 3.0)) / _F_DEN
    return f, f1, f2


def _spin_vars(rho_up, rho_dn):
    ru = np.asarray(rho_up, dtype=np.float64)
    rd = np.asarray(rho_dn, dtype=np.float64)
    rho = ru + rd
    m = rho > RHO_MIN
    rr = rho[m]
    z = np.clip((ru[m] - rd[m]) / rr, -ZETA_MAX, ZETA_MAX)
    return rho, m, rr, z


def _ec_spin(r, z):
    """eps_c(r_s, zeta) with the derivatives d/dr_s, d2/dr_s2, d/dzeta, d2/dzeta2, d2/dr_s dzeta."""
    u, u1, u2 = _ec_rs(r, U_PARAMS)
    p, p1, p2 = _ec_rs(r, P_PARAMS)
    f, f1, f2 = _fz(z)
    return (u + f * (p - u), u1 + f * (p1 - u1), u2 + f * (p2 - u2), f1 * (p - u), f2 * (p - u), f1 * (p1 - u1))


def eps_xc_spin(rho_up, rho_dn):
    """Energy per electron (Ha) of the spin-polarized LDA."""
    rho, m, rr, z = _spin_vars(rho_up, rho_dn)
    out = np.zeros_like(rho)
    r = rs_of(rr)
    ru, rd = 0.5 * rr * (1.0 + z), 0.5 * rr * (1.0 - z)
    ex = -0.75 * (6.0 / np.pi) ** (1.0 / 3.0) * (ru ** (4.0 / 3.0) + rd ** (4.0 / 3.0)) / rr
    out[m] = ex + _ec_spin(r, z)[0]
    return out


def v_xc_spin(rho_up, rho_dn):
    """Potentials d(rho eps_xc)/d rho_sigma, shape (2,) + grid (Ha)."""
    rho, m, rr, z = _spin_vars(rho_up, rho_dn)
    out = np.zeros((2,) + rho.shape)
    r = rs_of(rr)
    e, e_r, _, e_z, _, _ = _ec_spin(r, z)
    for s, sg in enumerate((1.0, -1.0)):
        rs_sig = 0.5 * rr * (1.0 + sg * z)
        vx = -(6.0 / np.pi) ** (1.0 / 3.0) * rs_sig ** (1.0 / 3.0)
        # d(rho eps)/d rho_s = eps - (r_s/3) eps_rs + (s - zeta) eps_zeta
        out[s][m] = vx + e - r / 3.0 * e_r + (sg - z) * e_z
    return out


def f_xc_spin(rho_up, rho_dn):
    """Kernel d v_xc^s / d rho_s', shape (2, 2) + grid (Ha bohr^3); symmetric in (s, s')."""
    rho, m, rr, z = _spin_vars(rho_up, rho_dn)
    out = np.zeros((2, 2) + rho.shape)
    r = rs_of(rr)
    e, e_r, e_rr, e_z, e_zz, e_rz = _ec_spin(r, z)
    a_r = 2.0 / 3.0 * e_r - r / 3.0 * e_rr      # d/dr_s of (eps - (r_s/3) eps_rs)
    sgn = (1.0, -1.0)
    for s in range(2):
        rs_sig = 0.5 * rr * (1.0 + sgn[s] * z)
        fx = -(1.0 / 3.0) * (6.0 / np.pi) ** (1.0 / 3.0) * rs_sig ** (-2.0 / 3.0)
        for t in range(2):
            # d/d rho_t = d/d rho + ((t - zeta)/rho) d/d zeta, with d r_s / d rho = -r_s / (3 rho)
            d_rho = -r / (3.0 * rr) * (a_r + (sgn[s] - z) * e_rz)
            d_zeta = -r / 3.0 * e_rz + (sgn[s] - z) * e_zz
            val = d_rho + (sgn[t] - z) / rr * d_zeta
            if s == t:
                val = val + fx
            out[s, t][m] = val
    return out
