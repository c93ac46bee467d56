"""Screening of the fifth force in NFW haloes, and the refinement level from
which the scalar-field iterations may be truncated.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the solver.  Plain
float64 numpy/scipy, written from the paper's equations in physical units,
with the enclosed mass integrated numerically from the density profile rather
than taken from its closed form:

  Eq. (nfw)        rho(r) = rho_s / ((r/r_s)(1 + r/r_s)^2)
  Eq. (nfwparams)  rho_s = (200/3) rho_c c^3 / (ln(1+c) - c/(1+c)),  r_s = R_200/c
  Eq. (r200)       R_200 = (3 M_200 / (4 pi 200 rho_c(z)))^(1/3)   [the printed
                   exponent -3 is read as 1/3: R_200 is the radius inside which
                   the mean density is 200 rho_c, as the text says]
  rho_c(z) = 3 H(z)^2 / (8 pi G)
  Eq. (rv)         r_V^3 = 16 r_c^2 G M(<r) / (9 beta^2)     (c = 1)
  Eq. (eomvarphi_sph2)
                   phi_,r = (4/(3 beta)) (r/r_V)^3 (sqrt(1 + (r_V/r)^3) - 1) G M / r^2
  F_5th = phi_,r / 2,  F_GR = G M(<r) / r^2,  G_eff - 1 = F_5th / F_GR (Sec. III.B)

Units: masses in M_sun/h, lengths in Mpc/h (physical), H in km/s/Mpc with
H0 = 100 h, so every h cancels.  Sec. V (conclusions): r_t is the radius where
G_eff - 1 falls to a chosen fraction; the levels whose cell size is at most
r_t are the truncated ones.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

G_MPC_KMS2_MSUN = 4.30091727e-9   # Newton's constant in Mpc (km/s)^2 / M_sun
H0_KMS_MPC_H = 100.0              # H0 in h km/s/Mpc
C_OVER_H0_MPC_H = 2997.92458      # c/H0 in Mpc/h


def rho_crit(e_z: float = 1.0) -> float:
    """Critical density 3 H^2 / (8 pi G) in (M_sun/h) / (Mpc/h)^3, H = E H0."""
    H = H0_KMS_MPC_H * e_z
    return 3.0 * H * H / (8.0 * math.pi * G_MPC_KMS2_MSUN)


def r200(m200: float, e_z: float = 1.0) -> float:
    """Eq. (r200) with exponent 1/3, Mpc/h."""
    return (3.0 * m200 / (4.0 * math.pi * 200.0 * rho_crit(e_z))) ** (1.0 / 3.0)


def nfw_params(m200: float, c200: float, e_z: float = 1.0):
    """(rho_s, r_s) of Eq. (nfwparams)."""
    mu = math.log(1.0 + c200) - c200 / (1.0 + c200)
    rho_s = 200.0 / 3.0 * rho_crit(e_z) * c200**3 / mu
    return rho_s, r200(m200, e_z) / c200


def nfw_density(r, m200: float, c200: float, e_z: float = 1.0):
    """Eq. (nfw)."""
    rho_s, rs = nfw_params(m200, c200, e_z)
    x = np.asarray(r, dtype=np.float64) / rs
    return rho_s / (x * (1.0 + x) ** 2)


def enclosed_mass(r: float, m200: float, c200: float, e_z: float = 1.0) -> float:
    """M(<r) = 4 pi int_0^r xi^2 rho(xi) d xi, by adaptive quadrature."""
    rho_s, rs = nfw_params(m200, c200, e_z)
    # integrate in u = xi / r_s: the integrand u / (1 + u)^2 is smooth at 0
    val, _ = integrate.quad(lambda u: u / (1.0 + u) ** 2, 0.0, r / rs, epsabs=0.0,
                            epsrel=1e-13, limit=200)
    return 4.0 * math.pi * rho_s * rs**3 * val


def force_ratio(r: float, m200: float, c200: float, rc: float, beta: float,
                e_z: float = 1.0) -> float:
    """F_5th / F_GR = G_eff - 1 at physical radius r (Mpc/h), Eqs. (rv) and
    (eomvarphi_sph2)."""
    M = enclosed_mass(r, m200, c200, e_z)
    gm = G_MPC_KMS2_MSUN * M                       # Mpc (km/s)^2
    rc_len = rc * C_OVER_H0_MPC_H                  # r_c in Mpc/h
    c_kms = C_OVER_H0_MPC_H * H0_KMS_MPC_H         # c in km/s (h cancels)
    rv3 = 16.0 * rc_len**2 * gm / (9.0 * beta**2 * c_kms**2)
    if rv3 == 0.0:                                 # r_c = 0: the unscreened limit
        return 1.0 / (3.0 * beta)
    y = r**3 / rv3                                 # (r / r_V)^3
    f_gr = gm / r**2
    phi_r = 4.0 / (3.0 * beta) * y * (math.sqrt(1.0 + 1.0 / y) - 1.0) * f_gr
    return 0.5 * phi_r / f_gr


def screening_radius(fraction: float, m200: float, c200: float, rc: float, beta: float,
                     e_z: float = 1.0) -> float:
    """r_t (Mpc/h): the radius inside which G_eff - 1 <= fraction (Sec. V).
    inf if the unscreened value 1/(3 beta) is not above fraction, 0 if
    fraction <= 0."""
    if fraction <= 0.0:
        return 0.0
    if fraction >= 1.0 / (3.0 * beta) or rc == 0.0:
        return math.inf
    R = r200(m200, e_z)
    g = lambda lr: force_ratio(math.exp(lr), m200, c200, rc, beta, e_z) - fraction
    lo, hi = math.log(R) - 1.0, math.log(R) + 1.0
    while g(lo) > 0.0:
        lo -= 2.0
    while g(hi) < 0.0:
        hi += 2.0
    return math.exp(optimize.brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500))


def truncation_level(h_domain: float, fraction: float, m200: float, c200: float, rc: float,
                     beta: float, e_z: float = 1.0) -> int:
    """First truncated refinement level k >= 1 (l_trunc = l_d + k): the
    coarsest refinement whose cell size h_domain / 2^k is at most r_t."""
    rt = screening_radius(fraction, m200, c200, rc, beta, e_z)
    if rt <= 0.0:
        raise ValueError("fraction must be > 0")
    k = 1
    while h_domain / 2.0**k > rt:
        k += 1
    return k
