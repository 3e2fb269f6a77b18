"""Perdew-Zunger 1981 LDA, spin-unpolarised (oracle).

r_s = (3 / (4 pi rho))^{1/3};  eps_x = -(3/4)(3/pi)^{1/3} rho^{1/3} = -0.458165.../r_s.
Correlation (Ceperley-Alder parametrisation):
  r_s >= 1: eps_c = g / (1 + b1 sqrt(r_s) + b2 r_s)
  r_s <  1: eps_c = A ln r_s + B + C r_s ln r_s + D r_s
v_xc = d(rho eps_xc)/d rho.  Readings: the r_s >= 1 branch is used at r_s = 1;
rho <= 1e-30 gives eps = v = 0; callers pass max(rho, 0).
"""
import numpy as np

GAMMA, BETA1, BETA2 = -0.1423, 1.0529, 0.3334
A_, B_, C_, D_ = 0.0311, -0.048, 0.0020, -0.0116


def pz81(rho):
    rho = np.asarray(rho, dtype=float)
    eps = np.zeros_like(rho)
    v = np.zeros_like(rho)
    ok = rho > 1e-30
    r = rho[ok]
    rs = (3.0 / (4.0 * np.pi * r)) ** (1.0 / 3.0)
    ex = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * r ** (1.0 / 3.0)
    vx = 4.0 / 3.0 * ex
    hi = rs >= 1.0
    ec = np.empty_like(rs)
    vc = np.empty_like(rs)
    s = np.sqrt(rs[hi])
    den = 1.0 + BETA1 * s + BETA2 * rs[hi]
    ec[hi] = GAMMA / den
    vc[hi] = ec[hi] * (1.0 + 7.0 / 6.0 * BETA1 * s + 4.0 / 3.0 * BETA2 * rs[hi]) / den
    lo = ~hi
    x = rs[lo]
    lx = np.log(x)
    ec[lo] = A_ * lx + B_ + C_ * x * lx + D_ * x
    vc[lo] = A_ * lx + (B_ - A_ / 3.0) + 2.0 / 3.0 * C_ * x * lx + (2.0 * D_ - C_) / 3.0 * x
    eps[ok] = ex + ec
    v[ok] = vx + vc
    return eps, v
