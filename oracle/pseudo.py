"""Analytic pseudopotential transforms (oracle).

Fourier convention: f(G) = integral f(r) exp(-i G.r) d^3r.

Appelbaum-Hamann-form local potential
    v(r) = -(Z/r) erf(sqrt(a) r) + (v1 + v2 r^2) exp(-a r^2)
    v(G) = -(4 pi Z/G^2) e^{-G^2/4a} + (pi/a)^{3/2} e^{-G^2/4a} [v1 + v2 (3/(2a) - G^2/(4a^2))]
Gaussian-form local potential (width rloc)
    v(r) = -(Z/r) erf(r/(sqrt2 rloc)) + e^{-r^2/(2 rloc^2)} [c1 + c2 (r/rloc)^2]
    v(G) = -(4 pi Z/G^2) e^{-G^2 rloc^2/2} + (2 pi)^{3/2} rloc^3 e^{-G^2 rloc^2/2} [c1 + c2 (3 - G^2 rloc^2)]
The G = 0 value used for the local energy is the finite part
lim_{G->0} [v(G) + 4 pi Z / G^2] (neutralising-background convention).

Kleinman-Bylander projector, channel l, width r_l, normalised radial part
    p_l(r) = sqrt2 r^l e^{-r^2/(2 r_l^2)} / (r_l^{l+3/2} sqrt(Gamma(l+3/2)))
    p_l(G) = 4 pi int r^2 p_l(r) j_l(G r) dr
           = 4 pi sqrt(pi) r_l^{l+3/2} G^l e^{-G^2 r_l^2/2} / sqrt(Gamma(l+3/2))
and beta_{I l m}(G) = p_l(|G|) (-i)^l Y_lm(G^) e^{-i G.R_I} / sqrt(Omega)
with real harmonics Y_00 = (4 pi)^-1/2, Y_1(x,y,z) = sqrt(3/(4 pi)) (x,y,z)/|G|.
"""
import math
import numpy as np


def local_ft(local, Z, G):
    """v_s(|G|) for G != 0 (G may be an array of magnitudes > 0)."""
    G = np.asarray(G, dtype=float)
    g2 = G * G
    if local["kind"] == "ah":
        a, v1, v2 = local["alpha"], local["v1"], local["v2"]
        e = np.exp(-g2 / (4 * a))
        return (-4 * np.pi * Z / g2 * e
                + (np.pi / a) ** 1.5 * e * (v1 + v2 * (1.5 / a - g2 / (4 * a * a))))
    if local["kind"] == "gauss":
        rl, c1, c2 = local["rloc"], local["c1"], local["c2"]
        e = np.exp(-0.5 * g2 * rl * rl)
        return (-4 * np.pi * Z / g2 * e
                + (2 * np.pi) ** 1.5 * rl ** 3 * e * (c1 + c2 * (3 - g2 * rl * rl)))
    raise ValueError(local["kind"])


def local_short_ft(local, Z, G):
    """v_s(G) + 4 pi Z / G^2: the transform without the bare Coulomb tail;
    finite at G = 0 (used by the quadrature checks)."""
    G = np.asarray(G, dtype=float)
    g2 = G * G
    if local["kind"] == "ah":
        a, v1, v2 = local["alpha"], local["v1"], local["v2"]
        e = np.exp(-g2 / (4 * a))
        with np.errstate(divide="ignore", invalid="ignore"):
            coul = np.where(g2 > 0, 4 * np.pi * Z * (1 - e) / np.where(g2 > 0, g2, 1), np.pi * Z / a)
        return coul + (np.pi / a) ** 1.5 * e * (v1 + v2 * (1.5 / a - g2 / (4 * a * a)))
    if local["kind"] == "gauss":
        rl, c1, c2 = local["rloc"], local["c1"], local["c2"]
        e = np.exp(-0.5 * g2 * rl * rl)
        with np.errstate(divide="ignore", invalid="ignore"):
            coul = np.where(g2 > 0, 4 * np.pi * Z * (1 - e) / np.where(g2 > 0, g2, 1),
                            2 * np.pi * Z * rl * rl)
        return coul + (2 * np.pi) ** 1.5 * rl ** 3 * e * (c1 + c2 * (3 - g2 * rl * rl))
    raise ValueError(local["kind"])


def local_g0(local, Z):
    """lim_{G->0} [v(G) + 4 pi Z/G^2]."""
    return float(local_short_ft(local, Z, np.array([0.0]))[0])


def local_real(local, Z, r):
    """v(r) in real space (for the quadrature checks)."""
    from scipy.special import erf
    r = np.asarray(r, dtype=float)
    if local["kind"] == "ah":
        a, v1, v2 = local["alpha"], local["v1"], local["v2"]
        return -Z / r * erf(np.sqrt(a) * r) + (v1 + v2 * r * r) * np.exp(-a * r * r)
    rl, c1, c2 = local["rloc"], local["c1"], local["c2"]
    return (-Z / r * erf(r / (np.sqrt(2) * rl))
            + np.exp(-0.5 * (r / rl) ** 2) * (c1 + c2 * (r / rl) ** 2))


def projector_real(l, rl, r):
    r = np.asarray(r, dtype=float)
    return (np.sqrt(2.0) * r ** l * np.exp(-0.5 * (r / rl) ** 2)
            / (rl ** (l + 1.5) * math.sqrt(math.gamma(l + 1.5))))


def projector_ft(l, rl, G):
    G = np.asarray(G, dtype=float)
    return (4 * np.pi * np.sqrt(np.pi) * rl ** (l + 1.5) * G ** l
            * np.exp(-0.5 * G * G * rl * rl) / math.sqrt(math.gamma(l + 1.5)))


def real_ylm(l, Gvec):
    """Real spherical harmonics of the direction of each G (rows); for l = 1
    the order is (x, y, z).  Returns an array (n_m, nG).  At G = 0 the l = 1
    values are set to 0 (the radial factor G^l vanishes there anyway)."""
    Gvec = np.asarray(Gvec, dtype=float)
    if l == 0:
        return np.full((1, len(Gvec)), 1.0 / np.sqrt(4 * np.pi))
    if l == 1:
        g = np.linalg.norm(Gvec, axis=1)
        safe = np.where(g > 0, g, 1.0)
        u = Gvec / safe[:, None]
        u[g == 0] = 0.0
        return np.sqrt(3.0 / (4 * np.pi)) * u.T
    raise ValueError("only l = 0, 1")
