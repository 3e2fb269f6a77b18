"""Ewald energy, forces and stress of point ions in a neutralising background
(oracle, FP64).

E = 1/2 sum_{I,J} sum'_L Z_I Z_J erfc(eta |R_I - R_J + L|) / |R_I - R_J + L|
  + (2 pi / Omega) sum_{G != 0} exp(-G^2 / (4 eta^2)) / G^2 |sum_I Z_I e^{i G.R_I}|^2
  - (eta / sqrt(pi)) sum_I Z_I^2 - pi (sum_I Z_I)^2 / (2 Omega eta^2)
The primed sum omits I = J at L = 0.  The result does not depend on eta;
each sum is cut where its terms fall below ~1e-16 relative.
"""
import numpy as np
from scipy.special import erfc

from .basis import cell_geometry


def default_eta(lattice, natoms):
    omega, _ = cell_geometry(lattice)
    return float(np.sqrt(np.pi) * (max(natoms, 1) / omega ** 2) ** (1.0 / 6.0))


def _lattice_points(A, rcut):
    """All L = n.A with |L| <= rcut (plus margin of one cell diagonal)."""
    B = 2 * np.pi * np.linalg.inv(A).T
    nmax = [int(np.ceil(rcut * np.linalg.norm(B[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-n, n + 1) for n in nmax]
    n = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    return n @ A


def _recip_points(B, gcut):
    A = 2 * np.pi * np.linalg.inv(B).T
    mmax = [int(np.ceil(gcut * np.linalg.norm(A[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-m, m + 1) for m in mmax]
    m = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    G = m @ B
    g2 = (G * G).sum(1)
    keep = (g2 > 0) & (g2 <= gcut * gcut)
    return G[keep]


def ewald(lattice, charges, positions, eta=None, want_stress=False):
    """Returns (energy, forces[nat,3]) or (energy, forces, stress[3,3]) where
    stress_ab = (1/Omega) dE/d eps_ab (symmetric strain, Cartesian)."""
    A = np.asarray(lattice, dtype=float)
    Z = np.asarray(charges, dtype=float)
    R = np.asarray(positions, dtype=float)
    nat = len(Z)
    omega, B = cell_geometry(A)
    if eta is None:
        eta = default_eta(A, nat)
    rcut = 6.2 / eta
    gcut = 2 * eta * 6.2
    Ls = _lattice_points(A, rcut + np.linalg.norm(A.sum(0)))
    E_real = 0.0
    F = np.zeros((nat, 3))
    S_real = np.zeros((3, 3))
    for i in range(nat):
        for j in range(nat):
            d = R[i] - R[j] + Ls  # vectors from ion j image to ion i
            r = np.sqrt((d * d).sum(1))
            use = (r > 1e-12) & (r <= rcut + 1e-9)
            d, r = d[use], r[use]
            ec = erfc(eta * r)
            E_real += 0.5 * Z[i] * Z[j] * (ec / r).sum()
            # -d/dr [erfc(eta r)/r]
            dphi = ec / (r * r) + 2 * eta / np.sqrt(np.pi) * np.exp(-(eta * r) ** 2) / r
            F[i] += Z[i] * Z[j] * ((dphi / r)[:, None] * d).sum(0)
            # dE/d eps_ab for pair term = 1/2 sum phi'(r) d_a d_b / r
            S_real -= 0.5 * Z[i] * Z[j] * np.einsum("k,ka,kb->ab", dphi / r, d, d)
    G = _recip_points(B, gcut)
    g2 = (G * G).sum(1)
    w = np.exp(-g2 / (4 * eta * eta)) / g2
    phase = np.exp(1j * (G @ R.T))  # (nG, nat)
    S = phase @ Z
    E_recip = 2 * np.pi / omega * (w * np.abs(S) ** 2).sum()
    # F_I = (4 pi / Omega) Z_I sum_G w G Im[conj(S) e^{i G.R_I}]
    im = np.imag(np.conj(S)[:, None] * phase)  # (nG, nat)
    F += 4 * np.pi / omega * Z[:, None] * (G.T @ (w[:, None] * im)).T
    E_self = -eta / np.sqrt(np.pi) * (Z * Z).sum()
    E_bg = -np.pi * Z.sum() ** 2 / (2 * omega * eta * eta)
    E = E_real + E_recip + E_self + E_bg
    if not want_stress:
        return E, F
    # reciprocal part: E_g = (2pi/Omega) sum w(G)|S|^2 ; under strain G -> (1-eps)G,
    # Omega -> Omega(1+tr eps); dw/dG^2 ...
    s2 = np.abs(S) ** 2
    x = g2 / (4 * eta * eta)
    # d/d eps_ab of [e^{-x}/g2] with dg2/deps_ab = -2 G_a G_b
    dwdg2 = -np.exp(-x) / g2 * (1.0 / (4 * eta * eta) + 1.0 / g2)
    S_recip = 2 * np.pi / omega * (
        np.einsum("k,ka,kb->ab", dwdg2 * s2 * (-2.0), G, G)) - E_recip * np.eye(3)
    S_bg = -E_bg * np.eye(3)
    stress = (S_real + S_recip + S_bg) / omega
    return E, F, stress
