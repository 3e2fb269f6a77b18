"""Fixed-basis stress of the discrete functional (oracle).

sigma_ab = (1/Omega) dF/d eps_ab for the homogeneous strain r -> (1 + eps) r
at a fixed set of Miller indices and fixed plane-wave coefficients (the
functional is stationary in the coefficients and occupations at
self-consistency).  Under the strain G -> (1 + eps)^-T G, so G.R is
invariant, d(G^2)/d eps_ab = -2 G_a G_b and Omega -> Omega (1 + tr eps);
the grid density scales as 1/Omega.  Term by term (symmetrised):
  kinetic   -(1/Omega) sum_i f_i sum_G G_a G_b |c_iG|^2
  Hartree   (1/Omega) [-delta_ab E_H + Omega sum_{G in D, G != 0} 4 pi |rho(G)|^2 G_a G_b / G^4]
  xc        delta_ab (E_xc - int v_xc rho) / Omega
  local     (1/Omega) [-delta_ab E_loc - 2 sum_{G in D, G != 0} sum_I dv/dq(q = G^2) G_a G_b Re(e^{iG.R_I} rho(G))]
  nonlocal  (1/Omega) sum_i f_i sum_p h_p 2 Re[conj(P_pi) dP_pi/d eps_ab],
            dP/d eps = sum_G conj(d beta/d eps) c_G, with d beta/d eps from the
            1/sqrt(Omega) factor, the radial transform through q = G^2 and,
            for l = 1, the direction factor G_m (d G_m / d eps_ab = -delta_mb G_a)
  Ewald     analytic (see ewald.py).
Pressure convention: sigma = (1/Omega) dE/d eps, so a compressed cell has
negative diagonal entries.
"""
import math

import numpy as np

from .lda import pz81
from .ewald import ewald


def _dv_dq(local, Z, q):
    """d v_s / d(q = G^2) for G != 0."""
    if local["kind"] == "ah":
        a, v1, v2 = local["alpha"], local["v1"], local["v2"]
        e = np.exp(-q / (4 * a))
        coul = -4 * np.pi * Z * (-(1 / (4 * a)) * e / q - e / (q * q))
        gauss = (np.pi / a) ** 1.5 * e * (-(1 / (4 * a)) * (v1 + v2 * (1.5 / a - q / (4 * a * a)))
                                          - v2 / (4 * a * a))
        return coul + gauss
    rl, c1, c2 = local["rloc"], local["c1"], local["c2"]
    e = np.exp(-0.5 * q * rl * rl)
    coul = -4 * np.pi * Z * (-(0.5 * rl * rl) * e / q - e / (q * q))
    A = (2 * np.pi) ** 1.5 * rl ** 3
    gauss = A * e * (-(0.5 * rl * rl) * (c1 + c2 * (3 - q * rl * rl)) - c2 * rl * rl)
    return coul + gauss


def _sym(M):
    return 0.5 * (M + M.T)


def stress(res):
    """Returns (sigma[3,3], parts dict) for an oracle SCF result."""
    st = res["setup"]
    om = st.omega
    C, f = res["C"], res["occupations"]
    rho = res["rho"]
    parts = {}
    # kinetic
    w = (f[None, :] * np.abs(C) ** 2).sum(1)  # per G
    parts["kinetic"] = -np.einsum("g,ga,gb->ab", w, st.G, st.G) / om
    # Hartree and local
    rhoG = np.fft.fftn(rho) / st.ntot
    nz = st.dmask & (st.g2grid > 0)
    Gd = st.Ggrid[nz]
    q = st.g2grid[nz]
    rg = rhoG[nz]
    e_h = 0.5 * om * (4 * np.pi * np.abs(rg) ** 2 / q).sum()
    parts["hartree"] = (-np.eye(3) * e_h
                        + om * np.einsum("g,ga,gb->ab", 4 * np.pi * np.abs(rg) ** 2 / q ** 2, Gd, Gd)) / om
    e_loc = float(om * np.real(np.conj(st.vloc_G[st.dmask]) * rhoG[st.dmask]).sum())
    loc = np.zeros((3, 3))
    for I, s in enumerate(st.symbols):
        sp = st.species[s]
        dv = _dv_dq(sp["local"], sp["Z"], q)
        re = np.real(np.exp(1j * (Gd @ st.pos[I])) * rg)
        loc += -2 * np.einsum("g,ga,gb->ab", dv * re, Gd, Gd)
    parts["local"] = (-np.eye(3) * e_loc + loc) / om
    # xc
    rc = np.maximum(rho, 0.0)
    exc, vxc = pz81(rc)
    e_xc = om / st.ntot * (rc * exc).sum()
    vrho = om / st.ntot * (vxc * rc).sum()
    parts["xc"] = np.eye(3) * (e_xc - vrho) / om
    # nonlocal
    nl = np.zeros((3, 3))
    if st.beta.shape[1]:
        P = st.beta.conj().T @ C  # (nproj, nb)
        col = 0
        for I, s in enumerate(st.symbols):
            phase = np.exp(-1j * (st.G @ st.pos[I])) / np.sqrt(om)
            for ch in st.species[s]["kb"]:
                l, rl, h = ch["l"], ch["r"], ch["h"]
                if l == 0:
                    amp = (4 * np.pi * np.sqrt(np.pi) * rl ** 1.5 / math.sqrt(math.gamma(1.5))
                           / np.sqrt(4 * np.pi))
                    e = np.exp(-0.5 * st.g2 * rl * rl)
                    base = amp * e * phase                    # beta(G)
                    dq = amp * (-0.5 * rl * rl) * e * phase   # d beta / dq
                    dbeta = np.zeros((3, 3, st.npw), dtype=complex)
                    for a in range(3):
                        for b in range(3):
                            dbeta[a, b] = (-0.5 * (a == b) * base
                                           + dq * (-2 * st.G[:, a] * st.G[:, b]))
                    dP = (dbeta.reshape(9, -1).conj() @ C).reshape(3, 3, -1)
                    Pp = P[col]
                    nl += h * 2 * np.real(np.einsum("n,abn->ab", f * np.conj(Pp), dP))
                    col += 1
                else:
                    amp = (4 * np.pi * np.sqrt(np.pi) * rl ** 2.5 / math.sqrt(math.gamma(2.5))
                           * np.sqrt(3 / (4 * np.pi)))
                    e = np.exp(-0.5 * st.g2 * rl * rl)
                    for m in range(3):
                        base = -1j * amp * st.G[:, m] * e * phase
                        dbeta = np.zeros((3, 3, st.npw), dtype=complex)
                        for a in range(3):
                            for b in range(3):
                                dGm = -0.5 * ((m == b) * st.G[:, a] + (m == a) * st.G[:, b])
                                dbeta[a, b] = (-0.5 * (a == b) * base
                                               + (-1j) * amp * phase * e * dGm
                                               + base * (-0.5 * rl * rl) * (-2 * st.G[:, a] * st.G[:, b]))
                        dP = (dbeta.reshape(9, -1).conj() @ C).reshape(3, 3, -1)
                        Pp = P[col]
                        nl += h * 2 * np.real(np.einsum("n,abn->ab", f * np.conj(Pp), dP))
                        col += 1
    parts["nonlocal"] = _sym(nl) / om
    _, _, s_ew = ewald(st.lattice, st.Z, st.pos, want_stress=True)
    parts["ewald"] = _sym(s_ew)
    for k in ("kinetic", "hartree", "local"):
        parts[k] = _sym(parts[k])
    total = sum(parts.values())
    return total, parts
