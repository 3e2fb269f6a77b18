"""Hellmann-Feynman forces of the discrete functional (oracle).

F_I = F_loc + F_nl + F_ewald with
  F_loc,I = sum_{G in D, G != 0} G v_s(|G|) Im[e^{i G.R_I} rho(G)]
  F_nl,I  = -sum_i f_i sum_{p on I} h_p 2 Re[conj(P_pi) dP_pi],
            P_pi = <beta_p|psi_i>,  dP_pi = <-i G beta_p|psi_i>
  F_ewald = -dE_ewald/dR_I (analytic).
At self-consistency these are -dF/dR_I of the Mermin free energy.
"""
import numpy as np

from .pseudo import local_ft


def hf_forces(res):
    st = res["setup"]
    rhoG = np.fft.fftn(res["rho"]) / st.ntot
    nz = st.dmask & (st.g2grid > 0)
    Gd = st.Ggrid[nz]
    g = np.sqrt(st.g2grid[nz])
    rg = rhoG[nz]
    F_loc = np.zeros((st.nat, 3))
    for I, s in enumerate(st.symbols):
        sp = st.species[s]
        v = local_ft(sp["local"], sp["Z"], g)
        z = v * np.exp(1j * (Gd @ st.pos[I])) * rg
        F_loc[I] = (Gd * np.imag(z)[:, None]).sum(0)
    F_nl = np.zeros((st.nat, 3))
    if st.beta.shape[1]:
        C, f = res["C"], res["occupations"]
        P = st.beta.conj().T @ C
        for a in range(3):
            dbeta = -1j * st.G[:, a][:, None] * st.beta
            dP = dbeta.conj().T @ C
            contrib = -2 * (f[None, :] * st.h[:, None] * np.real(np.conj(P) * dP)).sum(1)
            np.add.at(F_nl[:, a], st.proj_atom, contrib)
    F = F_loc + F_nl + st.f_ewald
    return F, {"local": F_loc, "nonlocal": F_nl, "ewald": st.f_ewald.copy()}
