"""Brillouin-zone sampling with k-points (oracle): the "rough K-points
sampling grid" that Section 2.3 lets the energy evaluations of a search use,
on the same discrete functional as the Gamma-point oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

Bloch states psi_nk(r) = e^{i k.r} u_nk(r) with
    u_nk(r) = Omega^-1/2 sum_G c_G e^{i G.r},   |k + G|^2 / 2 <= Ecut,
so every k has its own shifted sphere of coefficients, complex with no
relation between c(G) and c(-G).  For each k:
    (H_k u)_G = |k+G|^2/2 c_G + [V_eff u]_G + sum_p beta_kp(G) h_p <beta_kp|u>
    beta_{k,Ilm}(G) = p_l(|k+G|) (-i)^l Y_lm(k+G) e^{-i (k+G).R_I} / sqrt(Omega)
(the local potential acts on the periodic part on the same FFT grid).  With
weights w_k (sum w_k = 1):
    rho(r) = sum_k w_k sum_n f_nk |u_nk(r)|^2 / Omega,
    E_kin  = sum_k w_k sum_n f_nk sum_G |k+G|^2/2 |c|^2,
    E_nl   = sum_k w_k sum_n f_nk sum_p h_p |<beta_kp|u_nk>|^2,
and E_loc, E_H, E_xc, Ewald from rho and the ions as at Gamma.  Occupations:
fixed (the lowest N_el/2 states of every k doubly occupied) or Fermi-Dirac
with one chemical potential for all k (sum_k w_k sum_n f_nk = N_el).
Nonlocal forces carry the derivative -i (k + G) of the projector phase.
"""
import numpy as np
import scipy.linalg
from scipy.special import expit

from .hamiltonian import Setup
from .pseudo import projector_ft, real_ylm, local_ft
from .basis import box_index, check_grid
from .scf import potentials, energy_terms


def shifted_sphere(B, lattice, kfrac, ecut):
    """Every integer triple m with |(m + k) B|^2 / 2 <= ecut, k in units of
    the reciprocal basis vectors."""
    A = np.asarray(lattice, dtype=float)
    gmax = np.sqrt(2.0 * ecut)
    mmax = [int(np.floor(gmax * np.linalg.norm(A[i]) / (2 * np.pi) + abs(kfrac[i]))) + 1
            for i in range(3)]
    r = [np.arange(-mm, mm + 1) for mm in mmax]
    m = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    q = (m + np.asarray(kfrac)) @ B
    keep = 0.5 * (q * q).sum(1) <= ecut
    return m[keep]


class KSetup:
    """Everything of one k-point that depends on geometry only; the grid
    side (local potential, density set, Ewald) is the Gamma setup's."""

    def __init__(self, base, kfrac):
        self.base = base
        self.kf = np.asarray(kfrac, dtype=float)
        self.k = self.kf @ base.B
        self.millers = shifted_sphere(base.B, base.lattice, self.kf, base.ecut)
        if not check_grid(self.millers, base.grid):
            raise ValueError("grid too small for the wavefunction sphere at this k")
        self.q = (self.millers + self.kf) @ base.B  # k + G
        self.kin = 0.5 * (self.q * self.q).sum(1)
        self.npw = len(self.millers)
        self.box = box_index(self.millers, base.grid)
        self.beta, self.h, self.proj_atom = self._projectors()

    def _projectors(self):
        b = self.base
        cols, hs, owner = [], [], []
        g = np.sqrt((self.q * self.q).sum(1))
        for I, s in enumerate(b.symbols):
            phase = np.exp(-1j * (self.q @ b.pos[I]))
            for ch in b.species[s]["kb"]:
                l = ch["l"]
                radial = projector_ft(l, ch["r"], g)
                Y = real_ylm(l, self.q)
                for mm in range(Y.shape[0]):
                    cols.append(radial * (-1j) ** l * Y[mm] * phase / np.sqrt(b.omega))
                    hs.append(ch["h"])
                    owner.append(I)
        if not cols:
            return np.zeros((self.npw, 0), dtype=complex), np.zeros(0), np.zeros(0, int)
        return np.array(cols).T, np.array(hs), np.array(owner)

    def to_grid(self, C):
        b = self.base
        nb = C.shape[1]
        box = np.zeros((nb, b.ntot), dtype=complex)
        box[:, self.box] = C.T
        return np.fft.ifftn(box.reshape((nb,) + b.grid), axes=(1, 2, 3)) * b.ntot

    def from_grid(self, W):
        b = self.base
        F = np.fft.fftn(W, axes=(1, 2, 3)).reshape(W.shape[0], b.ntot) / b.ntot
        return F[:, self.box].T

    def apply_h(self, veff, C):
        out = self.kin[:, None] * C + self.from_grid(veff[None] * self.to_grid(C))
        if self.beta.shape[1]:
            out += self.beta @ (self.h[:, None] * (self.beta.conj().T @ C))
        return out

    def dense_h(self, veff):
        b = self.base
        Vt = np.fft.fftn(veff) / b.ntot
        m = self.millers
        d = m[:, None, :] - m[None, :, :]
        idx = ((np.mod(d[..., 0], b.grid[0]) * b.grid[1] + np.mod(d[..., 1], b.grid[1])) * b.grid[2]
               + np.mod(d[..., 2], b.grid[2]))
        H = Vt.reshape(-1)[idx]
        H[np.diag_indices(self.npw)] += self.kin
        if self.beta.shape[1]:
            H += (self.beta * self.h[None, :]) @ self.beta.conj().T
        return H

    def density(self, C, f):
        u = self.to_grid(C)
        return np.einsum("i,ixyz->xyz", f, np.abs(u) ** 2) / self.base.omega


def occupations_k(eps, weights, nelec, occ):
    """Occupations f[k][n] in [0, 2] and the entropy sum_k w_k S_k."""
    eps = [np.asarray(e, dtype=float) for e in eps]
    w = np.asarray(weights, dtype=float)
    if occ["kind"] == "fixed":
        nocc = int(round(nelec / 2))
        if abs(nocc * 2 - nelec) > 1e-9 or nocc > len(eps[0]):
            raise ValueError("fixed occupations need an even electron count <= 2 nbands")
        f = []
        for e in eps:
            fk = np.zeros(len(e))
            fk[np.argsort(e)[:nocc]] = 2.0
            f.append(fk)
        mu = 0.5 * (max(e[np.argsort(e)[nocc - 1]] for e in eps)
                    + min(e[np.argsort(e)[nocc]] if nocc < len(e) else e.max() for e in eps))
        return f, mu, 0.0
    sigma = float(occ["sigma"])
    allv = np.concatenate(eps)
    lo, hi = allv.min() - 40 * sigma, allv.max() + 40 * sigma
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        n = sum(wk * (2 * expit(-(e - mu) / sigma)).sum() for wk, e in zip(w, eps))
        if n > nelec:
            hi = mu
        else:
            lo = mu
    mu = 0.5 * (lo + hi)
    f, S = [], 0.0
    for wk, e in zip(w, eps):
        fk = 2 * expit(-(e - mu) / sigma)
        g = np.clip(fk / 2, 1e-300, 1.0)
        gm = np.clip(1 - fk / 2, 1e-300, 1.0)
        S += wk * (-2 * (g * np.log(g) + gm * np.log(gm)).sum())
        f.append(fk)
    return f, mu, S


def run_scf_k(system, kpts, weights, tol_e=1e-10, tol_rho=1e-9, maxiter=200, mix_alpha=0.5,
              kerker_q0=0.8, history=8, verbose=False):
    """Self-consistent solve with the k-points kpts (rows, units of the
    reciprocal basis vectors) and weights (normalised here).  Each k is
    diagonalised densely.  Same Pulay/Kerker mixing and stopping rule as
    the Gamma-point oracle."""
    base = Setup(system)
    w = np.asarray(weights, dtype=float)
    w = w / w.sum()
    ks = [KSetup(base, k) for k in kpts]
    occ = system["occupation"]
    sigma = float(occ.get("sigma", 0.0))
    nb = base.nbands
    rho_in = base.initial_density()
    g2 = base.g2grid
    kerker = np.where(g2 > 0, g2 / (g2 + kerker_q0 ** 2), 0.0)
    hist_in, hist_res = [], []
    e_prev = None
    for it in range(1, maxiter + 1):
        veff, _ = potentials(base, rho_in)
        eps, Cs = [], []
        for kst in ks:
            e, V = scipy.linalg.eigh(kst.dense_h(veff), subset_by_index=[0, nb - 1])
            eps.append(e)
            Cs.append(V)
        f, mu, S = occupations_k(eps, w, base.nelec, occ)
        rho_out = sum(wk * kst.density(C, fk) for wk, kst, C, fk in zip(w, ks, Cs, f))
        terms = energy_terms_k(base, ks, w, Cs, f, rho_out, S, sigma)
        e = terms["total"]
        R = rho_out - rho_in
        drho = base.omega / base.ntot * np.abs(R).sum() / max(base.nelec, 1e-30)
        de = abs(e - e_prev) if e_prev is not None else np.inf
        if verbose:
            print("oracle k scf %3d  E=%.12f  dE=%.2e  drho=%.2e" % (it, e, de, drho))
        if de < tol_e and drho < tol_rho:
            break
        e_prev = e
        hist_in.append(rho_in.copy())
        hist_res.append(R.copy())
        if len(hist_in) > history:
            hist_in.pop(0)
            hist_res.pop(0)
        n = len(hist_in)
        A = np.array([[np.vdot(hist_res[i], hist_res[j]).real for j in range(n)] for i in range(n)])
        scale = np.abs(np.diag(A)).max() or 1.0
        M = np.zeros((n + 1, n + 1))
        M[:n, :n] = A / scale
        M[:n, n] = 1.0
        M[n, :n] = 1.0
        rhs = np.zeros(n + 1)
        rhs[n] = 1.0
        coef = np.linalg.lstsq(M, rhs, rcond=None)[0][:n]
        r_opt = sum(c * r for c, r in zip(coef, hist_res))
        rho_opt = sum(c * r for c, r in zip(coef, hist_in))
        rho_in = rho_opt + mix_alpha * np.real(np.fft.ifftn(kerker * np.fft.fftn(r_opt)))
    else:
        raise RuntimeError("oracle k-point SCF did not converge in %d iterations" % maxiter)
    return {"setup": base, "ksetups": ks, "weights": w, "energy": e, "terms": terms,
            "eigenvalues": eps, "occupations": f, "mu": mu, "entropy": S, "rho": rho_out,
            "rho_in": rho_in, "C": Cs, "iterations": it}


def energy_terms_k(base, ks, w, Cs, f, rho_out, S, sigma):
    """Energy terms: the k sums of the band terms, the grid terms of the
    Gamma oracle from the density."""
    grid = energy_terms(base, np.zeros((base.npw, 0), complex), np.zeros(0), rho_out, S, sigma)
    e_kin = sum(wk * float((fk * (kst.kin[:, None] * np.abs(C) ** 2).sum(0)).sum())
                for wk, kst, C, fk in zip(w, ks, Cs, f))
    e_nl = 0.0
    for wk, kst, C, fk in zip(w, ks, Cs, f):
        if kst.beta.shape[1]:
            P = kst.beta.conj().T @ C
            e_nl += wk * float((fk[None, :] * kst.h[:, None] * np.abs(P) ** 2).sum())
    terms = dict(grid)
    terms["kinetic"] = e_kin
    terms["nonlocal"] = e_nl
    terms["total"] = sum(terms[k] for k in ("kinetic", "nonlocal", "local", "hartree", "xc",
                                             "ewald", "entropy"))
    return terms


def hf_forces_k(res):
    """Hellmann-Feynman forces: local part from rho (as at Gamma), nonlocal
    part summed over k with the phase derivative -i (k + G), Ewald."""
    base = res["setup"]
    rhoG = np.fft.fftn(res["rho"]) / base.ntot
    nz = base.dmask & (base.g2grid > 0)
    Gd = base.Ggrid[nz]
    g = np.sqrt(base.g2grid[nz])
    rg = rhoG[nz]
    F_loc = np.zeros((base.nat, 3))
    for I, s in enumerate(base.symbols):
        sp = base.species[s]
        v = local_ft(sp["local"], sp["Z"], g)
        z = v * np.exp(1j * (Gd @ base.pos[I])) * rg
        F_loc[I] = (Gd * np.imag(z)[:, None]).sum(0)
    F_nl = np.zeros((base.nat, 3))
    for wk, kst, C, fk in zip(res["weights"], res["ksetups"], res["C"], res["occupations"]):
        if not kst.beta.shape[1]:
            continue
        P = kst.beta.conj().T @ C
        for a in range(3):
            dP = (-1j * kst.q[:, a][:, None] * kst.beta).conj().T @ C
            contrib = -2 * wk * (fk[None, :] * kst.h[:, None] * np.real(np.conj(P) * dP)).sum(1)
            np.add.at(F_nl[:, a], kst.proj_atom, contrib)
    return F_loc + F_nl + base.f_ewald, {"local": F_loc, "nonlocal": F_nl,
                                         "ewald": base.f_ewald.copy()}


def monkhorst_pack(n):
    """Monkhorst-Pack mesh n[0] x n[1] x n[2] (fractional k, equal weights):
    k_i = (2 r_i - n_i - 1) / (2 n_i), r_i = 1..n_i."""
    axes = [(2 * np.arange(1, m + 1) - m - 1) / (2.0 * m) for m in n]
    k = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return k, np.full(len(k), 1.0 / len(k))
