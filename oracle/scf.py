"""Self-consistent field loop (oracle).

One SCF step (the loop of Section 2.4: rho_in -> solve the Kohn-Sham
equation -> rho_out -> mix):
  V_eff = V_loc + V_H[rho_in] + v_xc[rho_in]
  solve H[V_eff] psi_i = eps_i psi_i for the lowest nbands states
      (dense eigh of the full complex H where it fits, else LOBPCG to a
       tight residual; the result is the same fixed point either way)
  occupations: fixed (2 per band) or Fermi-Dirac f_i = 2/(1+e^{(eps_i-mu)/sigma})
  rho_out = sum_i f_i |psi_i|^2;  energy E[psi, rho_out]
  Pulay (DIIS) mixing of rho with a Kerker filter G^2/(G^2+q0^2).
Stops when successive free energies differ by < tol_e and
Omega/Ntot sum|rho_out - rho_in| / N_el < tol_rho.

Energy terms (Mermin free energy F = E - sigma S for Fermi-Dirac):
  E_kin = sum_i f_i sum_G |G|^2/2 |c_iG|^2
  E_nl  = sum_i f_i sum_p h_p |<beta_p|psi_i>|^2
  E_loc = Omega sum_{G in D} V_loc(G)* rho(G)
  E_H   = (Omega/2) sum_{G in D, G != 0} 4 pi |rho(G)|^2 / G^2
  E_xc  = (Omega/Ntot) sum_n rho_n eps_xc(rho_n)
  E_ion = Ewald
  S     = -2 sum_i [g ln g + (1-g) ln(1-g)],  g = f_i/2
"""
import warnings

import numpy as np
import scipy.linalg
from scipy.special import expit

from .hamiltonian import Setup
from .lda import pz81


def potentials(st, rho):
    """V_eff(r) and its parts from a grid density rho_in."""
    rhoG = np.fft.fftn(rho) / st.ntot
    vh_G = np.zeros(st.grid, dtype=complex)
    nz = st.dmask & (st.g2grid > 0)
    vh_G[nz] = 4 * np.pi * rhoG[nz] / st.g2grid[nz]
    vh = np.real(np.fft.ifftn(vh_G)) * st.ntot
    _, vxc = pz81(np.maximum(rho, 0.0))
    vloc = st.vloc_r()
    return vloc + vh + vxc, {"vloc": vloc, "vh": vh, "vxc": vxc}


def occupations(eps, nelec, occ):
    eps = np.asarray(eps, dtype=float)
    if occ["kind"] == "fixed":
        nocc = int(round(nelec / 2))
        if abs(nocc * 2 - nelec) > 1e-9 or nocc > len(eps):
            raise ValueError("fixed occupations need an even electron count <= 2 nbands")
        f = np.zeros(len(eps))
        f[:nocc] = 2.0
        mu = 0.5 * (eps[nocc - 1] + eps[nocc]) if nocc < len(eps) else eps[-1]
        return f, mu, 0.0
    sigma = float(occ["sigma"])
    lo, hi = eps.min() - 40 * sigma, eps.max() + 40 * sigma
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        n = (2 * expit(-(eps - mu) / sigma)).sum()
        if n > nelec:
            hi = mu
        else:
            lo = mu
    mu = 0.5 * (lo + hi)
    f = 2 * expit(-(eps - mu) / sigma)
    g = np.clip(f / 2, 1e-300, 1.0)
    gm = np.clip(1 - f / 2, 1e-300, 1.0)
    S = -2 * (g * np.log(g) + gm * np.log(gm)).sum()
    return f, mu, S


def energy_terms(st, C, f, rho_out, S=0.0, sigma=0.0):
    e_kin = float((f * (st.kin[:, None] * np.abs(C) ** 2).sum(0)).sum())
    if st.beta.shape[1]:
        P = st.beta.conj().T @ C
        e_nl = float((f[None, :] * st.h[:, None] * np.abs(P) ** 2).sum())
    else:
        e_nl = 0.0
    rhoG = np.fft.fftn(rho_out) / st.ntot
    e_loc = float(st.omega * np.real(np.conj(st.vloc_G[st.dmask]) * rhoG[st.dmask]).sum())
    nz = st.dmask & (st.g2grid > 0)
    e_h = float(0.5 * st.omega * (4 * np.pi * np.abs(rhoG[nz]) ** 2 / st.g2grid[nz]).sum())
    rc = np.maximum(rho_out, 0.0)
    exc, _ = pz81(rc)
    e_xc = float(st.omega / st.ntot * (rc * exc).sum())
    terms = {"kinetic": e_kin, "nonlocal": e_nl, "local": e_loc, "hartree": e_h,
             "xc": e_xc, "ewald": float(st.e_ewald), "entropy": float(-sigma * S)}
    terms["total"] = sum(terms.values())
    return terms


def eigensolve(st, veff, nb, X0=None, dense_max=3000, tol=1e-8, maxiter=400):
    """Lowest nb eigenpairs of H[V_eff] (ascending)."""
    if st.npw <= dense_max:
        H = st.dense_h(veff)
        w, V = scipy.linalg.eigh(H, subset_by_index=[0, nb - 1])
        return w, V
    from scipy.sparse.linalg import LinearOperator, lobpcg
    op = LinearOperator((st.npw, st.npw), matvec=lambda v: st.apply_h(veff, v.reshape(-1, 1)).ravel(),
                        matmat=lambda V: st.apply_h(veff, V), dtype=complex)
    if X0 is None:
        rng = np.random.default_rng(12345)
        X0 = (rng.standard_normal((st.npw, nb)) + 1j * rng.standard_normal((st.npw, nb)))
        X0 /= (1 + st.kin)[:, None]
    X = X0
    prec = 1.0 / (1.0 + st.kin)
    M = LinearOperator((st.npw, st.npw), dtype=complex,
                       matvec=lambda r: prec * r.ravel(),
                       matmat=lambda R: prec[:, None] * R)
    res = np.inf
    for attempt in range(6):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            w, V = lobpcg(op, X, largest=False, tol=tol, maxiter=maxiter, M=M)
        order = np.argsort(w)
        w, V = w[order], V[:, order]
        # orthonormalise and Rayleigh-Ritz once more for a clean subspace
        Q, _ = np.linalg.qr(V)
        HQ = st.apply_h(veff, Q)
        hs = Q.conj().T @ HQ
        ws, U = np.linalg.eigh(0.5 * (hs + hs.conj().T))
        V = Q @ U
        w = ws
        res = np.linalg.norm(HQ @ U - V * w[None, :], axis=0).max()
        if res < 10 * tol:
            return w, V
        X = V
    raise RuntimeError("oracle eigensolver did not converge (residual %.2e)" % res)


def run_scf(system, tol_e=1e-10, tol_rho=1e-9, maxiter=200, mix_alpha=0.5,
            kerker_q0=0.8, history=8, dense_max=3000, verbose=False, setup=None,
            rho0=None, stop_after=None):
    """Self-consistent solve.  stop_after=k returns after k iterations
    without raising (used only to time a bounded sample)."""
    st = setup if setup is not None else Setup(system)
    occ = system["occupation"]
    sigma = float(occ.get("sigma", 0.0))
    nb = st.nbands
    rho_in = st.initial_density() if rho0 is None else rho0.copy()
    g2full = st.g2grid
    kerker = np.where(g2full > 0, g2full / (g2full + kerker_q0 ** 2), 0.0)
    hist_in, hist_res = [], []
    e_prev = None
    X = None
    info = {}
    trace = []
    import time as _time
    t_start = _time.perf_counter()
    for it in range(1, maxiter + 1):
        veff, _ = potentials(st, rho_in)
        eps, C = eigensolve(st, veff, nb, X0=X, dense_max=dense_max)
        X = C
        f, mu, S = occupations(eps, st.nelec, occ)
        rho_out = st.density(C, f)
        terms = energy_terms(st, C, f, rho_out, S, sigma)
        e = terms["total"]
        R = rho_out - rho_in
        drho = st.omega / st.ntot * np.abs(R).sum() / max(st.nelec, 1e-30)
        de = abs(e - e_prev) if e_prev is not None else np.inf
        trace.append((e, de, drho, _time.perf_counter() - t_start))
        if verbose:
            print("oracle scf %3d  E=%.12f  dE=%.2e  drho=%.2e" % (it, e, de, drho))
        if (de < tol_e and drho < tol_rho) or (stop_after is not None and it >= stop_after):
            info = {"iterations": it, "drho": drho, "de": de, "trace": trace}
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
        KR = np.real(np.fft.ifftn(kerker * np.fft.fftn(r_opt)))
        rho_in = rho_opt + mix_alpha * KR
    else:
        raise RuntimeError("oracle SCF did not converge in %d iterations" % maxiter)
    return {"setup": st, "energy": e, "terms": terms, "eigenvalues": eps,
            "occupations": f, "mu": mu, "entropy": S, "rho": rho_out, "rho_in": rho_in,
            "C": C, "info": info}
