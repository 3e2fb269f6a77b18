"""Kohn-Sham Hamiltonian on the full complex plane-wave sphere (oracle).

(H psi)_G = |G|^2/2 c_G + (1/Ntot) FFT[V_eff(r_n) u(r_n)]_G + sum_p beta_p(G) h_p <beta_p|psi>
with u(r_n) = sum_G c_G e^{iG.r_n}.  The dense matrix of the same operator is
H_GG' = |G|^2/2 delta + V~((m - m') mod N) + sum_p beta_p(G) h_p beta_p(G')*,
V~(m) = (1/Ntot) sum_n V_eff(r_n) e^{-2 pi i m.n/N} (a circulant identity, so
the two agree to rounding even where the product aliases).
"""
import numpy as np

from .basis import (cell_geometry, sphere_millers, grid_gvectors, box_index,
                    check_grid)
from .pseudo import local_ft, local_g0, projector_ft, real_ylm
from .ewald import ewald


class Setup:
    """Everything that depends on geometry only."""

    def __init__(self, system, ewald_eta=None):
        self.system = system
        self.lattice = np.asarray(system["lattice"], dtype=float)
        self.grid = tuple(int(g) for g in system["grid"])
        self.ntot = int(np.prod(self.grid))
        self.omega, self.B = cell_geometry(self.lattice)
        self.pos = np.asarray(system["positions"], dtype=float).reshape(-1, 3)
        self.symbols = list(system["symbols"])
        self.species = system["species"]
        self.nat = len(self.symbols)
        self.Z = np.array([self.species[s]["Z"] for s in self.symbols], dtype=float)
        self.nelec = float(system["nelec"])
        self.nbands = int(system["nbands"])
        self.ecut = float(system["ecut"])
        # a fixed Miller set (system["millers"]) keeps the basis of a strained
        # cell identical to that of the reference cell
        if system.get("millers") is not None:
            self.millers = np.asarray(system["millers"], dtype=int).reshape(-1, 3)
        else:
            self.millers = sphere_millers(self.lattice, self.ecut)
        if not check_grid(self.millers, self.grid):
            raise ValueError("grid too small for the wavefunction sphere")
        self.G = self.millers @ self.B
        self.g2 = (self.G * self.G).sum(1)
        self.kin = 0.5 * self.g2
        self.npw = len(self.millers)
        self.box = box_index(self.millers, self.grid)
        # density set D on the grid
        self.Ggrid, self.dmask = grid_gvectors(self.lattice, self.grid)
        self.g2grid = (self.Ggrid * self.Ggrid).sum(-1)
        self.vloc_G = self._vloc_G()
        self.beta, self.h, self.proj_atom = self._projectors()
        self.e_ewald, self.f_ewald = ewald(self.lattice, self.Z, self.pos, eta=ewald_eta)

    # ---- local potential V_loc(G) on D, zero elsewhere -------------------
    def _vloc_G(self):
        V = np.zeros(self.grid, dtype=complex)
        Gd = self.Ggrid[self.dmask]
        g = np.sqrt(self.g2grid[self.dmask])
        nz = g > 0
        acc = np.zeros(len(Gd), dtype=complex)
        for s in sorted(set(self.symbols)):
            sp = self.species[s]
            idx = [i for i, t in enumerate(self.symbols) if t == s]
            Sf = np.exp(-1j * (Gd @ self.pos[idx].T)).sum(1)  # structure factor
            vs = np.zeros(len(Gd))
            vs[nz] = local_ft(sp["local"], sp["Z"], g[nz])
            vs[~nz] = local_g0(sp["local"], sp["Z"])
            acc += vs * Sf
        V[self.dmask] = acc / self.omega
        return V

    def vloc_r(self):
        return np.real(np.fft.ifftn(self.vloc_G)) * self.ntot

    # ---- Kleinman-Bylander projectors ------------------------------------
    def _projectors(self):
        cols, hs, owner = [], [], []
        g = np.sqrt(self.g2)
        for I, s in enumerate(self.symbols):
            phase = np.exp(-1j * (self.G @ self.pos[I]))
            for ch in self.species[s]["kb"]:
                l = ch["l"]
                radial = projector_ft(l, ch["r"], g)
                Y = real_ylm(l, self.G)
                for mm in range(Y.shape[0]):
                    cols.append(radial * (-1j) ** l * Y[mm] * phase / np.sqrt(self.omega))
                    hs.append(ch["h"])
                    owner.append(I)
        if not cols:
            return np.zeros((self.npw, 0), dtype=complex), np.zeros(0), np.zeros(0, int)
        return np.array(cols).T, np.array(hs), np.array(owner)

    # ---- transforms -----------------------------------------------------
    def to_grid(self, C):
        """u_i(r_n) = sum_G c_iG e^{iG.r_n} for columns of C (npw, nb) -> (nb, N1,N2,N3)."""
        nb = C.shape[1]
        box = np.zeros((nb, self.ntot), dtype=complex)
        box[:, self.box] = C.T
        box = box.reshape((nb,) + self.grid)
        return np.fft.ifftn(box, axes=(1, 2, 3)) * self.ntot

    def from_grid(self, W):
        """(1/Ntot) sum_n w(r_n) e^{-iG.r_n} on the sphere -> (npw, nb)."""
        nb = W.shape[0]
        F = np.fft.fftn(W, axes=(1, 2, 3)).reshape(nb, self.ntot) / self.ntot
        return F[:, self.box].T

    def apply_h(self, veff_r, C, chunk=64):
        out = np.empty_like(C)
        for s in range(0, C.shape[1], chunk):
            c = C[:, s:s + chunk]
            u = self.to_grid(c)
            out[:, s:s + chunk] = self.kin[:, None] * c + self.from_grid(veff_r[None] * u)
        if self.beta.shape[1]:
            P = self.beta.conj().T @ C
            out += self.beta @ (self.h[:, None] * P)
        return out

    def dense_h(self, veff_r):
        Vt = np.fft.fftn(veff_r) / self.ntot
        m = self.millers
        d = m[:, None, :] - m[None, :, :]
        idx = ((np.mod(d[..., 0], self.grid[0]) * self.grid[1]
                + np.mod(d[..., 1], self.grid[1])) * self.grid[2]
               + np.mod(d[..., 2], self.grid[2]))
        H = Vt.reshape(-1)[idx]
        H[np.diag_indices(self.npw)] += self.kin
        if self.beta.shape[1]:
            H += (self.beta * self.h[None, :]) @ self.beta.conj().T
        return H

    def density(self, C, f, chunk=64):
        """rho(r_n) = sum_i f_i |u_i(r_n)|^2 / Omega."""
        rho = np.zeros(self.grid)
        for s in range(0, C.shape[1], chunk):
            u = self.to_grid(C[:, s:s + chunk])
            rho += np.einsum("i,ixyz->xyz", f[s:s + chunk], np.abs(u) ** 2)
        return rho / self.omega

    def initial_density(self):
        """Superposition of normalised Gaussians of charge Z (width rho0_width)
        synthesised from the set D, plus a uniform part carrying any electrons
        not balanced by ionic charge, so that it integrates to N_el exactly."""
        R = np.zeros(self.grid, dtype=complex)
        Gd = self.Ggrid[self.dmask]
        g2 = self.g2grid[self.dmask]
        acc = np.zeros(len(Gd), dtype=complex)
        for I, s in enumerate(self.symbols):
            w = self.species[s]["rho0_width"]
            acc += self.Z[I] * np.exp(-0.5 * g2 * w * w) * np.exp(-1j * (Gd @ self.pos[I]))
        R[self.dmask] = acc / self.omega
        R[0, 0, 0] += (self.nelec - self.Z.sum()) / self.omega
        return np.real(np.fft.ifftn(R)) * self.ntot
