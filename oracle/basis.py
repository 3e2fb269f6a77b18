"""Plane-wave basis and FFT-grid bookkeeping (oracle).

Conventions (Hartree atomic units):
  lattice rows a_i; Omega = |det A|; reciprocal rows b_i = 2 pi (A^-1)^T.
  G = sum_i m_i b_i.  Grid point n = (n1,n2,n3) sits at r_n = sum_i n_i/N_i a_i.
  psi(r_n) = Omega^-1/2 sum_G c_G exp(2 pi i m.n/N)   (so sum |c|^2 = 1),
  rho(G)   = (1/Ntot) sum_n rho(r_n) exp(-2 pi i m.n/N).
The wavefunction basis is the full sphere |G|^2/2 <= Ecut.  The density
set D holds every grid frequency with |m_i| < N_i/2 (Nyquist planes are
excluded so that potentials built from D stay real).
"""
import numpy as np


def cell_geometry(lattice):
    A = np.asarray(lattice, dtype=float)
    omega = abs(np.linalg.det(A))
    B = 2.0 * np.pi * np.linalg.inv(A).T
    return omega, B


def sphere_millers(lattice, ecut):
    """Every integer triple m with |m B|^2 / 2 <= ecut (full sphere)."""
    A = np.asarray(lattice, dtype=float)
    _, B = cell_geometry(A)
    gmax = np.sqrt(2.0 * ecut)
    # m_i = G . a_i / (2 pi), so |m_i| <= gmax |a_i| / (2 pi)
    mmax = [int(np.floor(gmax * np.linalg.norm(A[i]) / (2 * np.pi))) + 1 for i in range(3)]
    r = [np.arange(-mm, mm + 1) for mm in mmax]
    m = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    G = m @ B
    keep = 0.5 * (G * G).sum(1) <= ecut
    return m[keep]


def grid_frequencies(grid):
    """Integer frequency of every grid index along each axis, in [-N/2, N/2)."""
    return [np.fft.fftfreq(n, 1.0 / n).round().astype(int) for n in grid]


def grid_gvectors(lattice, grid):
    """G vectors (N1,N2,N3,3) of every grid frequency and the mask of D."""
    _, B = cell_geometry(lattice)
    f = grid_frequencies(grid)
    m = np.stack(np.meshgrid(*f, indexing="ij"), axis=-1)
    G = m @ B
    mask = np.ones(tuple(grid), dtype=bool)
    for ax in range(3):
        n = grid[ax]
        ok = np.abs(f[ax]) * 2 < n
        shape = [1, 1, 1]
        shape[ax] = n
        mask &= ok.reshape(shape)
    return G, mask


def box_index(millers, grid):
    """Flat index of each Miller triple in the (N1,N2,N3) FFT box (m mod N)."""
    m = np.asarray(millers)
    i = np.mod(m[:, 0], grid[0])
    j = np.mod(m[:, 1], grid[1])
    k = np.mod(m[:, 2], grid[2])
    return (i * grid[1] + j) * grid[2] + k


def check_grid(millers, grid):
    """The grid must hold the wavefunction sphere: N_i >= 2 max|m_i| + 1."""
    mm = np.abs(np.asarray(millers)).max(0)
    return all(grid[i] >= 2 * mm[i] + 1 for i in range(3))
