"""Pins of the oracle's Hamiltonian: empty-lattice eigenvalues and
degeneracies, constant-potential shift, the FFT operator against a dense
matrix whose potential coefficients are explicit brute-force Fourier sums,
Hermitian and time-reversal structure, and dense against iterative
diagonalisation."""
import numpy as np
import pytest

from oracle.hamiltonian import Setup
from oracle.scf import eigensolve
from workloads import make_system, tiny_system


def _empty(a=7.0, ecut=4.0, grid=(16, 16, 16), nb=40):
    return make_system("empty", np.eye(3) * a, [], np.zeros((0, 3)), ecut, grid, nb,
                       {"kind": "fixed"})


def test_empty_lattice_levels():
    a = 7.0
    st = Setup(_empty(a))
    w, _ = eigensolve(st, np.zeros(st.grid), 33)
    unit = 0.5 * (2 * np.pi / a) ** 2
    # |m|^2 = 0, 1, 2, 3, 4 with multiplicities 1, 6, 12, 8, 6
    expect = np.repeat([0, 1, 2, 3, 4], [1, 6, 12, 8, 6]) * unit
    assert np.abs(w - expect).max() < 1e-12


def test_constant_potential_shift():
    st = Setup(_empty())
    w0, _ = eigensolve(st, np.zeros(st.grid), 27)
    w1, _ = eigensolve(st, np.full(st.grid, -0.37), 27)
    assert np.abs(w1 - w0 + 0.37).max() < 1e-12


def test_fft_operator_equals_bruteforce_dense_matrix():
    # tiny grid so the Fourier coefficients can be summed explicitly
    sysd = tiny_system("sip", ecut=1.2, grid=(7, 8, 9), nbands=4)
    st = Setup(sysd)
    rng = np.random.default_rng(3)
    V = rng.standard_normal(st.grid)
    N1, N2, N3 = st.grid
    n = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"), -1)
    m = st.millers
    H = np.zeros((st.npw, st.npw), dtype=complex)
    for i in range(st.npw):
        d = m[i] - m  # (npw,3)
        ph = np.exp(-2j * np.pi * (n[..., 0, None] * d[:, 0] / N1 + n[..., 1, None] * d[:, 1] / N2
                                   + n[..., 2, None] * d[:, 2] / N3))
        H[i] = (V[..., None] * ph).sum((0, 1, 2)) / (N1 * N2 * N3)
    H[np.diag_indices(st.npw)] += st.kin
    H += (st.beta * st.h[None, :]) @ st.beta.conj().T
    assert np.abs(H - st.dense_h(V)).max() < 1e-12
    C = rng.standard_normal((st.npw, 3)) + 1j * rng.standard_normal((st.npw, 3))
    assert np.abs(H @ C - st.apply_h(V, C)).max() < 1e-11


def test_hermitian_and_time_reversal():
    st = Setup(tiny_system("sip", ecut=2.0, grid=(12, 12, 12)))
    V = np.random.default_rng(5).standard_normal(st.grid)
    H = st.dense_h(V)
    assert np.abs(H - H.conj().T).max() < 1e-13
    # real potential and real projectors in r: H(-G,-G') = conj H(G,G')
    m = st.millers
    key = {tuple(x): i for i, x in enumerate(m)}
    neg = np.array([key[tuple(-x)] for x in m])
    assert np.abs(H[np.ix_(neg, neg)] - H.conj()).max() < 1e-13


def test_dense_equals_iterative():
    st = Setup(tiny_system("sip", ecut=3.0, grid=(12, 12, 12)))
    V = 0.3 * np.random.default_rng(8).standard_normal(st.grid)
    wd, Vd = eigensolve(st, V, 12)
    wi, Vi = eigensolve(st, V, 12, dense_max=0, tol=1e-9)
    assert np.abs(wd - wi).max() < 1e-10
    # invariant subspaces agree (compare projectors, not vectors)
    Pd = Vd[:, :8] @ Vd[:, :8].conj().T
    Pi = Vi[:, :8] @ Vi[:, :8].conj().T
    assert np.abs(Pd - Pi).max() < 1e-7
