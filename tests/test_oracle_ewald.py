"""Pins of the oracle's Ewald sum against textbook Madelung constants, eta
independence, Newton's third law and finite differences."""
import numpy as np
import pytest

from oracle.ewald import ewald

FCC = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=float)


def test_nacl_madelung():
    # rock salt: energy per ion pair = -M / r_nn, M = 1.747565 (r_nn = a/2)
    a = 2.7
    pos = np.vstack([FCC, FCC + [0.5, 0, 0]]) * a
    E, F = ewald(np.eye(3) * a, [1] * 4 + [-1] * 4, pos)
    assert abs(-E / 4 * (a / 2) - 1.747565) < 2e-6
    assert np.abs(F).max() < 1e-12


def test_cscl_madelung():
    a = 3.1
    E, F = ewald(np.eye(3) * a, [1, -1], [[0, 0, 0], [a / 2] * 3])
    assert abs(-E * (a * np.sqrt(3) / 2) - 1.762675) < 2e-6


def test_zincblende_madelung():
    a = 5.0
    pos = np.vstack([FCC, FCC + 0.25]) * a
    E, F = ewald(np.eye(3) * a, [1] * 4 + [-1] * 4, pos)
    assert abs(-E / 4 * (a * np.sqrt(3) / 4) - 1.638055) < 2e-6


@pytest.mark.parametrize("basis,per_cell,const", [
    ([[0, 0, 0], [.5, .5, .5]], 2, -0.895929),   # bcc
    (FCC.tolist(), 4, -0.895874),                 # fcc
    ([[0, 0, 0]], 1, -0.880059),                  # simple cubic
])
def test_one_component_plasma(basis, per_cell, const):
    # unit charges in a neutralising background: E per ion = const / r_s
    a = 4.0
    E, _ = ewald(np.eye(3) * a, [1] * per_cell, np.array(basis) * a)
    rs = (3 * a ** 3 / per_cell / (4 * np.pi)) ** (1 / 3)
    assert abs(E / per_cell * rs - const) < 2e-6


def _random_cell(seed, nat=5):
    rng = np.random.default_rng(seed)
    A = np.diag(rng.uniform(6, 9, 3)) + rng.uniform(-1, 1, (3, 3))
    pos = rng.uniform(0, 1, (nat, 3)) @ A
    Z = rng.choice([1.0, 2.0, 4.0], nat)
    return A, Z, pos


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_eta_independence_and_newton(seed):
    A, Z, pos = _random_cell(seed)
    E1, F1 = ewald(A, Z, pos, eta=0.35)
    E2, F2 = ewald(A, Z, pos, eta=0.9)
    assert abs(E1 - E2) < 1e-10 * max(1, abs(E1))
    assert np.abs(F1 - F2).max() < 1e-10
    assert np.abs(F1.sum(0)).max() < 1e-12 * max(1, np.abs(F1).max()) * 100


def test_forces_match_energy_differences():
    A, Z, pos = _random_cell(7)
    _, F = ewald(A, Z, pos)
    h = 1e-4
    for I, a in [(0, 0), (2, 1), (4, 2)]:
        p1, p2 = pos.copy(), pos.copy()
        p1[I, a] += h
        p2[I, a] -= h
        fd = -(ewald(A, Z, p1)[0] - ewald(A, Z, p2)[0]) / (2 * h)
        assert abs(fd - F[I, a]) < 1e-7


def test_stress_matches_strain_differences():
    A, Z, pos = _random_cell(9)
    omega = abs(np.linalg.det(A))
    _, _, S = ewald(A, Z, pos, want_stress=True)
    h = 1e-5
    for a, b in [(0, 0), (1, 2), (2, 2), (0, 1)]:
        eps = np.zeros((3, 3))
        eps[a, b] = eps[b, a] = h / (2 if a != b else 1)
        Ep = ewald(A @ (np.eye(3) + eps).T, Z, pos @ (np.eye(3) + eps).T)[0]
        Em = ewald(A @ (np.eye(3) - eps).T, Z, pos @ (np.eye(3) - eps).T)[0]
        fd = (Ep - Em) / (2 * h) / omega
        assert abs(fd - S[a, b]) < 1e-7
