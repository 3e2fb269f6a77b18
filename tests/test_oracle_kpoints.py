"""Pins of the oracle's k-point sampling (the "rough K-points" that Section
2.3 allows for the DFT level): empty-lattice levels at a zone-boundary k in
closed form, a constant potential's shift, time reversal eps(k) = eps(-k),
periodicity in the reciprocal lattice, k = 0 against the Gamma-point oracle,
a primitive cell sampled at k = 0 and b1/2 against the doubled supercell at
Gamma (energy and forces: the folding identity exercises the k + G kinetic
and projector terms, the k-weighted density and the occupations), and a
central finite-difference force at k != 0."""
import copy

import numpy as np
import pytest

from oracle.hamiltonian import Setup
from oracle.kpoints import KSetup, run_scf_k, hf_forces_k, monkhorst_pack
from oracle.scf import run_scf
from oracle.forces import hf_forces
from workloads import make_system, tiny_system

FIXED = {"kind": "fixed"}


def _empty_box(a, ecut, grid):
    s = make_system("empty", np.eye(3) * a, [], np.zeros((0, 3)), ecut, grid, 28, FIXED)
    s["nelec"] = 0.0
    return s


def test_empty_lattice_levels_at_the_zone_boundary():
    # k = b1/2: |k + G|^2 = (2 pi/a)^2 [(m1 + 1/2)^2 + m2^2 + m3^2]; the lowest
    # values in units of (2 pi/a)^2 / 2 and their counts:
    # 1/4 (m1 in {0,-1}): 2;  1/4 + 1: 2 x 4 = 8;  1/4 + 2 (2 x 4) and 9/4 + 0 (2): 10;
    # 9/4 + 1: 2 x 4 = 8
    a = 8.0
    base = Setup(_empty_box(a, 2.5, (16, 16, 16)))
    ks = KSetup(base, (0.5, 0.0, 0.0))
    unit = 0.5 * (2 * np.pi / a) ** 2
    expect = unit * np.array([0.25] * 2 + [1.25] * 8 + [2.25] * 10 + [3.25] * 8)
    eps = np.linalg.eigvalsh(ks.dense_h(np.zeros(base.grid)))[:28]
    assert np.abs(eps - expect).max() < 1e-12
    # a constant potential V0 shifts every level by V0
    eps2 = np.linalg.eigvalsh(ks.dense_h(np.full(base.grid, -0.37)))[:28]
    assert np.abs(eps2 - (expect - 0.37)).max() < 1e-12


@pytest.fixture(scope="module")
def sip():
    s = tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    base = Setup(s)
    veff = np.real(np.fft.ifftn(np.fft.fftn(base.initial_density())))  # any real lattice-periodic V
    return s, base, 0.3 * veff - 0.1


def test_time_reversal_and_reciprocal_periodicity(sip):
    s, base, veff = sip
    k = np.array([0.21, -0.13, 0.37])
    e = np.linalg.eigvalsh(KSetup(base, k).dense_h(veff))[:20]
    e_minus = np.linalg.eigvalsh(KSetup(base, -k).dense_h(veff))[:20]
    e_shift = np.linalg.eigvalsh(KSetup(base, k + np.array([1.0, 0.0, -1.0])).dense_h(veff))[:20]
    assert np.abs(e - e_minus).max() < 1e-10
    assert np.abs(e - e_shift).max() < 1e-10


def test_gamma_k_equals_gamma_oracle():
    s = tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    r0 = run_scf(s)
    F0, _ = hf_forces(r0)
    rk = run_scf_k(s, [[0.0, 0.0, 0.0]], [1.0])
    Fk, _ = hf_forces_k(rk)
    assert abs(rk["energy"] - r0["energy"]) < 1e-9
    assert np.abs(Fk - F0).max() < 1e-7


@pytest.fixture(scope="module")
def folded():
    """Primitive cell at k in {0, b1/2} (weights 1/2) and its 2 x 1 x 1
    supercell at Gamma: the supercell's plane waves are exactly the union of
    the two primitive spheres, its grid doubles along a1 at the same
    spacing, so the two are one discrete problem."""
    # Fermi-Dirac smearing (one chemical potential for both sides) with 16
    # buffer bands per k above the 16 occupied ones: the states one side keeps
    # and the other drops then hold charge far below the tolerances below
    # (with 8 buffer bands their tails still move the terms by ~1e-7)
    s = tiny_system("sip", ecut=3.0, grid=(12, 12, 12), nbands=32)
    A = np.array(s["lattice"])
    pos = np.array(s["positions"])
    sup = make_system("super", np.vstack([2 * A[0], A[1], A[2]]), s["symbols"] * 2,
                      np.vstack([pos, pos + A[0]]), s["ecut"], (24, 12, 12), 2 * s["nbands"],
                      s["occupation"])
    rs = run_scf(sup, tol_e=1e-13, tol_rho=1e-11)
    Fs, _ = hf_forces(rs)
    rk = run_scf_k(s, [[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]], [0.5, 0.5], tol_e=1e-13, tol_rho=1e-11)
    Fk, _ = hf_forces_k(rk)
    return s, rs, Fs, rk, Fk


def test_supercell_folding_energy(folded):
    s, rs, Fs, rk, Fk = folded
    assert abs(rs["energy"] - 2 * rk["energy"]) < 1e-10
    for t in ("kinetic", "nonlocal", "local", "hartree", "xc", "ewald", "entropy"):
        assert abs(rs["terms"][t] - 2 * rk["terms"][t]) < 1e-10, t
    # the supercell spectrum is the union of the two k spectra (below the
    # highest kept state of either k)
    both = np.sort(np.concatenate(rk["eigenvalues"]))
    top = min(e[-1] for e in rk["eigenvalues"])
    keep = both[both <= top]
    assert np.abs(np.sort(rs["eigenvalues"])[:len(keep)] - keep).max() < 1e-10


def test_supercell_folding_forces(folded):
    s, rs, Fs, rk, Fk = folded
    n = len(s["symbols"])
    assert np.abs(Fs[:n] - Fk).max() < 1e-10
    assert np.abs(Fs[n:] - Fk).max() < 1e-10
    assert np.abs(Fk).max() > 1e-3  # the jittered cell carries real forces


def test_kpoint_force_is_the_energy_derivative():
    s = tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    k, w = monkhorst_pack((2, 1, 1))
    r = run_scf_k(s, k, w)
    F, _ = hf_forces_k(r)
    I, ax, h = 3, 1, 1e-3
    e = []
    for sgn in (1, -1):
        t = copy.deepcopy(s)
        p = np.array(t["positions"])
        p[I, ax] += sgn * h
        t["positions"] = p.tolist()
        e.append(run_scf_k(t, k, w)["energy"])
    fd = -(e[0] - e[1]) / (2 * h)
    assert abs(fd - F[I, ax]) < 2e-6
