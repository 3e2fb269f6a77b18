"""Pins of the oracle's SCF energy and forces: uniform-gas closed form,
grid-vector translation, atom permutation, Newton's third law within the
egg-box error, symmetry zeros and central finite differences."""
import copy

import numpy as np
import pytest

from oracle.scf import run_scf
from oracle.forces import hf_forces
from oracle.lda import pz81
from workloads import make_system, tiny_system, diamond_cells, sheet_random


def test_one_band_jellium():
    a = 8.0
    s = make_system("jellium", np.eye(3) * a, [], np.zeros((0, 3)), 2.0, (10, 10, 10), 1,
                    {"kind": "fixed"})
    s["nelec"] = 2.0
    r = run_scf(s)
    rho = 2.0 / a ** 3
    exc, vxc = pz81(np.array([rho]))
    t = r["terms"]
    assert r["info"]["iterations"] <= 2
    assert abs(t["kinetic"]) < 1e-14 and abs(t["hartree"]) < 1e-14
    assert abs(r["energy"] - 2 * exc[0]) < 1e-12
    assert abs(r["eigenvalues"][0] - vxc[0]) < 1e-12
    assert np.abs(r["rho"] - rho).max() < 1e-14


@pytest.fixture(scope="module")
def si_tiny():
    s = tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    r = run_scf(s)
    F, parts = hf_forces(r)
    return s, r, F, parts


def test_grid_translation_exact(si_tiny):
    s, r, F, _ = si_tiny
    s2 = copy.deepcopy(s)
    A = np.array(s["lattice"])
    t = 3 * A[0] / 12 + 5 * A[2] / 12
    s2["positions"] = (np.array(s["positions"]) + t).tolist()
    r2 = run_scf(s2)
    F2, _ = hf_forces(r2)
    assert abs(r2["energy"] - r["energy"]) < 1e-9
    assert np.abs(F2 - F).max() < 1e-7


def test_permutation(si_tiny):
    s, r, F, _ = si_tiny
    perm = [3, 0, 7, 1, 6, 2, 5, 4]
    s2 = copy.deepcopy(s)
    s2["positions"] = [s["positions"][i] for i in perm]
    s2["symbols"] = [s["symbols"][i] for i in perm]
    r2 = run_scf(s2)
    F2, _ = hf_forces(r2)
    assert abs(r2["energy"] - r["energy"]) < 1e-9
    assert np.abs(F2 - F[perm]).max() < 1e-7


def test_force_sum(si_tiny):
    _, _, F, parts = si_tiny
    assert np.abs(parts["ewald"].sum(0)).max() < 1e-12
    # egg-box: total only approximately balanced on a coarse grid
    assert np.abs(F.sum(0)).max() < 5e-3


def test_finite_difference_forces(si_tiny):
    s, r, F, _ = si_tiny
    h = 1e-3
    for I, a in [(1, 0), (3, 2), (6, 1)]:
        e = []
        for sg in (1, -1):
            s2 = copy.deepcopy(s)
            s2["positions"][I][a] += sg * h
            e.append(run_scf(s2)["energy"])
        assert abs(-(e[0] - e[1]) / (2 * h) - F[I, a]) < 2e-6


def test_perfect_diamond_zero_forces():
    lat, pos = diamond_cells(10.26, (1, 1, 1), 0.0, 0)
    s = make_system("d0", lat, ["Si-AH"] * 8, pos, 3.0, (12, 12, 12), 20, {"kind": "fixed"})
    r = run_scf(s)
    F, _ = hf_forces(r)
    assert np.abs(F).max() < 1e-8


def test_flat_sheet_no_normal_force():
    lat, pos = sheet_random(4, 6.0, 6.0, 8.0, 2.4, 4)
    s = make_system("sheet", lat, ["C-G"] * 4, pos, 5.0, (16, 16, 20), 12,
                    {"kind": "fermi", "sigma": 0.01})
    r = run_scf(s)
    F, _ = hf_forces(r)
    assert np.abs(F[:, 2]).max() < 1e-8
    assert np.abs(F[:, :2]).max() > 1e-3


def test_dense_and_iterative_scf_agree():
    s = tiny_system("c", ecut=4.0, grid=(16, 16, 16))
    rd = run_scf(s)
    ri = run_scf(s, dense_max=0)
    assert abs(rd["energy"] - ri["energy"]) < 1e-9
    Fd, _ = hf_forces(rd)
    Fi, _ = hf_forces(ri)
    assert np.abs(Fd - Fi).max() < 1e-6
