"""Pins of the oracle's fixed-basis stress.

The stress is (1/Omega) dF/d eps at a fixed Miller set, so a central
difference of the self-consistent free energy over a strained cell (lattice
and positions strained together, same Miller set and grid) fixes every term
at once; a dropped term, a wrong sign or a transposed index would show there.
The per-term traces are fixed independently by virial identities:
tr sigma_kin = -2 E_kin / Omega (sum of G^2 |c|^2 is twice the kinetic
energy) and tr sigma_H = -E_H / Omega (-3 E_H from the volume plus 2 E_H from
the G^-2 factor).
"""
import numpy as np
import pytest

import workloads
from oracle.scf import run_scf
from oracle.stress import stress

TOL = dict(tol_e=1e-12, tol_rho=1e-11, maxiter=300)


def _strained(system, millers, eps):
    A = np.asarray(system["lattice"], dtype=float)
    P = np.asarray(system["positions"], dtype=float).reshape(-1, 3)
    M = np.eye(3) + eps
    s = dict(system)
    s["lattice"] = (A @ M.T).tolist()
    s["positions"] = (P @ M.T).tolist()
    s["millers"] = millers
    return s


def _fd(system, res, a, b, h=1e-4):
    eps = np.zeros((3, 3))
    eps[a, b] += 0.5 * h
    eps[b, a] += 0.5 * h
    mill = res["setup"].millers
    ep = run_scf(_strained(system, mill, eps), **TOL)["energy"]
    em = run_scf(_strained(system, mill, -eps), **TOL)["energy"]
    return (ep - em) / (2 * h) / res["setup"].omega


@pytest.fixture(scope="module", params=["si", "sip", "c"])
def solved(request):
    s = workloads.tiny_system(request.param)
    return request.param, s, run_scf(s, **TOL)


@pytest.mark.parametrize("comp", [(0, 0), (1, 2)])
def test_stress_matches_strain_differences(solved, comp):
    kind, s, r = solved
    if kind != "sip" and comp == (1, 2):
        comp = (0, 1)
    sig, _ = stress(r)
    fd = _fd(s, r, *comp)
    assert abs(fd - sig[comp]) < 2e-9, (kind, comp, fd, sig[comp])


def test_stress_virial_traces(solved):
    _, _, r = solved
    _, parts = stress(r)
    om = r["setup"].omega
    t = r["terms"]
    assert np.trace(parts["kinetic"]) == pytest.approx(-2 * t["kinetic"] / om, rel=1e-12)
    assert np.trace(parts["hartree"]) == pytest.approx(-t["hartree"] / om, rel=1e-12)
    for k, v in parts.items():
        assert np.allclose(v, v.T, atol=1e-15), k


def test_stress_rotation_covariance():
    """Rotating the cell and positions rotates the stress tensor."""
    s = workloads.tiny_system("sip")
    r = run_scf(s, **TOL)
    sig, _ = stress(r)
    th = 0.3
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    A = np.asarray(s["lattice"]) @ R.T
    P = np.asarray(s["positions"]).reshape(-1, 3) @ R.T
    s2 = dict(s, lattice=A.tolist(), positions=P.tolist(), millers=r["setup"].millers)
    sig2, _ = stress(run_scf(s2, **TOL))
    assert np.allclose(sig2, R @ sig @ R.T, atol=1e-9)
