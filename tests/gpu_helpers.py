"""Test-side helpers shared by the GPU tests: mapping between the packed
half-sphere storage of the HIP path and the oracle's full complex basis.
(Test infrastructure; neither the oracle nor the library imports this.)"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def half_to_full_index(gpu_millers, oracle_millers):
    key = {tuple(int(v) for v in m): i for i, m in enumerate(oracle_millers)}
    pos = np.array([key[tuple(int(v) for v in m)] for m in gpu_millers])
    neg = np.array([key[tuple(-int(v) for v in m)] for m in gpu_millers])
    return pos, neg


def pack(C, pos):
    """Full complex coefficients (npw, nb) -> packed (nb, 2*npw_half)."""
    h = C[pos]  # (nh, nb)
    out = np.zeros((C.shape[1], 2 * len(pos)))
    out[:, 0::2] = np.sqrt(2) * h.real.T
    out[:, 1::2] = np.sqrt(2) * h.imag.T
    out[:, 0] = h[0].real
    out[:, 1] = 0.0
    return out


def random_real_function_coeffs(npw, nb, pos, neg, seed):
    rng = np.random.default_rng(seed)
    C = np.zeros((npw, nb), dtype=complex)
    v = rng.standard_normal((len(pos), nb)) + 1j * rng.standard_normal((len(pos), nb))
    v[0] = v[0].real
    C[pos] = v
    C[neg] = np.conj(v)
    return C


def load_golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def full_coefficients(psi, millers_gpu, oracle_millers):
    """Packed half-sphere bands (nb, 2*nh) -> full complex coefficients (npw, nb)."""
    pos, neg = half_to_full_index(millers_gpu, oracle_millers)
    h = (psi[:, 0::2] + 1j * psi[:, 1::2]) / np.sqrt(2)
    h[:, 0] = psi[:, 0]
    C = np.zeros((len(oracle_millers), psi.shape[0]), dtype=complex)
    C[neg] = np.conj(h.T)
    C[pos] = h.T
    return C


def oracle_state_check(system, stt, forces, e_rtol, f_tol, say=say, stress=None, s_tol=None):
    """Hand the GPU's converged state (bands, occupations, density, V_eff) to
    the oracle and recompute, in FP64 with the oracle's own arithmetic: the
    density from the bands, every energy term, the Hellmann-Feynman forces and
    the eigen-residual under the oracle's Hamiltonian at V_eff."""
    from oracle.hamiltonian import Setup
    from oracle.scf import energy_terms, occupations
    from oracle.forces import hf_forces
    st = Setup(system)
    C = full_coefficients(stt["psi"], stt["millers"], st.millers)
    f = stt["occ"]
    rho = np.transpose(stt["rho"], (2, 1, 0))
    veff = np.transpose(stt["veff"], (2, 1, 0))
    say("  oracle check: setup done, %d plane waves" % st.npw)
    rho_o = st.density(C, f)
    say("  oracle check: density done")
    d_rho = np.abs(rho_o - rho).max() / np.abs(rho).max()
    occ = system["occupation"]
    _, _, S = occupations(stt["eig"], st.nelec, occ)
    terms = energy_terms(st, C, f, rho, S, float(occ.get("sigma", 0.0)))
    out = {"density": d_rho}
    for k in ("kinetic", "nonlocal", "local", "hartree", "xc", "ewald"):
        out[k] = abs(terms[k] - stt["terms"][k]) / max(1.0, abs(terms[k]))
    say("  oracle check: energy terms done")
    F_o, _ = hf_forces({"setup": st, "rho": rho, "C": C, "occupations": f})
    say("  oracle check: forces done")
    out["forces"] = np.abs(F_o - forces).max()
    if stress is not None:
        from oracle.stress import stress as oracle_stress
        sig_o, _ = oracle_stress({"setup": st, "rho": rho, "C": C, "occupations": f})
        out["stress"] = np.abs(sig_o - stress).max()
        say("  oracle check: stress done")
    HC = st.apply_h(veff, C)
    res = np.linalg.norm(HC - C * stt["eig"][None, :], axis=0)
    out["residual_charged"] = res[f > 1e-2].max()
    say("  oracle check of GPU state: " + "  ".join("%s %.1e" % kv for kv in out.items()))
    assert d_rho < e_rtol
    for k in ("kinetic", "nonlocal", "local", "hartree", "xc", "ewald"):
        assert out[k] < e_rtol, k
    assert out["forces"] < f_tol
    if stress is not None:
        assert out["stress"] < s_tol
    return out
