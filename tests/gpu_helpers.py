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


def same_system(a, b):
    """True when two workload dicts describe the same discrete problem."""
    return (a["nbands"] == b["nbands"] and list(a["grid"]) == list(b["grid"])
            and a["ecut"] == b["ecut"] and list(a["symbols"]) == list(b["symbols"])
            and np.array_equal(np.asarray(a["lattice"]), np.asarray(b["lattice"]))
            and np.array_equal(np.asarray(a["positions"]), np.asarray(b["positions"]))
            and a["occupation"] == b["occupation"])


def load_golden(name, system=None):
    """The oracle's stored result for `name`, or None if none is stored.
    With `system`, a stored result computed for a different problem (say
    an older band count) is an error, not a reference."""
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)
    if system is not None:
        assert same_system(ref["system"], system), \
            "stored oracle result %s was computed for another problem; regenerate it" % name
    return ref


def full_coefficients(psi, millers_gpu, oracle_millers):
    """Packed half-sphere bands (nb, 2*nh) -> full complex coefficients (npw, nb)."""
    pos, neg = half_to_full_index(millers_gpu, oracle_millers)
    h = (psi[:, 0::2] + 1j * psi[:, 1::2]) / np.sqrt(2)
    h[:, 0] = psi[:, 0]
    C = np.zeros((len(oracle_millers), psi.shape[0]), dtype=complex)
    C[neg] = np.conj(h.T)
    C[pos] = h.T
    return C


def oracle_state_check(system, stt, forces, e_rtol, f_tol, say=say, stress=None, s_tol=None,
                       res_tol=None, v_tol=1e-8):
    """Hand the GPU's converged state (bands, occupations, input and output
    density, V_eff) to the oracle and recompute, in FP64 with the oracle's own
    arithmetic: V_eff from the input density, the output density from the
    bands, every energy term, the Hellmann-Feynman forces and the
    eigen-residual |H psi - eps psi| of every band holding charge under the
    oracle's Hamiltonian at V_eff (asserted below res_tol: the bands are the
    self-consistent solution, not only self-consistent with themselves)."""
    from oracle.hamiltonian import Setup
    from oracle.scf import energy_terms, occupations, potentials
    from oracle.forces import hf_forces
    st = Setup(system)
    C = full_coefficients(stt["psi"], stt["millers"], st.millers)
    f = stt["occ"]
    rho = np.transpose(stt["rho"], (2, 1, 0))
    veff = np.transpose(stt["veff"], (2, 1, 0))
    say("  oracle check: setup done, %d plane waves" % st.npw)
    out_v = None
    if "rho_in" in stt:
        veff_o, _ = potentials(st, np.transpose(stt["rho_in"], (2, 1, 0)))
        out_v = np.abs(veff_o - veff).max()
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
    charged = f > 1e-6
    out["residual_charged"] = res[charged].max()
    # weighted by the occupation fraction f/2: how far each band moves the
    # density and the energy (what the residual gate of the solver bounds)
    out["residual_weighted"] = (0.5 * f[charged] * res[charged]).max()
    if out_v is not None:
        out["veff_from_rho_in"] = out_v
    say("  oracle check of GPU state: " + "  ".join("%s %.1e" % kv for kv in out.items()))
    assert d_rho < e_rtol
    for k in ("kinetic", "nonlocal", "local", "hartree", "xc", "ewald"):
        assert out[k] < e_rtol, k
    assert out["forces"] < f_tol
    if stress is not None:
        assert out["stress"] < s_tol
    if out_v is not None:
        assert out_v < v_tol
    if res_tol is not None:
        assert out["residual_weighted"] < res_tol
    return out
