"""k-point sampling on the GPU (the FP64 complex-band path) against the
oracle's k-point SCF: energy per atom within 1e-6 Ha, forces within 1e-4
Ha/bohr, every energy term, and the eigenvalues of every band holding
charge at every k; the k-point set {Gamma} against the Gamma-point path;
time reversal eps(k) = eps(-k) of the GPU's own bands."""
import numpy as np
import pytest

from tests.gpu_helpers import say
import workloads

pytestmark = pytest.mark.gpu


def _solve(s, k, w, **kw):
    import paper_1603_02732_amd as sgo
    ctx = sgo.context_from_system(s, sgo.SGO_FP64)
    ctx.set_kpoints(k, w)
    info = ctx.scf(**kw)
    E, terms = ctx.energy()
    return ctx, info, E, terms, ctx.forces()


def test_kpoints_match_oracle():
    from oracle.kpoints import run_scf_k, hf_forces_k, monkhorst_pack
    s = workloads.tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    k, w = monkhorst_pack((2, 2, 1))
    say("k-points oracle: %d k" % len(k))
    ref = run_scf_k(s, k, w)
    Fref, _ = hf_forces_k(ref)
    ctx, info, E, terms, F = _solve(s, k, w, tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    eig, occ = ctx.kpoint_eigenvalues()
    nat = len(s["symbols"])
    dE = abs(E - ref["energy"]) / nat
    dF = np.abs(F - Fref).max()
    say("  info", info, "dE/atom %.2e  max dF %.2e" % (dE, dF))
    assert info["converged"]
    assert dE < 1e-6
    assert dF < 1e-4
    for t in ("kinetic", "nonlocal", "local", "hartree", "xc", "ewald"):
        say("   %-8s gpu %.10f oracle %.10f" % (t, terms[t], ref["terms"][t]))
        assert abs(terms[t] - ref["terms"][t]) < 1e-6 * nat, t
    for ik in range(len(k)):
        f = np.asarray(ref["occupations"][ik])
        held = f > 1e-6
        de = np.abs(eig[ik][held] - np.asarray(ref["eigenvalues"][ik])[held]).max()
        say("  k %d eigenvalue err %.2e" % (ik, de))
        assert de < 1e-5
        assert np.abs(occ[ik] - f).max() < 1e-5


def test_gamma_kpoint_equals_gamma_path():
    import paper_1603_02732_amd as sgo
    s = workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18))
    ctx, info, E, terms, F = _solve(s, [[0.0, 0.0, 0.0]], [1.0], tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    g = sgo.context_from_system(s, sgo.SGO_FP64)
    g.scf(tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    Eg, _ = g.energy()
    Fg = g.forces()
    say("  gamma via k-points %.12f, gamma path %.12f, max dF %.2e" % (E, Eg, np.abs(F - Fg).max()))
    assert abs(E - Eg) < 1e-8
    assert np.abs(F - Fg).max() < 1e-6


def test_kpoint_time_reversal_and_errors():
    import paper_1603_02732_amd as sgo
    s = workloads.tiny_system("sip", ecut=3.0, grid=(12, 12, 12))
    k = np.array([[0.25, 0.1, 0.0], [-0.25, -0.1, 0.0]])
    ctx, info, E, terms, F = _solve(s, k, [1.0, 1.0], tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    eig, _ = ctx.kpoint_eigenvalues()
    say("  eps(k) - eps(-k): %.2e" % np.abs(eig[0] - eig[1]).max())
    assert np.abs(eig[0] - eig[1]).max() < 1e-8
    with pytest.raises(sgo.SgoError):
        ctx.stress()
    c32 = sgo.context_from_system(s, sgo.SGO_FP32)
    with pytest.raises(sgo.SgoError):
        c32.set_kpoints(k, [1.0, 1.0])
    with pytest.raises(sgo.SgoError):
        ctx.set_kpoints(k, [1.0, -1.0])
