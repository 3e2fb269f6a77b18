"""Full-size workloads in the launch configuration the benchmark uses.

The candidates of the uneven population with a stored oracle result (the
smallest, a median one and the slowest to converge) are compared with it
directly: energy per atom within 1e-5 Ha and forces within 5e-4 Ha/bohr.
For sampled candidates, and for the 128-atom cell whose oracle SCF would
take hours, the GPU's converged state is also handed to the oracle, which
recomputes V_eff from the input density, the output density from the bands,
every energy term, the Hellmann-Feynman forces and the eigen-residual of
every band holding charge under its own Hamiltonian (asserted: the bands
are the self-consistent solution, not only consistent with themselves);
plus properties that hold at any size."""
import numpy as np
import pytest

from tests.gpu_helpers import say, oracle_state_check, load_golden
import workloads

pytestmark = pytest.mark.gpu

# solver settings of the uneven population (the bench's): mixing weight 0.3
# and the residual gate on the CG steps; the gate's final bound on the
# occupation-weighted residual (f/2)|H psi - eps psi| is max(1e-4, 0.1
# sqrt(1e-5)) = 3.2e-4 Ha, asserted below with a factor 3 for the oracle's
# FP64 Hamiltonian acting on the FP32 bands
C4_OPTS = dict(tol_e=1e-5, tol_rho=3e-4, max_iter=300, mix_alpha=0.3, cg_tol=1e-4)
RES_TOL = 1e-3
C4_GOLDEN = (14, 56, 7)


def test_c4_uneven_population_fp32():
    import paper_1603_02732_amd as sgo
    pop = workloads.config_c4()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP32)
    for s in pop:
        B.add_system(s)
    E, F, st = B.scf(sgo.default_opts(**C4_OPTS))
    say("C4: status", np.bincount(st + 6, minlength=7).tolist(),
        "iterations", [B.info(i)["iterations"] for i in range(len(pop))])
    assert np.all(st == 0)
    nat = np.array([len(s["symbols"]) for s in pop])
    for i in range(len(pop)):
        assert np.isfinite(E[i]) and np.all(np.isfinite(F[i]))
        assert np.abs(F[i].sum(0)).max() < 5e-2  # egg-box level
    checked = 0
    for k in C4_GOLDEN:
        ref = load_golden("C4-%d" % k, pop[k])
        if ref is None:
            continue
        dE = abs(E[k] - ref["energy"]) / nat[k]
        dF = np.abs(F[k] - np.array(ref["forces"])).max()
        say("C4-%d vs oracle: dE/atom %.2e  max dF %.2e" % (k, dE, dF))
        assert dE <= 1e-5
        assert dF <= 5e-4
        checked += 1
    assert checked >= 1
    picks = [int(np.argmin(nat)), int(np.argsort(nat)[len(nat) // 2]), int(np.argmax(nat))]
    for i in picks:
        s = pop[i]
        say("candidate %d: %d atoms grid %s bands %d" % (i, nat[i], s["grid"], s["nbands"]))
        oracle_state_check(s, B.state(i), F[i], e_rtol=2e-6, f_tol=5e-4, res_tol=RES_TOL)


def test_c5_large_cell_fp32_with_stress():
    """128-atom Si cell (FFT 108x54x54, 282 bands, s+p projectors): solve to
    the benchmark gate, then hand the state to the oracle, which recomputes
    energies, forces and the fixed-basis stress from the same bands and
    density (the stress here differs from the oracle's only by summation
    order, so its bound is far below the parity tolerance)."""
    import time
    import paper_1603_02732_amd as sgo
    s = workloads.config_c5()
    B = sgo.Batch(1, precision=sgo.SGO_FP32)
    B.add_system(s)
    t0 = time.perf_counter()
    E, F, st = B.scf(sgo.default_opts(tol_e=1e-5, tol_rho=3e-4, max_iter=200, cg_tol=1e-4))
    sig = B.stress()[0]
    say("C5: status %d iterations %d  %.2f s  E %.8f" % (st[0], B.info(0)["iterations"],
                                                         time.perf_counter() - t0, E[0]))
    say("C5 stress diag (Ha/bohr^3)", np.diag(sig))
    assert st[0] == 0
    assert np.abs(F[0].sum(0)).max() < 5e-2
    assert np.allclose(sig, sig.T)
    oracle_state_check(s, B.state(0), F[0], e_rtol=2e-6, f_tol=5e-4, stress=sig, s_tol=1e-7,
                       res_tol=RES_TOL)
