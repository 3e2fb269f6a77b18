"""Full-size workloads in the launch configuration the benchmark uses, where
an oracle SCF would take hours: the GPU's converged state of sampled
candidates is handed to the oracle, which recomputes the density from the
bands, every energy term, the Hellmann-Feynman forces and the eigen-residual
under its own Hamiltonian; plus properties that hold at any size."""
import numpy as np
import pytest

from tests.gpu_helpers import say, oracle_state_check
import workloads

pytestmark = pytest.mark.gpu


def test_c4_uneven_population_fp32():
    import paper_1603_02732_amd as sgo
    pop = workloads.config_c4()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP32)
    for s in pop:
        B.add_system(s)
    E, F, st = B.scf(sgo.default_opts(tol_e=1e-5, tol_rho=1e-3, max_iter=300))
    say("C4: status", np.bincount(st + 6, minlength=7).tolist(),
        "iterations", [B.info(i)["iterations"] for i in range(len(pop))])
    assert np.all(st == 0)
    nat = np.array([len(s["symbols"]) for s in pop])
    for i in range(len(pop)):
        assert np.isfinite(E[i]) and np.all(np.isfinite(F[i]))
        assert np.abs(F[i].sum(0)).max() < 5e-2  # egg-box level
    picks = [int(np.argmin(nat)), int(np.argsort(nat)[len(nat) // 2]), int(np.argmax(nat))]
    for i in picks:
        s = pop[i]
        say("candidate %d: %d atoms grid %s bands %d" % (i, nat[i], s["grid"], s["nbands"]))
        oracle_state_check(s, B.state(i), F[i], e_rtol=2e-6, f_tol=5e-4)
