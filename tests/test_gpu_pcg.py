"""Force-fitted PCG and curved-line-search relaxations (Section 2.3) on the
batched evaluator against the oracle's own implementations of the same
algorithms."""
import numpy as np
import pytest

from tests.gpu_helpers import say
import workloads

pytestmark = pytest.mark.gpu

KW = dict(tol_e=1e-11, tol_rho=1e-9, max_iter=300)


def _pop():
    return [workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=31),
            workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=32)]


def test_pcg_relaxation_matches_oracle():
    import paper_1603_02732_amd as sgo
    from oracle.pcg import relax_pcg
    pop = _pop()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    E, F, X, prm, st = B.relax_pcg(2, refit=1, **KW)
    assert np.all(st == 0)
    for i, s in enumerate(pop):
        Eo, Xo, Fo = relax_pcg(s, 2, refit=1)
        nat = len(s["symbols"])
        say("  cand %d PCG energies gpu %s oracle %s fit %s" % (i, np.round(E[i], 7), np.round(Eo, 7),
                                                             np.round(prm[i], 5)))
        assert np.abs(E[i] - Eo).max() / nat < 1e-6
        assert np.abs(X[i] - Xo).max() < 1e-4
        assert np.abs(F[i] - Fo).max() < 1e-4
        assert Eo[-1] < Eo[0]


def test_cls_relaxation_matches_oracle():
    import paper_1603_02732_amd as sgo
    from oracle.cls import relax_cls
    pop = _pop()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    E, F, X, prm, st = B.relax_cls(2, **KW)
    assert np.all(st == 0)
    for i, s in enumerate(pop):
        Eo, Xo, Fo = relax_cls(s, 2)
        nat = len(s["symbols"])
        say("  cand %d CLS energies gpu %s oracle %s fit %s" % (i, np.round(E[i], 7), np.round(Eo, 7),
                                                             np.round(prm[i], 5)))
        assert np.abs(E[i] - Eo).max() / nat < 1e-6
        assert np.abs(X[i] - Xo).max() < 1e-4
        assert np.abs(F[i] - Fo).max() < 1e-4
