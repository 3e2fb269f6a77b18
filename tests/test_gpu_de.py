"""One differential-evolution generation on the batched evaluator (Section
2.2 operators, Section 2.3 CG relaxation of every child, greedy selection)
against the oracle: trial structures and the draw each target used exactly
as the oracle's operators give them, relaxed child energies as the oracle's
relaxation of those trials, selection and survivors by the greedy rule."""
import copy

import numpy as np
import pytest

from tests.gpu_helpers import say
import workloads
from workloads.search import de_draws

pytestmark = pytest.mark.gpu

KW = dict(tol_e=1e-11, tol_rho=1e-9, max_iter=300)


def _population(n=5):
    return [workloads.tiny_system("c", ecut=4.0, grid=(15, 15, 15), seed=40 + k) for k in range(n)]


def _check_generation(B, pop, parents, E0, draws, crossover, relax_steps, dmin, oracle_relax):
    import paper_1603_02732_amd as sgo
    from oracle import de
    from oracle.relax import relax_cg
    species = [0] * len(pop[0]["symbols"])
    lat = np.asarray(pop[0]["lattice"], dtype=float)
    opts = sgo.de_opts(crossover=crossover, relax_steps=relax_steps, dmin=dmin,
                       attempts=draws["r"].shape[1])
    res = B.de_generation(parents, E0, draws, de=opts, **KW)
    tr_o, used_o = de.make_trials(parents, E0, species, lat, draws,
                                  crossover="plane" if crossover == sgo.SGO_DE_PLANE else "sphere",
                                  dmin=dmin)
    say("  crossover %d attempts used gpu %s oracle %s status %s"
        % (crossover, list(res["attempt_used"]), list(used_o), list(res["status"])))
    assert list(res["attempt_used"]) == list(used_o)
    for a, b in zip(res["trial"], tr_o):
        assert np.abs(a - b).max() < 1e-12
    assert np.all(res["status"] == 0)
    if oracle_relax:
        for i, s in enumerate(pop):
            t = copy.deepcopy(s)
            t["positions"] = tr_o[i].tolist()
            Eo, Xo, Fo = relax_cg(t, relax_steps)
            nat = len(s["symbols"])
            say("  child %d relaxed gpu %.8f oracle %.8f parent %.8f take %d"
                % (i, res["e_trial"][i], Eo[-1], E0[i], res["take"][i]))
            assert abs(res["e_trial"][i] - Eo[-1]) / nat < 1e-6
    # greedy selection and survivors
    take = (res["status"] == 0) & (res["e_trial"] < np.asarray(E0))
    assert np.array_equal(res["take"], take.astype(np.int32))
    for i in range(len(pop)):
        if take[i]:
            assert res["e_survivor"][i] == res["e_trial"][i]
        else:
            assert res["e_survivor"][i] == E0[i]
            assert np.array_equal(res["survivors"][i], np.asarray(parents[i], dtype=float))
    return res


def test_de_generation_matches_oracle():
    import paper_1603_02732_amd as sgo
    pop = _population()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    E0, _, st = B.scf(**KW)
    assert np.all(st == 0)
    parents = [np.asarray(s["positions"], dtype=float) for s in pop]
    draws = de_draws(len(pop), 3, seed=7, radius=(1.0, 2.0), offset_scale=0.3)
    say("generation 1: plane scheme, 1 CG step per child")
    res = _check_generation(B, pop, parents, list(E0), draws, sgo.SGO_DE_PLANE, 1, 1.8, True)
    # the batch now holds the survivors: a fresh solve reproduces their energies
    E1, _, st1 = B.scf(**KW)
    assert np.all(st1 == 0)
    assert np.abs(E1 - res["e_survivor"]).max() < 1e-7
    say("generation 2: sphere scheme from the survivors, no relaxation")
    draws2 = de_draws(len(pop), 3, seed=8, radius=(1.0, 2.5), offset_scale=0.3)
    _check_generation(B, pop, res["survivors"], list(res["e_survivor"]), draws2,
                      sgo.SGO_DE_SPHERE, 0, 1.8, False)


def test_de_generation_rejects_invalid_draws():
    import paper_1603_02732_amd as sgo
    pop = _population(4)
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    parents = [np.asarray(s["positions"], dtype=float) for s in pop]
    draws = de_draws(len(pop), 1, seed=9)
    draws["r"][2, 0] = [2, 0, 1]  # the target among its own donors
    with pytest.raises(sgo.SgoError):
        B.de_generation(parents, [0.0] * 4, draws, de=sgo.de_opts(attempts=1), **KW)


def test_de_generation_needs_four_candidates_and_valid_options():
    import paper_1603_02732_amd as sgo
    pop = _population(3)
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    parents = [np.asarray(s["positions"], dtype=float) for s in pop]
    draws = {"r": np.zeros((3, 1, 3), dtype=np.int32), "normal": np.ones((3, 1, 3)),
             "axis": np.ones((3, 1, 3)), "offset": np.zeros((3, 1, 3)), "radius": np.ones((3, 1))}
    with pytest.raises(sgo.SgoError) as err:
        B.de_generation(parents, [0.0] * 3, draws, de=sgo.de_opts(attempts=1), **KW)
    assert err.value.code == sgo.SGO_EINVAL
    pop4 = _population(4)
    B4 = sgo.Batch(4, precision=sgo.SGO_FP64)
    for s in pop4:
        B4.add_system(s)
    parents4 = [np.asarray(s["positions"], dtype=float) for s in pop4]
    d4 = de_draws(4, 1, seed=3)
    for bad in (sgo.de_opts(attempts=0), sgo.de_opts(relax_steps=-1), sgo.de_opts(dmin=-1.0),
                sgo.de_opts(mutation=7), sgo.de_opts(crossover=5)):
        with pytest.raises(sgo.SgoError) as err:
            B4.de_generation(parents4, [0.0] * 4, d4, de=bad, **KW)
        assert err.value.code == sgo.SGO_EINVAL
