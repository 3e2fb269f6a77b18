"""The batched engine (one launch covers a population of candidates with
uneven atoms, grids and bands; converged candidates are masked out) against
the same candidates solved one at a time, and against the oracle."""
import numpy as np
import pytest

from tests.gpu_helpers import say, load_golden
import workloads

pytestmark = pytest.mark.gpu


def _population():
    a = workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=11)
    b = workloads.tiny_system("sip", ecut=3.0, grid=(12, 12, 15), seed=12)
    c = workloads.tiny_system("si", ecut=3.0, grid=(12, 12, 12), seed=13)
    d = workloads.tiny_system("c", ecut=4.0, grid=(16, 15, 16), seed=14, nbands=11)
    return [a, b, c, d]


def test_batch_equals_individual_fp64():
    import paper_1603_02732_amd as sgo
    pop = _population()
    say("batch of", len(pop), [s["grid"] for s in pop])
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    opts = sgo.default_opts(tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    E, F, st = B.scf(opts)
    assert list(st) == [0] * len(pop)
    for i, s in enumerate(pop):
        ctx = sgo.context_from_system(s, sgo.SGO_FP64)
        ctx.scf(opts)
        e1, _ = ctx.energy()
        f1 = ctx.forces()
        nat = len(s["symbols"])
        say("  cand %d: batch %.10f single %.10f  iters %d" % (i, E[i], e1, B.info(i)["iterations"]))
        assert abs(E[i] - e1) / nat < 1e-8
        assert np.abs(F[i] - f1).max() < 1e-6


def test_batch_matches_oracle_small():
    from oracle.scf import run_scf
    from oracle.forces import hf_forces
    import paper_1603_02732_amd as sgo
    pop = _population()[:2]
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP32)
    for s in pop:
        B.add_system(s)
    E, F, st = B.scf(sgo.default_opts(tol_e=1e-7, tol_rho=1e-6, max_iter=200))
    for i, s in enumerate(pop):
        r = run_scf(s)
        Fr, _ = hf_forces(r)
        nat = len(s["symbols"])
        dE = abs(E[i] - r["energy"]) / nat
        dF = np.abs(F[i] - Fr).max()
        say("  fp32 batch cand %d dE/atom %.2e dF %.2e" % (i, dE, dF))
        assert dE < 1e-5 and dF < 5e-4


def test_c3_population_fp32():
    import paper_1603_02732_amd as sgo
    pop = workloads.config_c3()
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP32)
    for s in pop:
        B.add_system(s)
    say("C3 population", len(pop))
    E, F, st = B.scf(sgo.default_opts(tol_e=1e-6, tol_rho=1e-4, max_iter=150))
    say("  status", list(st), "iters", [B.info(i)["iterations"] for i in range(len(pop))])
    assert np.all(st == 0)
    for k in range(2):
        ref = load_golden("C3-%d" % k, pop[k])
        if ref is None:
            continue
        dE = abs(E[k] - ref["energy"]) / 13
        dF = np.abs(F[k] - np.array(ref["forces"])).max()
        say("  C3-%d dE/atom %.2e dF %.2e" % (k, dE, dF))
        assert dE < 1e-5 and dF < 5e-4
    # translation of a candidate by a lattice vector leaves it unchanged
    for k in range(len(pop)):
        assert np.all(np.isfinite(F[k]))
        assert np.abs(F[k].sum(0)).max() < 5e-2


@pytest.mark.parametrize("prec,K", [("fp64", 1), ("fp32", 1), ("fp32", 3)])
def test_graph_replay_equals_eager(prec, K):
    """The SCF iterations after the first replay one captured HIP graph of K
    iterations (candidates that converge inside it mask themselves on the
    device); results and iteration counts must equal the eagerly launched
    sequence, call after call."""
    import paper_1603_02732_amd as sgo
    p = sgo.SGO_FP64 if prec == "fp64" else sgo.SGO_FP32
    pop = _population()
    B = sgo.Batch(len(pop), precision=p)
    for s in pop:
        B.add_system(s)
    kw = dict(tol_e=1e-9, tol_rho=1e-7, max_iter=200)
    for rep in range(3):
        B.reset()
        Ee, Fe, ste = B.scf(sgo.default_opts(use_graph=0, **kw))
        it_e = [B.info(i)["iterations"] for i in range(len(pop))]
        B.reset()
        Eg, Fg, stg = B.scf(sgo.default_opts(use_graph=K, **kw))
        it_g = [B.info(i)["iterations"] for i in range(len(pop))]
        dE = np.abs(Ee - Eg).max()
        dF = max(np.abs(a - b).max() for a, b in zip(Fe, Fg))
        say("  %s K=%d rep %d: graph vs eager dE %.2e dF %.2e iters %s %s"
            % (prec, K, rep, dE, dF, it_e, it_g))
        assert it_e == it_g and list(ste) == list(stg)
        assert dE == 0.0 and dF == 0.0


def test_cg_relaxation_matches_oracle():
    """Batched CG relaxation (3 steps, two evaluations each) against the
    oracle's own implementation of the same algorithm on small clusters."""
    import paper_1603_02732_amd as sgo
    from oracle.relax import relax_cg
    pop = [workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=31),
           workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=32)]
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    E, F, X, st = B.relax_cg(3, tol_e=1e-11, tol_rho=1e-9, max_iter=300)
    assert np.all(st == 0)
    for i, s in enumerate(pop):
        Eo, Xo, Fo = relax_cg(s, 3)
        nat = len(s["symbols"])
        say("  cand %d energies gpu %s oracle %s" % (i, np.round(E[i], 7), np.round(Eo, 7)))
        assert np.abs(E[i] - Eo).max() / nat < 1e-6
        assert Eo[-1] < Eo[0]  # the relaxation lowers the energy overall
        assert np.abs(X[i] - Xo).max() < 1e-4
        assert np.abs(F[i] - Fo).max() < 1e-4


def test_plane_groups_agree_with_one_plane_per_wavefront():
    """The H psi plane kernel with several z-planes per workgroup (the
    default where it fills the lanes better; forced sizes 2, 3 and 8, so that
    the last group of a candidate is partial) against one plane per
    wavefront, on an uneven FP32 batch: each line goes through the same
    transform either way, so the solves agree to FP32 rounding."""
    import paper_1603_02732_amd as sgo
    pop = _population()
    nat = [len(s["symbols"]) for s in pop]
    opts = sgo.default_opts(tol_e=1e-8, tol_rho=1e-6, max_iter=200)
    out = {}
    try:
        for grp in (1, 0, 2, 3, 8):
            sgo.set_tuning("SGO_PLANE_GROUP", grp)
            B = sgo.Batch(len(pop), precision=sgo.SGO_FP32)
            for s in pop:
                B.add_system(s)
            E, F, st = B.scf(opts)
            B.close()
            assert np.all(st == 0)
            out[grp] = (E, F)
    finally:
        sgo.set_tuning("SGO_PLANE_GROUP", 0)
    E1, F1 = out[1]
    for grp in (0, 2, 3, 8):
        E, F = out[grp]
        dE = max(abs(a - b) / n for a, b, n in zip(E, E1, nat))
        dF = max(float(np.abs(a - b).max()) for a, b in zip(F, F1))
        say("  plane group %d vs 1: dE/atom %.2e dF %.2e%s" % (grp, dE, dF,
            " (bit for bit)" if dE == 0 and dF == 0 else ""))
        assert dE < 1e-6 and dF < 1e-4


class _NoMemory:
    """Caller allocator with nothing to give: every request returns NULL."""

    def __init__(self, sgo):
        self.alloc = sgo.ALLOC_FN(lambda nbytes, user: None)
        self.free = sgo.FREE_FN(lambda ptr, user: None)


def test_concurrent_batches_report_a_hard_error_first():
    """Two batches at once, one stopping unconverged (SGO_ENOTCONV) and one
    whose arena allocation fails (SGO_ENOMEM): the call returns the
    allocation error, which no candidate status can stand in for."""
    import torch
    import paper_1603_02732_amd as sgo
    pop = _population()
    opts = sgo.default_opts(max_iter=2)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    Bs = []
    for half, stream in zip((pop[:2], pop[2:]), streams):
        b = sgo.Batch(len(half), precision=sgo.SGO_FP64)
        b.set_stream(stream.cuda_stream)
        for s in half:
            b.add_system(s)
        Bs.append(b)
    Bs[1].set_allocator(_NoMemory(sgo))
    with pytest.raises(sgo.SgoError) as err:
        sgo.batches_scf(Bs, opts)
    torch.cuda.synchronize()
    say("  unconverged batch beside a failed allocation: code %d" % err.value.code)
    assert err.value.code == sgo.SGO_ENOMEM
    _, _, st = Bs[0].scf(opts)  # alone, the first batch only stops unconverged
    assert np.all(st == sgo.SGO_ENOTCONV)


def test_concurrent_batches_with_iteration_graphs():
    """Concurrent batches whose SCF iterations run as captured graphs of 2
    iterations: while one batch's thread captures, the others keep reading
    their status and results, ordered on their own streams (a read on the
    legacy null stream would depend on the capturing stream and break the
    capture).  Each batch gives the state the eager concurrent solve gives."""
    import torch
    import paper_1603_02732_amd as sgo
    pop = _population()
    halves = [pop[:2], pop[2:]]
    out = {}
    for g in (0, 2):
        opts = sgo.default_opts(tol_e=1e-8, tol_rho=1e-6, max_iter=200, use_graph=g)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        Bs = []
        for half, stream in zip(halves, streams):
            b = sgo.Batch(len(half), precision=sgo.SGO_FP32)
            b.set_stream(stream.cuda_stream)
            for s in half:
                b.add_system(s)
            Bs.append(b)
        for rep in range(2):
            for b in Bs:
                b.reset()
            E, F, st = sgo.batches_scf(Bs, opts)
            torch.cuda.synchronize()
            assert np.all(st == 0)
        out[g] = (E, F)
        for b in Bs:
            b.close()
    nat = [len(s["symbols"]) for s in pop]
    dE = max(abs(a - b) / n for a, b, n in zip(out[0][0], out[2][0], nat))
    dF = max(float(np.abs(a - b).max()) for a, b in zip(out[0][1], out[2][1]))
    say("  concurrent batches, graphs of 2 iterations vs eager: dE %.2e dF %.2e" % (dE, dF))
    assert dE < 1e-6 and dF < 1e-4


def test_concurrent_batches_match_one_batch():
    """A population solved as two batches on two streams from two host
    threads gives each candidate the state one batch gives it (converged
    tightly: the random starting bands differ with the candidate's index)."""
    import torch
    import paper_1603_02732_amd as sgo
    pop = _population()
    opts = sgo.default_opts(tol_e=1e-10, tol_rho=1e-8, max_iter=200)
    B = sgo.Batch(len(pop), precision=sgo.SGO_FP64)
    for s in pop:
        B.add_system(s)
    E, F, st = B.scf(opts)
    assert np.all(st == 0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    halves = [pop[:2], pop[2:]]
    Bs = []
    for half, stream in zip(halves, streams):
        b = sgo.Batch(len(half), precision=sgo.SGO_FP64)
        b.set_stream(stream.cuda_stream)
        for s in half:
            b.add_system(s)
        Bs.append(b)
    sgo.profile_begin("k_gram")
    E2, F2, st2 = sgo.batches_scf(Bs, opts)
    torch.cuda.synchronize()
    prof = sgo.profile_end()
    assert np.all(st2 == 0)
    nat = [len(s["symbols"]) for s in pop]
    dE = max(abs(a - b) / n for a, b, n in zip(E, E2, nat))
    dF = max(float(np.abs(a - b).max()) for a, b in zip(F, F2))
    say("  two streams vs one batch: dE %.2e dF %.2e, profiled k_gram launches %d" % (dE, dF, prof["launches"]))
    assert dE < 1e-8 and dF < 1e-5
    assert prof["launches"] > 0 and prof["ms"] > 0
    with pytest.raises(sgo.SgoError):
        sgo.batches_scf([Bs[0], Bs[0]], opts)  # one handle twice
