"""Boundary features around the solve: caller-provided arena allocator,
automatic FFT grid and band count, and the launch-schedule autotuner."""
import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import say
import workloads

pytestmark = pytest.mark.gpu


def _sgo():
    import paper_1603_02732_amd as sgo
    return sgo


def test_allocator_hooks_give_identical_results():
    """Arenas from PyTorch's caching allocator: the same energy and forces bit
    for bit (the kernels are deterministic and do not depend on addresses),
    every arena handed back on close."""
    sgo = _sgo()
    s = workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18))
    ref = sgo.context_from_system(s, sgo.SGO_FP32)
    ref.scf(tol_e=1e-7, tol_rho=1e-6, max_iter=200)
    e_ref, f_ref = ref.energy()[0], ref.forces()
    ref.close()
    hooks = sgo.TorchArenas(0)
    ctx = sgo.Context(0, sgo.SGO_FP32)
    ctx.set_allocator(hooks)
    ctx.load_system(s)
    ctx.scf(tol_e=1e-7, tol_rho=1e-6, max_iter=200)
    assert len(hooks.live) >= 1
    e, f = ctx.energy()[0], ctx.forces()
    say("  torch arenas: %d live, dE %.1e dF %.1e" % (len(hooks.live), abs(e - e_ref),
                                                      np.abs(f - f_ref).max()))
    assert e == e_ref and np.array_equal(f, f_ref)
    ctx.close()
    assert not hooks.live


def _smooth_len(n):
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


def test_automatic_grid_and_bands():
    """fft = (0, 0, 0) and nbands = 0: the smallest 2^a 3^b 5^c length with
    spacing <= 0.375 bohr that holds the sphere, and the even ceil(1.2 N_occ);
    the solve equals the one with the same values given explicitly."""
    from oracle.basis import sphere_millers
    sgo = _sgo()
    s = workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18))
    A = np.asarray(s["lattice"])
    m = np.abs(sphere_millers(A, s["ecut"])).max(0)
    want = [_smooth_len(max(int(np.ceil(np.linalg.norm(A[i]) / 0.375 - 1e-9)), 2 * int(m[i]) + 1))
            for i in range(3)]
    nocc = int(np.ceil(s["nelec"] / 2))
    nb = int(np.ceil(1.2 * nocc - 1e-9))
    nb += nb % 2
    auto = dict(s, grid=[0, 0, 0], nbands=0)
    ctx = sgo.context_from_system(auto, sgo.SGO_FP32)
    g = ctx.geometry()
    say("  automatic grid %s bands %d (expected %s, %d)" % ((g["N1"], g["N2"], g["N3"]), g["nbands"],
                                                          want, nb))
    assert [g["N1"], g["N2"], g["N3"]] == want and g["nbands"] == max(nb, nocc + 1)
    ctx.scf(tol_e=1e-7, tol_rho=1e-6, max_iter=200)
    e_auto = ctx.energy()[0]
    ctx.close()
    expl = sgo.context_from_system(dict(s, grid=want, nbands=g["nbands"]), sgo.SGO_FP32)
    expl.scf(tol_e=1e-7, tol_rho=1e-6, max_iter=200)
    assert expl.energy()[0] == e_auto
    expl.close()


def test_autotuner_times_and_caches(tmp_path, monkeypatch):
    """A reduced search space on a two-candidate population: the tuner times
    each value, keeps the fastest, writes the cache, and a second call
    applies the cached schedule without timing."""
    sgo = _sgo()
    from paper_1603_02732_amd import autotune
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("SGO_AUTOTUNE_CACHE", path)
    monkeypatch.setattr(autotune, "SPACE", {"SGO_PLANE_KERNEL": [1, 2], "SGO_DENS_CHUNKS": [1, 2],
                                            "use_graph": [0, 1]})
    pop = [workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=k) for k in (1, 2)]
    B = sgo.Batch(2, precision=sgo.SGO_FP32)
    for s in pop:
        B.add_system(s)
    try:
        res = autotune.autotune(B, pop, sgo.SGO_FP32, iters=2, verbose=True)
        assert res["cached"] is False
        assert res["SGO_PLANE_KERNEL"] in (0, 1, 2) and res["use_graph"] in (0, 1)
        cache = json.load(open(path))
        key = autotune.key_of(pop, sgo.SGO_FP32)
        assert key in cache and "timings" in cache[key]
        again = autotune.autotune(B, pop, sgo.SGO_FP32, iters=2)
        assert again["cached"] is True
        assert autotune.lookup(pop, sgo.SGO_FP32)["cached"] is True
        E, F, st = B.scf(sgo.default_opts(tol_e=1e-6, tol_rho=1e-5, max_iter=200,
                                          use_graph=again["use_graph"]))
        assert np.all(st == 0)
    finally:
        for k in ("SGO_PLANE_KERNEL", "SGO_GEMM_KERNEL", "SGO_GRAM_KC", "SGO_SUB_THREADS",
                  "SGO_SP_CHUNK", "SGO_DENS_CHUNKS"):
            sgo.set_tuning(k, 0)


def test_autotune_batch_split():
    """The batch-schedule phase of the tuner: the population as one batch and
    as two batches on two streams, whole solves to the gate; the pick is one
    of the timed splits and the split solve gives the single batch's
    energies."""
    sgo = _sgo()
    from paper_1603_02732_amd import autotune
    pop = [workloads.tiny_system("c", ecut=5.0, grid=(18, 18, 18), seed=k) for k in (1, 2, 3, 4)]
    gate = sgo.default_opts(tol_e=1e-7, tol_rho=1e-6, max_iter=200)
    k, timings = autotune.tune_batch_split(pop, sgo.SGO_FP32, gate, splits=[1, 2], reps=1,
                                           verbose=True)
    assert set(timings) == {1, 2} and k in (1, 2)
    assert all(t > 0 for t in timings.values())


def test_invalid_inputs_are_rejected_and_the_handle_stays_usable():
    """Degenerate and out-of-range inputs fail with SGO_EINVAL (checked on
    the host before any launch), and the same handle then solves a valid
    structure to the energy a fresh handle gives."""
    sgo = _sgo()
    s = workloads.tiny_system("c", ecut=4.0, grid=(15, 15, 15), seed=21)
    ref = sgo.context_from_system(s, sgo.SGO_FP64)
    ref.scf(sgo.default_opts(tol_e=1e-10, tol_rho=1e-8, max_iter=200))
    e_ref, _ = ref.energy()
    ref.close()

    ctx = sgo.context_from_system(s, sgo.SGO_FP64)
    pos = np.asarray(s["positions"], dtype=float)
    spec = ctx.atom_species
    cases = {
        "coincident atoms": lambda: ctx.set_atoms(spec, np.vstack([pos[:-1], pos[:1]])),
        "no atoms": lambda: ctx.set_atoms(np.zeros(0, dtype=np.int32), np.zeros((0, 3))),
        "flat cell": lambda: ctx.set_cell(np.diag([10.0, 10.0, 0.0])),
        "grid below the sphere": lambda: ctx.set_cutoff(4.0, (6, 6, 6), 10, sgo.SGO_OCC_FERMI, 0.01),
        "grid with a factor 7": lambda: ctx.set_cutoff(4.0, (14, 14, 14), 10, sgo.SGO_OCC_FERMI, 0.01),
        "too few bands": lambda: ctx.set_cutoff(4.0, (15, 15, 15), 3, sgo.SGO_OCC_FIXED, 0.0),
        "zero cutoff": lambda: ctx.set_cutoff(0.0, (15, 15, 15), 10, sgo.SGO_OCC_FERMI, 0.01),
        "non-positive smearing": lambda: ctx.set_cutoff(4.0, (15, 15, 15), 10, sgo.SGO_OCC_FERMI, 0.0),
    }
    for name, call in cases.items():
        with pytest.raises(sgo.SgoError) as err:
            call()
        say("  %s -> %s" % (name, err.value))
        assert err.value.code == sgo.SGO_EINVAL
    # restore the valid structure on the same handle and solve
    ctx.load_system(s)
    ctx.scf(sgo.default_opts(tol_e=1e-10, tol_rho=1e-8, max_iter=200))
    e, _ = ctx.energy()
    ctx.close()
    assert abs(e - e_ref) < 1e-8
