"""Autotuner of the launch schedule.

For a given population (a `Batch` already loaded with its candidates) it
times a fixed number of SCF iterations of the real workload under each
candidate value of one schedule parameter at a time (coordinate descent over
the Gram K range, subspace-solver threads, stick pairs per z block, density
chunks and graph replay), keeps the fastest, and caches the winning schedule
in a JSON file keyed by (device architecture, candidate shapes, precision).
A later call with the same key applies the cached schedule without timing.

Timing uses wall time around complete synchronous solves of `iters`
iterations (the library synchronises its stream before returning).
"""
import hashlib
import json
import os
import time

import numpy as np

from . import set_tuning, default_opts, SGO_ENOTCONV

SPACE = {
    "SGO_PLANE_KERNEL": [1, 2],
    "SGO_PLANE_GROUP": [1, 2, 3, 4, 5, 6, 8],
    "SGO_GEMM_KERNEL": [1, 2],
    "SGO_GRAM_KERNEL": [1, 2],
    "SGO_GRAM_KC": [256, 512, 1024, 2048],
    "SGO_SUB_THREADS": [64, 128, 256, 512],
    "SGO_DENS_CHUNKS": [1, 2, 4, 8],
    "SGO_RR_SWEEPS": [1, 2],
    "SGO_JAC_GRID": [96, 160, 100000],
    "SGO_GEMM_WAVES": [4, 6],
    "SGO_GRAM_TILE": [64],
    "use_graph": [0, 1, 2, 4],
}
# keys that only act from some band count on (largest band count of the
# population must reach it, else the key is not timed)
MIN_BANDS = {"SGO_JAC_GRID": 96, "SGO_GEMM_WAVES": 64}
# batch schedule: the population split into this many batches, each on its
# own stream from its own host thread (sgo_batches_scf), timed as whole
# solves to the caller's gate
BATCH_SPLITS = [1, 2, 4]
# schedules tuned for the standard workloads, shipped with the package and
# consulted when the user cache has no entry (python -m
# paper_1603_02732_amd.autotune --write-table regenerates it on the device)
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")
PRECISION_NAME = {0: "fp64", 1: "fp32", 2: "fp32bf16proj"}


def cache_path():
    return os.environ.get("SGO_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sgo", "autotune.json"))


def key_of(systems, precision, arch="gfx950"):
    shape = [(tuple(s["grid"]), int(s["nbands"]), len(s["symbols"])) for s in systems]
    h = hashlib.sha1(json.dumps([arch, precision, shape]).encode()).hexdigest()[:16]
    return "%s-%s-n%d-%s" % (arch, PRECISION_NAME.get(precision, str(precision)), len(systems), h)


def _time(batch, opts, reps=2):
    best = float("inf")
    for _ in range(reps):
        batch.reset()
        t0 = time.perf_counter()
        batch.scf(opts)
        best = min(best, time.perf_counter() - t0)
    return best


def apply(schedule):
    for k, v in schedule.items():
        if k.startswith("SGO_"):
            set_tuning(k, v)


def _load(path):
    if os.path.exists(path):
        try:
            return json.load(open(path))
        except (OSError, ValueError):
            return {}
    return {}


def lookup(systems, precision):
    """The cached (user cache, then package table) schedule for this
    population, applied, or None."""
    key = key_of(systems, precision)
    for path in (cache_path(), TABLE):
        entry = _load(path).get(key)
        if entry:
            apply(entry["schedule"])
            return dict(entry["schedule"], cached=True, source=os.path.basename(path))
    return None


def autotune(batch, systems, precision, iters=4, use_cache=True, verbose=False, path=None):
    """Returns the schedule (dict) and applies it.  `use_graph` in the result
    is for the caller's solve options."""
    key = key_of(systems, precision)
    path = path or cache_path()
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        apply(cache[key]["schedule"])
        return dict(cache[key]["schedule"], cached=True)
    sched = {k: 0 for k in SPACE}
    apply(sched)

    def opts():
        # a fixed number of iterations: the stop tests can never be met
        # iters iterations after the first (a graph of K iterations needs
        # K of them before max_iter)
        return default_opts(tol_e=-1.0, tol_rho=-1.0, max_iter=iters + 1,
                            use_graph=sched["use_graph"])

    batch.scf(opts())  # warm-up (allocation, first-touch)
    base = _time(batch, opts())
    timings = {"default": base}
    nb_max = max(int(x["nbands"]) for x in systems)
    for name, values in SPACE.items():
        if nb_max < MIN_BANDS.get(name, 0):
            continue
        best_v, best_t = sched[name], base
        for v in values:
            trial = dict(sched)
            trial[name] = v
            apply(trial)
            sched_backup = sched
            sched = trial
            t = _time(batch, opts())
            sched = sched_backup
            timings["%s=%d" % (name, v)] = t
            if verbose:
                print("autotune %s=%d: %.2f ms" % (name, v, t * 1e3), flush=True)
            if t < best_t * 0.98:
                best_v, best_t = v, t
        sched[name] = best_v
        base = best_t
        apply(sched)
    out = {"schedule": sched, "seconds_per_%d_iterations" % iters: base, "timings": timings}
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = out
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(sched, cached=False, timings=timings, seconds_per_iterations=base)


def tune_batch_split(systems, precision, gate_opts, splits=None, reps=5, verbose=False):
    """Time whole cold solves of the population to the caller's gate, as one
    batch and split into k batches solved at once on k streams (one host
    thread each), taking the median of `reps` solves.  Each stream should
    have a hardware queue of its own (GPU_MAX_HW_QUEUES >= k + 4 set before
    the HIP runtime starts): with HIP's default of 4 the streams share queues
    depending on how many streams the process created before them.  Returns
    (best k, {k: seconds})."""
    import torch
    from . import Batch, batches_scf
    timings = {}
    for k in splits or BATCH_SPLITS:
        if k > len(systems):
            continue
        bounds = [len(systems) * j // k for j in range(k + 1)]
        streams = [torch.cuda.Stream() for _ in range(k)]
        bs = []
        for j in range(k):
            b = Batch(bounds[j + 1] - bounds[j], precision=precision)
            b.set_stream(streams[j].cuda_stream)
            for x in systems[bounds[j]:bounds[j + 1]]:
                b.add_system(x)
            bs.append(b)

        def solve():
            for b in bs:
                b.reset()
            if k == 1:
                bs[0].scf(gate_opts)
            else:
                batches_scf(bs, gate_opts)
            torch.cuda.synchronize()

        solve()  # warm-up and allocation
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            solve()
            ts.append(time.perf_counter() - t0)
        for b in bs:
            b.close()
        timings[k] = float(np.median(ts))
        if verbose:
            print("autotune batches=%d: median %.2f ms (min %.2f, max %.2f)"
                  % (k, timings[k] * 1e3, min(ts) * 1e3, max(ts) * 1e3), flush=True)
    best_k = min(timings, key=timings.get)
    if timings[best_k] > 0.98 * timings.get(1, float("inf")):
        best_k = 1
    return best_k, timings


def _main():
    """Tune the standard populations on this device and write the table."""
    # a hardware queue per concurrent batch (see tune_batch_split), raised
    # to at least 8 before the runtime starts
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 8:
        os.environ["GPU_MAX_HW_QUEUES"] = "8"
    import argparse
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--write-table", action="store_true",
                    help="write the package table (or --table-path) instead of the user cache")
    ap.add_argument("--table-path", default=TABLE)
    ap.add_argument("--iters", type=int, default=4)
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    from . import Batch, SGO_FP32
    out = {}
    for name, pop in (("C3", workloads.config_c3()),):
        B = Batch(len(pop), precision=SGO_FP32)
        for s in pop:
            B.add_system(s)
        res = autotune(B, pop, SGO_FP32, iters=a.iters, use_cache=False, verbose=True)
        B.close()
        gate = default_opts(tol_e=1e-5, tol_rho=1.5e-4, cg_tol=1e-4, max_iter=150, mix_alpha=0.3,
                            kerker_q0=0.3, ncg_first=6, use_graph=res["use_graph"])
        k, tk = tune_batch_split(pop, SGO_FP32, gate, verbose=True)
        res["batches"] = k
        path = a.table_path if a.write_table else cache_path()
        table = _load(path)
        entry = table.get(key_of(pop, SGO_FP32), {})
        entry["timings"] = res.pop("timings")
        entry["seconds_per_%d_iterations" % a.iters] = res.pop("seconds_per_iterations")
        entry["schedule"] = {kk: v for kk, v in res.items() if kk != "cached"}
        entry["batch_split_seconds"] = {str(kk): v for kk, v in tk.items()}
        table[key_of(pop, SGO_FP32)] = entry
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1)
        print(name, res, flush=True)
        out[name] = res
    return out


if __name__ == "__main__":
    _main()
