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
