"""Seeded random draws for the structure-search operators (Section 2.2).

Only random numbers: donor indices, plane normals and turning axes, sphere
offsets and radii, and uniform streams for random placement.  None of the
operators' arithmetic lives here.
"""
import numpy as np


def de_draws(n, attempts, seed, radius=(1.5, 3.0), offset_scale=0.5):
    """Draws for n targets x attempts: r [n, a, 3] three distinct donors
    other than the target, normal and axis [n, a, 3] Gaussian vectors, offset
    [n, a, 3] Gaussian with std offset_scale, radius [n, a] uniform."""
    rng = np.random.default_rng(seed)
    r = np.zeros((n, attempts, 3), dtype=np.int32)
    for i in range(n):
        others = np.array([j for j in range(n) if j != i])
        for a in range(attempts):
            r[i, a] = rng.choice(others, size=3, replace=False)
    return {"r": r,
            "normal": rng.normal(size=(n, attempts, 3)),
            "axis": rng.normal(size=(n, attempts, 3)),
            "offset": offset_scale * rng.normal(size=(n, attempts, 3)),
            "radius": rng.uniform(radius[0], radius[1], size=(n, attempts))}


def uniforms(count, seed):
    """Uniform stream in [0, 1) for random placement."""
    return np.random.default_rng(seed).random(count)
