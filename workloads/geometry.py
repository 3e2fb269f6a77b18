"""Seeded geometry generators (positions in bohr, Cartesian).

All randomness comes from numpy.random.default_rng(seed) (PCG64); draws are
made atom by atom in x, y, z order.  No generator here evaluates any part of
the electronic-structure method.
"""
import math
import numpy as np

_DIAMOND_FRAC = [(0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0),
                 (0.25, 0.25, 0.25), (0.25, 0.75, 0.75), (0.75, 0.25, 0.75),
                 (0.75, 0.75, 0.25)]


def _min_image(d, lengths, periodic):
    d = np.array(d, dtype=float)
    for k in range(len(periodic)):
        if periodic[k]:
            d[..., k] -= np.round(d[..., k] / lengths[k]) * lengths[k]
    return d


def diamond_cells(a, reps, jitter, seed):
    """Diamond structure of reps[0] x reps[1] x reps[2] cubic cells of side a,
    every Cartesian coordinate displaced by U(-jitter, +jitter)."""
    rng = np.random.default_rng(seed)
    pos = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                for f in _DIAMOND_FRAC:
                    pos.append([(i + f[0]) * a, (j + f[1]) * a, (k + f[2]) * a])
    pos = np.array(pos, dtype=float)
    if jitter > 0:
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    lattice = np.diag([reps[0] * a, reps[1] * a, reps[2] * a])
    return lattice, pos


def sheet_random(n, lx, ly, lz, dmin, seed, sweeps=200, step=0.6):
    """Flat sheet of n atoms at z = lz/2 with random in-plane positions and
    minimum periodic distance dmin.

    Random sequential placement jams below the areal density some sheet
    workloads ask for, so the sheet is drawn as a hard-disk Monte Carlo
    chain: start from a staggered row lattice that satisfies dmin, then make
    `sweeps` passes of uniform trial moves of size `step`, each accepted only
    if every distance stays >= dmin.  Deterministic for a given seed.
    """
    rng = np.random.default_rng(seed)
    lengths = np.array([lx, ly, lz])
    per = (True, True, False)
    best = None
    for ncol in range(1, n + 1):
        if n % ncol:
            continue
        nrow = n // ncol
        sx, sy = lx / ncol, ly / nrow
        pts = np.array([[(c + 0.5 * (r % 2)) * sx + 0.25 * sx, (r + 0.5) * sy]
                        for r in range(nrow) for c in range(ncol)])
        d = _min_image(pts[:, None, :] - pts[None, :, :], lengths[:2], per[:2])
        dist = np.hypot(d[..., 0], d[..., 1]) + np.eye(n) * 1e9
        if best is None or dist.min() > best[0]:
            best = (dist.min(), pts)
    if best[0] < dmin:
        raise ValueError("sheet too dense for the requested minimum distance")
    pts = best[1].copy()
    for _ in range(sweeps):
        for i in range(n):
            trial = pts[i] + rng.uniform(-step, step, size=2)
            trial = np.mod(trial, lengths[:2])
            d = _min_image(pts - trial, lengths[:2], per[:2])
            r = np.hypot(d[:, 0], d[:, 1])
            r[i] = 1e9
            if r.min() >= dmin:
                pts[i] = trial
    pos = np.column_stack([pts, np.full(n, 0.5 * lz)])
    lattice = np.diag([lx, ly, lz])
    return lattice, pos


def _rsa(rng, n, sampler, dmin, lengths, periodic, max_fail=10000):
    pos = []
    fails = 0
    while len(pos) < n:
        p = sampler(rng)
        if pos:
            d = _min_image(np.array(pos) - p, lengths, periodic)
            ok = np.sqrt((d * d).sum(1)).min() >= dmin
        else:
            ok = True
        if ok:
            pos.append(p)
            fails = 0
        else:
            fails += 1
            if fails > max_fail:
                return None
    return np.array(pos)


def cluster_ball(n, box, radius, dmin, seed):
    """n atoms uniform in the ball of `radius` about the centre of a cubic box
    (rejection from the cube), minimum distance dmin.  After 10^4 consecutive
    failures the candidate restarts from seed + 10^6."""
    lengths = np.array([box, box, box], dtype=float)
    centre = lengths / 2

    def sampler(rng):
        while True:
            p = rng.uniform(-radius, radius, size=3)
            if (p * p).sum() <= radius * radius:
                return centre + p

    s = seed
    while True:
        pos = _rsa(np.random.default_rng(s), n, sampler, dmin, lengths,
                   (False, False, False))
        if pos is not None:
            return np.diag(lengths), pos
        s += 10 ** 6


def grid_rule(length, h=0.375):
    """Smallest 2^a 3^b 5^c >= length / h."""
    target = math.ceil(length / h - 1e-9)
    n = target
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


def nbands_rule(nocc, factor=1.2):
    """ceil(factor * nocc) rounded up to an even number."""
    nb = math.ceil(factor * nocc - 1e-9)
    return nb + (nb % 2)


def population_uneven(count, seed0, nmin=8, nmax=40, lmin=12.0, lmax=22.0, dmin=2.4):
    """Population of candidates with uneven atom counts and cells.

    Candidate k uses seed seed0 + k: n ~ U{nmin..nmax}; cubic with p = 1/2
    else orthorhombic; lengths ~ U[lmin, lmax]; atoms uniform in the periodic
    cell with minimum-image distance dmin (restart at seed + 10^6 after 10^4
    consecutive failures)."""
    out = []
    for k in range(count):
        seed = seed0 + k
        rng = np.random.default_rng(seed)
        n = int(rng.integers(nmin, nmax + 1))
        if rng.uniform() < 0.5:
            L = rng.uniform(lmin, lmax)
            lengths = np.array([L, L, L])
        else:
            lengths = rng.uniform(lmin, lmax, size=3)
        s = seed
        while True:
            pos = _rsa(np.random.default_rng(s + 7919), n,
                       lambda r: r.uniform(0, 1, size=3) * lengths, dmin, lengths,
                       (True, True, True))
            if pos is not None:
                break
            s += 10 ** 6
        out.append((np.diag(lengths), pos))
    return out
