"""Differential-evolution operators of the structure search (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).  Section 2.2 describes
the global search: random initialisation with distance checks, mutation
(Eq. 1, and the triangle form of Eq. 2), cut-and-splice crossover (plane and
sphere schemes) and greedy selection.  Every random number an operator uses
is an argument, so the same draws give the same result on any
implementation.

Readings where the text leaves the operator open:
  * structures are Cartesian position arrays [natoms, 3] in one fixed cell
    (the search varies positions; the cell is not mutated), and mutation
    combines the coordinate vectors atom by atom in stored order;
  * the "mass centre" is the unweighted centroid (the populations searched
    here have one element);
  * plane scheme: child = atoms of P1 strictly on the +n side of the plane
    through P1's centroid, plus atoms of P2 on the other side (or on it) of
    the plane through P2's centroid, P2's atoms translated by c1 - c2.  If
    the child's per-species counts differ from P1's, the normal is turned
    about the axis a (made unit and orthogonal to n) to the first angle in
    (0, 2 pi) at which they match: the side of each atom changes only at
    the angles where it lies on the plane, so the candidates are the
    midpoints between consecutive such angles (and angle 0 itself);
  * sphere scheme: spheres of radius r about each parent's centroid plus a
    common offset t; the child takes P2's atoms inside its sphere
    (translated by c1 - c2) and, per species, the atoms of P1 farthest from
    P1's sphere centre that complete P1's count (P1's sphere grows or shrinks
    until the counts match);
  * child atoms fill P1's species slots in order: for each slot of species s,
    first P1's atoms of s (in P1 order), then P2's (in P2 order);
  * minimum distances and distance fingerprints use the minimum-image
    convention over the 27 neighbouring cells; a child is rejected below
    max(d_min, 1e-3 bohr) (the evaluator refuses coincident atoms);
  * similarity of two structures = mean absolute difference of their sorted
    pair-distance lists;
  * selection keeps the child when its energy is strictly lower and its
    evaluation converged.
"""
import math

import numpy as np


# ------------------------------------------------------------------ mutation
def mutate_classic(x1, x2, x3, F):
    """Eq. 1: V = X_r3 + F (X_r1 - X_r2)."""
    x1, x2, x3 = (np.asarray(v, dtype=float) for v in (x1, x2, x3))
    return x3 + F * (x1 - x2)


def mutate_triangle(x1, x2, x3, f1, f2, f3):
    """Eq. 2: V = (X1 + X2 + X3)/3 + (p2 - p1)(X1 - X2) + (p3 - p2)(X2 - X3)
    + (p1 - p3)(X3 - X1) with p_k = |f_k| / (|f1| + |f2| + |f3|); equal
    weights 1/3 when all three fitness values are zero."""
    x1, x2, x3 = (np.asarray(v, dtype=float) for v in (x1, x2, x3))
    s = abs(f1) + abs(f2) + abs(f3)
    if s > 0:
        p1, p2, p3 = abs(f1) / s, abs(f2) / s, abs(f3) / s
    else:
        p1 = p2 = p3 = 1.0 / 3.0
    return ((x1 + x2 + x3) / 3.0 + (p2 - p1) * (x1 - x2) + (p3 - p2) * (x2 - x3)
            + (p1 - p3) * (x3 - x1))


# ----------------------------------------------------------------- crossover
def _fill_slots(species, take1, take2):
    """Child slot order: per species, P1's chosen atoms then P2's, assigned to
    the slots of that species in P1's order.  Returns [(parent, index)]."""
    species = list(species)
    out = [None] * len(species)
    for s in sorted(set(species)):
        slots = [j for j, t in enumerate(species) if t == s]
        src = [(0, j) for j in take1 if species[j] == s] + [(1, j) for j in take2 if species[j] == s]
        assert len(src) == len(slots)
        for k, j in enumerate(slots):
            out[j] = src[k]
    return out


def _counts(species, idx):
    c = {}
    for j in idx:
        c[species[j]] = c.get(species[j], 0) + 1
    return c


def cross_plane(p1, p2, species, normal, axis):
    """Plane cut-and-splice.  Returns (child [natoms, 3], source list of
    (parent 0/1, atom index), angle used) or None when no orientation gives
    P1's composition."""
    p1 = np.asarray(p1, dtype=float)
    p2 = np.asarray(p2, dtype=float)
    species = list(species)
    n = np.asarray(normal, dtype=float)
    n = n / np.linalg.norm(n)
    a = np.asarray(axis, dtype=float)
    a = a - (a @ n) * n
    a = a / np.linalg.norm(a)
    w = np.cross(a, n)  # n(theta) = n cos(theta) + w sin(theta)
    c1, c2 = p1.mean(0), p2.mean(0)
    r1, r2 = p1 - c1, p2 - c2
    want = _counts(species, range(len(species)))

    def split(theta):
        nt = n * math.cos(theta) + w * math.sin(theta)
        above = [j for j in range(len(p1)) if r1[j] @ nt > 0]
        below = [j for j in range(len(p2)) if not (r2[j] @ nt > 0)]
        return above, below

    # angles where an atom crosses the plane: (r.n) cos + (r.w) sin = 0
    ev = []
    for r in list(r1) + list(r2):
        u, v = float(r @ n), float(r @ w)
        if u == 0.0 and v == 0.0:
            continue
        t = math.atan2(-u, v) % math.pi
        ev += [t, t + math.pi]
    ev = sorted(set(ev))
    cands = [0.0]
    if ev:
        for k in range(len(ev)):
            lo = ev[k]
            hi = ev[k + 1] if k + 1 < len(ev) else ev[0] + 2 * math.pi
            cands.append(0.5 * (lo + hi))
    for theta in cands:
        above, below = split(theta)
        if len(above) + len(below) != len(species):
            continue
        got = _counts(species, above)
        for s, c in _counts(species, below).items():
            got[s] = got.get(s, 0) + c
        if got == want:
            src = _fill_slots(species, above, below)
            child = np.array([p1[j] if par == 0 else p2[j] + (c1 - c2) for par, j in src])
            return child, src, theta
    return None


def cross_sphere(p1, p2, species, offset, radius):
    """Sphere cut-and-splice.  Returns (child, source list)."""
    p1 = np.asarray(p1, dtype=float)
    p2 = np.asarray(p2, dtype=float)
    species = list(species)
    t = np.asarray(offset, dtype=float)
    c1, c2 = p1.mean(0), p2.mean(0)
    s1, s2 = c1 + t, c2 + t
    inside2 = [j for j in range(len(p2)) if np.linalg.norm(p2[j] - s2) < radius]
    k = _counts(species, inside2)
    take1 = []
    for s in sorted(set(species)):
        idx = [j for j in range(len(p1)) if species[j] == s]
        # farthest first; ties by index
        idx.sort(key=lambda j: (-np.linalg.norm(p1[j] - s1), j))
        take1 += sorted(idx[:len(idx) - k.get(s, 0)])
    take1.sort()
    src = _fill_slots(species, take1, inside2)
    child = np.array([p1[j] if par == 0 else p2[j] + (c1 - c2) for par, j in src])
    return child, src


# -------------------------------------------------------- checks and selection
def pair_distances(lattice, pos):
    """Minimum-image distances of every pair i < j (27 neighbouring cells)."""
    A = np.asarray(lattice, dtype=float)
    pos = np.asarray(pos, dtype=float)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)],
                      dtype=float) @ A
    out = []
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            d = pos[i] - pos[j] + shifts
            out.append(np.sqrt((d * d).sum(1)).min())
    return np.array(out)


def min_distance(lattice, pos):
    d = pair_distances(lattice, pos)
    return float(d.min()) if len(d) else math.inf


def similarity(lattice, pa, pb):
    """Mean absolute difference of the sorted pair-distance lists."""
    da = np.sort(pair_distances(lattice, pa))
    db = np.sort(pair_distances(lattice, pb))
    return float(np.abs(da - db).mean()) if len(da) else 0.0


def select(e_parent, e_child, child_ok):
    """Greedy selection: 1 where the child replaces its parent."""
    return np.array([1 if (ok and ec < ep) else 0
                     for ep, ec, ok in zip(e_parent, e_child, child_ok)], dtype=np.int32)


# ------------------------------------------------------------ initialisation
def init_positions(lattice, natoms, region, params, dmin, uniforms):
    """Random placement with the distance check.  region 0: whole cell
    (fractional uniform); 1: ball of radius params[0] about the cell centre;
    2: slab, fractional x, y uniform and z within params[0] bohr of the
    centre plane (thickness 2 params[0]).  Each trial atom consumes three
    uniforms; a trial closer than dmin (minimum image) to a placed atom is
    rejected.  Returns (positions, uniforms consumed) or None when the
    uniforms run out."""
    A = np.asarray(lattice, dtype=float)
    u = np.asarray(uniforms, dtype=float)
    centre = A.sum(0) / 2
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)],
                      dtype=float) @ A
    pos = []
    k = 0
    while len(pos) < natoms:
        if k + 3 > len(u):
            return None
        a, b, c = u[k], u[k + 1], u[k + 2]
        k += 3
        if region == 0:
            x = np.array([a, b, c]) @ A
        elif region == 1:
            R = params[0]
            r = R * a ** (1.0 / 3.0)
            ct = 2.0 * b - 1.0
            st = math.sqrt(max(0.0, 1.0 - ct * ct))
            ph = 2.0 * math.pi * c
            x = centre + r * np.array([st * math.cos(ph), st * math.sin(ph), ct])
        else:
            h = params[0]
            zc = 0.5 + (2.0 * c - 1.0) * h / np.linalg.norm(A[2])
            x = np.array([a, b, zc]) @ A
        ok = True
        for p in pos:
            d = x - p + shifts
            if np.sqrt((d * d).sum(1)).min() < dmin:
                ok = False
                break
        if ok:
            pos.append(x)
    return np.array(pos), k


def jitter_cell(lattice, delta, u3):
    """Lattice vectors scaled by 1 + delta (2 u_k - 1), k = 1..3."""
    A = np.array(lattice, dtype=float)
    for k in range(3):
        A[k] *= 1.0 + delta * (2.0 * u3[k] - 1.0)
    return A


# ---------------------------------------------------------------- generation
def make_trials(parents, e_parent, species, lattice, draws, mutation="triangle", crossover="plane",
                F=0.5, fitness_shift=True, dmin=0.0, sim_tol=0.0):
    """Trial structures of one generation (before their relaxation): for
    target i, the first draw whose mutant-target crossover gives an
    acceptable child (P1 = mutant, P2 = target; distance and similarity
    checks); the target itself when none does.  Returns (trials,
    attempt_used with -1 for none)."""
    n = len(parents)
    e = np.asarray(e_parent, dtype=float)
    f = e - e.min() if fitness_shift else e.copy()
    r = np.asarray(draws["r"])
    trials, used = [], []
    for i in range(n):
        got = None
        for a in range(r.shape[1]):
            r1, r2, r3 = (int(v) for v in r[i, a])
            x1, x2, x3 = (np.asarray(parents[k], dtype=float) for k in (r1, r2, r3))
            if mutation == "triangle":
                v = mutate_triangle(x1, x2, x3, f[r1], f[r2], f[r3])
            else:
                v = mutate_classic(x1, x2, x3, F)
            if crossover == "plane":
                res = cross_plane(v, parents[i], species, draws["normal"][i][a], draws["axis"][i][a])
                if res is None:
                    continue
                child = res[0]
            else:
                child, _ = cross_sphere(v, parents[i], species, draws["offset"][i][a],
                                        draws["radius"][i][a])
            if min_distance(lattice, child) < max(dmin, 1e-3):
                continue
            if sim_tol > 0 and any(similarity(lattice, child, parents[j]) < sim_tol for j in range(n)):
                continue
            got = (child, a)
            break
        if got is None:
            trials.append(np.asarray(parents[i], dtype=float).copy())
            used.append(-1)
        else:
            trials.append(got[0])
            used.append(got[1])
    return trials, np.array(used, dtype=np.int32)
