"""Pins of the structure-search operators of the oracle (Section 2.2):
closed forms of the mutation, hand-checked and brute-force crossovers,
distance and similarity invariants, selection and placement rules."""
import math

import numpy as np
from oracle import de


# ------------------------------------------------------------------ mutation
def test_triangle_weights_closed_form():
    # With the three donors the unit vectors of R^3, Eq. 2 returns its own
    # weights; expanding the printed form gives 4/3 - 3 p_k for donor k.
    e = np.eye(3)
    for f in [(-3.0, -1.0, -2.0), (2.0, 5.0, 1.0), (-0.5, 0.0, 4.0)]:
        p = np.abs(f) / np.abs(f).sum()
        v = de.mutate_triangle(e[0], e[1], e[2], *f)
        assert np.allclose(v, 4.0 / 3.0 - 3.0 * p, atol=1e-15)
        assert abs(v.sum() - 1.0) < 1e-15  # an affine combination
    # the worked case f = (-3, -1, -2): p = (1/2, 1/6, 1/3)
    v = de.mutate_triangle(e[0], e[1], e[2], -3.0, -1.0, -2.0)
    assert np.allclose(v, [-1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0], atol=1e-15)


def test_triangle_special_cases():
    rng = np.random.default_rng(1)
    x1, x2, x3 = rng.normal(size=(3, 5, 3))
    centroid = (x1 + x2 + x3) / 3
    # equal |f| (also of mixed sign) and all-zero fitness give the centroid
    for f in [(2.0, 2.0, 2.0), (-1.0, 1.0, -1.0), (0.0, 0.0, 0.0)]:
        assert np.allclose(de.mutate_triangle(x1, x2, x3, *f), centroid, atol=1e-14)
    # identical donors give that donor
    assert np.allclose(de.mutate_triangle(x1, x1, x1, -1.0, -2.0, -7.0), x1, atol=1e-14)
    # translation covariance (weights sum to one)
    t = np.array([0.3, -1.2, 2.5])
    v0 = de.mutate_triangle(x1, x2, x3, -1.0, -2.0, -4.0)
    v1 = de.mutate_triangle(x1 + t, x2 + t, x3 + t, -1.0, -2.0, -4.0)
    assert np.allclose(v1, v0 + t, atol=1e-13)
    # the donor with the smallest |f| gets the largest weight
    e = np.eye(3)
    w = de.mutate_triangle(e[0], e[1], e[2], 0.1, 3.0, 1.0)
    assert np.argmax(w) == 0 and np.argmin(w) == 1


def test_classic_mutation():
    rng = np.random.default_rng(2)
    x1, x2, x3 = rng.normal(size=(3, 4, 3))
    assert np.array_equal(de.mutate_classic(x1, x2, x3, 0.0), x3)
    assert np.array_equal(de.mutate_classic(x1, x1, x3, 0.7), x3)
    assert np.allclose(de.mutate_classic(x1, x2, x3, 0.5) - x3, 0.5 * (x1 - x2), atol=1e-15)


# ----------------------------------------------------------------- crossover
def _line(xs, y=0.0):
    return np.array([[x, y, 0.0] for x in xs])


def test_plane_hand_example():
    # P1 on the x axis at -3, -1, 1, 3; P2 at -3.5, -0.5, 0.5, 3.5 shifted by
    # (0, 2, 0); plane normal +x through each centroid.  The child keeps
    # P1's x > 0 atoms and P2's x <= 0 atoms moved onto P1's centroid.
    p1 = _line([-3, -1, 1, 3])
    p2 = _line([-3.5, -0.5, 0.5, 3.5], y=2.0)
    child, src, theta = de.cross_plane(p1, p2, [0] * 4, [1, 0, 0], [0, 0, 1])
    assert theta == 0.0
    assert src == [(0, 2), (0, 3), (1, 0), (1, 1)]
    assert np.allclose(child, _line([1, 3, -3.5, -0.5]), atol=1e-15)


def _brute_plane(p1, p2, species, normal, axis, steps=200000):
    """Scan the turning angle finely and return the source sets at the first
    angle whose per-species counts match P1's."""
    n = np.asarray(normal, float) / np.linalg.norm(normal)
    a = np.asarray(axis, float) - (np.dot(axis, n)) * n
    a /= np.linalg.norm(a)
    w = np.cross(a, n)
    r1, r2 = p1 - p1.mean(0), p2 - p2.mean(0)
    want = sorted(species)
    for k in range(steps):
        t = 2 * math.pi * k / steps
        nt = n * math.cos(t) + w * math.sin(t)
        up = [j for j in range(len(p1)) if r1[j] @ nt > 0]
        dn = [j for j in range(len(p2)) if not (r2[j] @ nt > 0)]
        if sorted([species[j] for j in up] + [species[j] for j in dn]) == want:
            return set(up), set(dn), t
    return None


def _split(p1, p2, normal, axis, t):
    n = np.asarray(normal, float) / np.linalg.norm(normal)
    a = np.asarray(axis, float) - (np.dot(axis, n)) * n
    a /= np.linalg.norm(a)
    nt = n * math.cos(t) + np.cross(a, n) * math.sin(t)
    r1, r2 = p1 - p1.mean(0), p2 - p2.mean(0)
    return ({j for j in range(len(p1)) if r1[j] @ nt > 0},
            {j for j in range(len(p2)) if not (r2[j] @ nt > 0)})


def test_plane_turns_to_the_first_matching_angle():
    rng = np.random.default_rng(3)
    hits = 0
    for trial in range(12):
        p1 = rng.normal(size=(7, 3)) * 2
        p2 = rng.normal(size=(7, 3)) * 2
        normal, axis = rng.normal(size=3), rng.normal(size=3)
        res = de.cross_plane(p1, p2, [0] * 7, normal, axis)
        bf = _brute_plane(p1, p2, [0] * 7, normal, axis)
        assert (res is None) == (bf is None)
        if res is None:
            continue
        child, src, theta = res
        up = {j for par, j in src if par == 0}
        dn = {j for par, j in src if par == 1}
        assert (up, dn) == bf[:2]
        # the first matching orientation of the scan lies in the interval of
        # orientations the returned angle represents: same split all along
        assert bf[2] <= theta + 1e-12
        for t in np.linspace(bf[2], theta, 9):
            assert _split(p1, p2, normal, axis, t) == (up, dn)
        hits += theta > 0
        # child atoms are the parents' atoms, P2's moved by c1 - c2
        shift = p1.mean(0) - p2.mean(0)
        for (par, j), x in zip(src, child):
            assert np.allclose(x, p1[j] if par == 0 else p2[j] + shift, atol=1e-14)
    assert hits > 0  # some cases needed a turn


def test_plane_keeps_species_counts():
    rng = np.random.default_rng(4)
    species = [0, 0, 0, 1, 1, 2, 2, 2]
    for trial in range(10):
        p1 = rng.normal(size=(8, 3)) * 2
        p2 = rng.normal(size=(8, 3)) * 2
        res = de.cross_plane(p1, p2, species, rng.normal(size=3), rng.normal(size=3))
        if res is None:
            continue
        child, src, _ = res
        # every slot holds an atom of the slot's species
        assert [species[j] for _, j in src] == species
        assert len({(par, j) for par, j in src}) == 8


def test_sphere_hand_example():
    # P2's atoms within radius 1.2 of its centroid (the two middle ones) go
    # in; P1 keeps its two atoms farthest from its centroid.
    p1 = _line([-3, -1, 1, 3])
    p2 = _line([-3.5, -0.5, 0.5, 3.5], y=2.0)
    child, src = de.cross_sphere(p1, p2, [0] * 4, [0, 0, 0], 1.2)
    assert src == [(0, 0), (0, 3), (1, 1), (1, 2)]
    assert np.allclose(child, _line([-3, 3, -0.5, 0.5]), atol=1e-15)
    # radius 0: the child is P1
    child, src = de.cross_sphere(p1, p2, [0] * 4, [0, 0, 0], 0.0)
    assert np.array_equal(child, p1) and all(par == 0 for par, _ in src)


def test_sphere_brute_force():
    rng = np.random.default_rng(5)
    species = [0, 0, 0, 0, 1, 1, 1]
    for trial in range(10):
        p1 = rng.normal(size=(7, 3)) * 2
        p2 = rng.normal(size=(7, 3)) * 2
        t = 0.5 * rng.normal(size=3)
        R = rng.uniform(0.5, 3.0)
        child, src = de.cross_sphere(p1, p2, species, t, R)
        s2 = p2.mean(0) + t
        inside = {j for j in range(7) if np.linalg.norm(p2[j] - s2) < R}
        assert {j for par, j in src if par == 1} == inside
        s1 = p1.mean(0) + t
        kept = {j for par, j in src if par == 0}
        for sp in set(species):
            mine = [j for j in range(7) if species[j] == sp]
            k = sum(1 for j in inside if species[j] == sp)
            far = sorted(mine, key=lambda j: -np.linalg.norm(p1[j] - s1))[:len(mine) - k]
            assert {j for j in kept if species[j] == sp} == set(far)
        assert [species[j] for _, j in src] == species


# -------------------------------------------------------- checks and selection
def test_min_distance_minimum_image():
    L = 10.0
    A = np.eye(3) * L
    pos = np.array([[0.1, 5, 5], [L - 0.1, 5, 5]])
    assert abs(de.min_distance(A, pos) - 0.2) < 1e-12
    # against explicit images over a wider range
    rng = np.random.default_rng(6)
    A = np.diag([9.0, 11.0, 10.0])
    pos = rng.uniform(0, 1, size=(6, 3)) @ A
    d = de.pair_distances(A, pos)
    k = 0
    for i in range(6):
        for j in range(i + 1, 6):
            best = min(np.linalg.norm(pos[i] - pos[j] + np.array([a, b, c]) @ A)
                       for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3))
            assert abs(d[k] - best) < 1e-12
            k += 1
    assert math.isinf(de.min_distance(A, pos[:1]))


def test_similarity_invariances():
    rng = np.random.default_rng(7)
    A = np.eye(3) * 40.0
    pa = rng.normal(size=(6, 3)) * 2 + 20
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    pb = (pa - 20) @ q.T + 20 + np.array([0.5, -0.3, 0.2])
    pb = pb[rng.permutation(6)]
    assert de.similarity(A, pa, pa) == 0.0
    assert de.similarity(A, pa, pb) < 1e-12
    pc = pa.copy()
    pc[0] += 1.0
    assert de.similarity(A, pa, pc) > 1e-3


def test_select():
    ep = [-1.0, -2.0, -3.0, -4.0]
    ec = [-1.5, -2.0, -2.5, -9.0]
    assert list(de.select(ep, ec, [True, True, True, False])) == [1, 0, 0, 0]


# ------------------------------------------------------------ initialisation
def test_init_positions_rules():
    A = np.diag([8.0, 9.0, 10.0])
    u = np.random.default_rng(8).random(300)
    # no distance check: every trial is kept and lands at its fractional point
    pos, used = de.init_positions(A, 5, 0, [0.0], 0.0, u)
    assert used == 15
    assert np.allclose(pos, u[:15].reshape(5, 3) @ A, atol=1e-14)
    # ball: inside the radius about the centre, distances respected
    pos, used = de.init_positions(A, 6, 1, [3.0], 2.0, u)
    assert np.all(np.linalg.norm(pos - A.sum(0) / 2, axis=1) <= 3.0 + 1e-12)
    assert de.min_distance(A, pos) >= 2.0 and used % 3 == 0 and used >= 18
    # slab: |z - centre| <= h
    pos, used = de.init_positions(A, 6, 2, [1.0], 1.5, u)
    assert np.all(np.abs(pos[:, 2] - 5.0) <= 1.0 + 1e-12)
    # running out of uniforms
    assert de.init_positions(A, 50, 1, [1.0], 2.0, u[:30]) is None


def test_jitter_cell():
    A = np.diag([8.0, 9.0, 10.0])
    B = de.jitter_cell(A, 0.1, [0.0, 0.5, 1.0])
    assert np.allclose(np.diag(B), [7.2, 9.0, 11.0], atol=1e-14)


def test_make_trials_fallback_and_draw_order():
    rng = np.random.default_rng(9)
    parents = [rng.normal(size=(5, 3)) * 2 + 10 for _ in range(5)]
    A = np.eye(3) * 20
    draws = {"r": np.array([[[(i + k + 1) % 5, (i + k + 2) % 5, (i + k + 3) % 5]
                             for k in range(2)] for i in range(5)]),
             "normal": rng.normal(size=(5, 2, 3)), "axis": rng.normal(size=(5, 2, 3)),
             "offset": rng.normal(size=(5, 2, 3)) * 0.3, "radius": np.full((5, 2), 2.0)}
    E = [-1.0, -2.0, -1.5, -3.0, -2.5]
    # an impossible distance requirement rejects every draw: parents come back
    tr, used = de.make_trials(parents, E, [0] * 5, A, draws, dmin=1e3)
    assert list(used) == [-1] * 5
    assert all(np.array_equal(a, b) for a, b in zip(tr, parents))
    # no checks: the first draw is always used and is the operators' result
    tr, used = de.make_trials(parents, E, [0] * 5, A, draws, crossover="sphere")
    assert list(used) == [0] * 5
    f = np.array(E) - min(E)
    r = draws["r"][2, 0]
    v = de.mutate_triangle(parents[r[0]], parents[r[1]], parents[r[2]], *f[r])
    child, _ = de.cross_sphere(v, parents[2], [0] * 5, draws["offset"][2][0], 2.0)
    assert np.array_equal(tr[2], child)
