"""Structure-search operators of the library (host code behind the C-ABI)
against the oracle on the same seeded draws: integer choices (which atoms,
which draw, selection) bit-exact, coordinates to 1e-12 bohr."""
import numpy as np
import pytest

from oracle import de

sgo = pytest.importorskip("paper_1603_02732_amd")
try:
    sgo.load_library()
except OSError as e:  # pragma: no cover
    pytest.skip(str(e), allow_module_level=True)

TOL = 1e-12


def test_mutation_parity():
    rng = np.random.default_rng(11)
    for trial in range(20):
        x1, x2, x3 = rng.normal(size=(3, 13, 3)) * 4
        f = rng.normal(size=3) * 10
        if trial == 0:
            f[:] = 0.0
        v = sgo.de_mutate(x1, x2, x3, f)
        assert np.abs(v - de.mutate_triangle(x1, x2, x3, *f)).max() < TOL
        v = sgo.de_mutate(x1, x2, x3, f, scheme=sgo.SGO_DE_CLASSIC, F=0.6)
        assert np.abs(v - de.mutate_classic(x1, x2, x3, 0.6)).max() < TOL


@pytest.mark.parametrize("species", [[0] * 13, [0] * 6 + [1] * 4 + [2] * 3])
def test_plane_parity(species):
    rng = np.random.default_rng(12)
    n = len(species)
    found = 0
    for trial in range(40):
        p1 = rng.normal(size=(n, 3)) * 3 + 12
        p2 = rng.normal(size=(n, 3)) * 3 + 11
        normal, axis = rng.normal(size=3), rng.normal(size=3)
        g = sgo.de_cross_plane(p1, p2, species, normal, axis)
        o = de.cross_plane(p1, p2, species, normal, axis)
        assert (g is None) == (o is None)
        if g is None:
            continue
        found += 1
        assert [tuple(int(v) for v in t) for t in g[1]] == o[1]
        assert np.abs(g[0] - o[0]).max() < TOL
        assert abs(g[2] - o[2]) < 1e-13
    assert found >= 10


@pytest.mark.parametrize("species", [[0] * 13, [1, 0] * 5 + [2, 2]])
def test_sphere_parity(species):
    rng = np.random.default_rng(13)
    n = len(species)
    for trial in range(40):
        p1 = rng.normal(size=(n, 3)) * 3 + 12
        p2 = rng.normal(size=(n, 3)) * 3 + 11
        t = rng.normal(size=3) * 0.5
        R = rng.uniform(0.0, 6.0)
        g = sgo.de_cross_sphere(p1, p2, species, t, R)
        o = de.cross_sphere(p1, p2, species, t, R)
        assert [tuple(int(v) for v in s) for s in g[1]] == o[1]
        assert np.abs(g[0] - o[0]).max() < TOL


def test_distance_similarity_parity():
    rng = np.random.default_rng(14)
    for A in (np.eye(3) * 12.0, np.array([[10.0, 0, 0], [3.0, 9.0, 0], [1.0, 2.0, 11.0]])):
        for trial in range(5):
            pa = rng.uniform(0, 1, size=(9, 3)) @ A
            pb = rng.uniform(0, 1, size=(9, 3)) @ A
            assert abs(sgo.de_min_distance(A, pa) - de.min_distance(A, pa)) < TOL
            assert abs(sgo.de_similarity(A, pa, pb) - de.similarity(A, pa, pb)) < TOL
    assert np.isinf(sgo.de_min_distance(np.eye(3), np.zeros((1, 3))))


@pytest.mark.parametrize("region,params,dmin", [(0, [0.0], 2.5), (1, [4.0], 2.0), (2, [1.5], 2.2)])
def test_init_parity(region, params, dmin):
    A = np.diag([12.0, 13.0, 14.0])
    for seed in range(4):
        u = np.random.default_rng(100 + seed).random(600)
        g = sgo.de_init_positions(A, 10, region, params, dmin, u)
        o = de.init_positions(A, 10, region, params, dmin, u)
        assert (g is None) == (o is None)
        if g is not None:
            assert g[1] == o[1]
            assert np.abs(g[0] - o[0]).max() < TOL
    # exhausted uniforms
    assert sgo.de_init_positions(A, 40, 1, [1.0], 2.0, u[:60]) is None


def test_jitter_parity():
    rng = np.random.default_rng(16)
    A = np.array([[10.0, 0, 0], [3.0, 9.0, 0], [1.0, 2.0, 11.0]])
    for trial in range(5):
        u = rng.random(3)
        assert np.abs(sgo.de_jitter_cell(A, 0.05, u) - de.jitter_cell(A, 0.05, u)).max() < TOL


def test_select_parity():
    rng = np.random.default_rng(15)
    ep = rng.normal(size=50)
    ec = ep + rng.normal(size=50) * 0.1
    ec[3] = ep[3]  # a tie keeps the parent
    st = np.zeros(50, dtype=np.int32)
    st[7] = sgo.SGO_ENOTCONV
    ok = st == 0
    assert np.array_equal(sgo.de_select(ep, ec, st), de.select(ep, ec, ok))
    assert np.array_equal(sgo.de_select(ep, ec), de.select(ep, ec, [True] * 50))


def test_invalid_arguments():
    lib = sgo.load_library()
    assert lib.sgo_de_mutate(3, None, None, None, 0.0, 0.0, 0.0, 0, 0.5, None) == sgo.SGO_EINVAL
    p = np.zeros((4, 3))
    p[:, 0] = [0, 1, 2, 3]
    with pytest.raises(sgo.SgoError):
        sgo.de_cross_plane(p, p, [0] * 4, [0, 0, 0], [0, 0, 1])  # zero normal
    with pytest.raises(sgo.SgoError):
        sgo.de_cross_plane(p, p, [0] * 4, [1, 0, 0], [2, 0, 0])  # axis along the normal
    with pytest.raises(sgo.SgoError):
        sgo.de_cross_sphere(p, p, [0] * 4, [0, 0, 0], -1.0)
