"""Force-fitted preconditioner of the library (host code behind the C-ABI)
against the oracle: Morse energy and forces to rounding, the analytic Hessian
against the oracle's second differences (their truncation error), the fit
and the preconditioner to 1e-7."""
import numpy as np
import pytest

from oracle import pcg
import workloads

sgo = pytest.importorskip("paper_1603_02732_amd")
try:
    sgo.load_library()
except OSError as e:  # pragma: no cover
    pytest.skip(str(e), allow_module_level=True)


def _configs():
    out = []
    for seed in range(3):
        lat, pos = workloads.cluster_ball(9, 20.0, 4.0, 2.6, 300 + seed)
        out.append((lat, pos))
    lat, pos = workloads.diamond_cells(10.26, (1, 1, 1), 0.2, 7)  # periodic images
    out.append((lat, pos))
    return out


def test_morse_parity():
    for lat, pos in _configs():
        prm = (0.21, 1.25, 2.7)
        e, F = sgo.ff_morse(lat, pos, prm)
        assert abs(e - pcg.morse_energy(lat, pos, *prm)) < 1e-12 * max(1.0, abs(e))
        assert np.abs(F - pcg.morse_forces(lat, pos, *prm)).max() < 1e-13


def test_hessian_parity():
    for lat, pos in _configs()[:2] + _configs()[3:]:
        prm = (0.21, 1.25, 2.7)
        H = sgo.ff_hessian(lat, pos, prm)
        Ho = pcg.hessian_fd(lat, pos, *prm)
        assert np.abs(H - H.T).max() == 0.0
        assert np.abs(H - Ho).max() < 1e-5 * np.abs(H).max()


def test_fit_parity():
    rng = np.random.default_rng(21)
    cfg = _configs()
    lat, pos = cfg[0]
    cases = [[(pos, pcg.morse_forces(lat, pos, 0.15, 1.7, 2.9))],
             [(pos, 0.05 * rng.normal(size=pos.shape)),
              (pos + 0.1 * rng.normal(size=pos.shape), 0.05 * rng.normal(size=pos.shape))],
             [(cfg[3][1], 0.03 * rng.normal(size=cfg[3][1].shape))]]
    lats = [lat, lat, cfg[3][0]]
    for L, samples in zip(lats, cases):
        po = np.array(pcg.fit_morse(L, samples))
        pg = sgo.ff_fit(L, [s[0] for s in samples], [s[1] for s in samples])
        assert np.abs(pg - po).max() < 1e-7 * np.abs(po).max(), (pg, po)


def test_preconditioner_parity():
    for lat, pos in _configs()[:2]:
        H = pcg.hessian_fd(lat, pos, 0.21, 1.25, 2.7)
        P = sgo.ff_preconditioner(H)
        Po = pcg.preconditioner(H)
        assert np.abs(P - Po).max() < 1e-9 * np.abs(Po).max()


def test_guided_curve_parity():
    from oracle import cls
    for lat, pos in _configs():
        for prm in ((0.21, 1.25, 2.7), (0.05, 0.8, 3.3)):
            g = sgo.ff_guided_curve(lat, pos, prm)
            o = cls.guided_curve(lat, prm, pos)
            # same node count; rounding differences of the force sums grow
            # along a 200-step descent (an iterated map), to ~1e-8 bohr here
            assert g.shape == o.shape
            assert np.abs(g - o).max() < 1e-6
