"""Pins of the curved-line-search relaxation of the oracle (Section 2.3, CLS
re-derived): the guided curve of a Morse dimer runs along the bond to the
pair minimum, the polyline parametrisation is continuous with unit largest
displacement rate, and on an energy surface that is itself the fitted field
the relaxation descends monotonically to its minimum."""
import math

import numpy as np

from oracle import cls, pcg

BOX = np.eye(3) * 30.0


def test_dimer_curve_runs_along_the_bond_to_the_minimum():
    D, a, r0 = 0.3, 1.2, 2.6
    x0 = np.array([[13.0, 15.0, 15.0], [13.0 + 3.4, 15.0, 15.0]])
    nodes = cls.guided_curve(BOX, (D, a, r0), x0)
    assert len(nodes) > 2
    # both atoms move along x only, symmetrically, h per node (equal forces)
    assert np.abs(nodes[:, :, 1:] - x0[None, :, 1:]).max() < 1e-14
    step = np.abs(np.diff(nodes[:, 0, 0]))
    assert np.allclose(step, cls.H_STEP, atol=1e-14)
    assert np.allclose(nodes[:, 0, 0] + nodes[:, 1, 0], x0[0, 0] + x0[1, 0], atol=1e-12)
    # it stops within one node (2h of separation) of r0, where |F| < ftol or the sign flips
    r_end = nodes[-1, 1, 0] - nodes[-1, 0, 0]
    assert abs(r_end - r0) < 2 * cls.H_STEP + 1e-12


def test_curve_parametrisation():
    rng = np.random.default_rng(3)
    x0 = 15.0 + rng.normal(size=(5, 3)) * 1.8
    nodes = cls.guided_curve(BOX, (0.2, 1.3, 2.5), x0)
    h = cls.H_STEP
    for k in range(len(nodes) - 1):
        p, t = cls.curve_point(nodes, k * h)
        assert np.abs(p - nodes[k]).max() < 1e-12
        # the most-forced atom moves at unit rate along the curve
        assert abs(np.linalg.norm(t, axis=1).max() - 1.0) < 1e-12
    p, _ = cls.curve_point(nodes, h * (len(nodes) - 1))
    assert np.abs(p - nodes[-1]).max() < 1e-12


def test_cls_descends_on_its_own_field():
    prm = (0.25, 1.4, 2.6)
    rng = np.random.default_rng(4)
    pts = [np.full(3, 15.0)]
    while len(pts) < 5:
        q = 15.0 + rng.normal(size=3) * 1.6
        if min(np.linalg.norm(q - p) for p in pts) > 2.2:
            pts.append(q)
    x0 = np.array(pts)

    def ev(x):
        return pcg.morse_energy(BOX, x, *prm), pcg.morse_forces(BOX, x, *prm)

    E, x, F = cls.cls_core(ev, x0, lambda samples: prm, BOX, 6)
    assert np.all(np.diff(E) < 1e-12)  # monotone descent
    F0 = pcg.morse_forces(BOX, x0, *prm)
    assert np.linalg.norm(F, axis=1).max() < 0.2 * np.linalg.norm(F0, axis=1).max()
