"""Curved line search relaxation (oracle), the CLS option of Section 2.3.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 2.3 describes CLS in outline: fit a classical force field to the
DFT forces, let the fitted field define a guided curve from the current
structure towards its own minimum, minimise the DFT energy along that
curve, and repeat.  The steps below are a re-derivation from that outline
(the paper defers the details to another publication).

Readings:
  * force field and fit: the Morse pair form and fit of the PCG option
    (`oracle.pcg.fit_morse`), refitted before every step to every
    (positions, DFT forces) sample of the relaxation so far;
  * guided curve: the steepest-descent path of the fitted energy, traced
    with steps that move the most-forced atom by h = 0.02 bohr,
    x_{k+1} = x_k + h F_FF(x_k) / max_atom |F_FF(x_k)|, until
    max_atom |F_FF| < 1e-3 Ha/bohr or 200 steps; the curve is the polyline
    through x_0 .. x_K parametrised by s = k h (+ the fraction of a segment),
    so s bounds the largest atom displacement along the way;
  * DFT line minimisation along the curve: g(s) = dE/ds = -F(x(s)).x'(s)
    with x' the tangent of the segment holding s (the first segment's at
    s = 0); trial s1 = min(s_end, 0.3 bohr), at most twice the previous
    accepted s; secant s2 = s1 g(0) / (g(0) - g(s1)) when g increases,
    else 4 s1, clamped to [0.1 s1, 4 s1] and to the curve's end; the
    structure moves to x(s2).  Two DFT evaluations per step, as CG.
  * a curve of zero length (the fitted field already at rest) falls back to
    a step along the DFT forces: the two-point curve x_0, x_0 + h F / max|F|.
"""
import numpy as np

from .pcg import fit_morse, morse_forces
from .relax import evaluate

H_STEP = 0.02
F_TOL = 1e-3
K_MAX = 200
S_CAP = 0.3


def guided_curve(lattice, params, x0, h=H_STEP, ftol=F_TOL, kmax=K_MAX):
    """Nodes [K+1, natoms, 3] of the fitted field's steepest-descent path."""
    x = np.array(x0, dtype=float)
    nodes = [x.copy()]
    for _ in range(kmax):
        F = morse_forces(lattice, x, *params)
        fm = np.linalg.norm(F, axis=1).max()
        if fm < ftol:
            break
        x = x + h * F / fm
        nodes.append(x.copy())
    return np.array(nodes)


def curve_point(nodes, s, h=H_STEP):
    """x(s) on the polyline and the tangent dx/ds of the segment holding s."""
    K = len(nodes) - 1
    k = min(int(np.floor(s / h)), K - 1)
    k = max(k, 0)
    t = s / h - k
    tang = (nodes[k + 1] - nodes[k]) / h
    return nodes[k] + t * (nodes[k + 1] - nodes[k]), tang


def cls_core(evaluate_fn, x0, fit_fn, lattice, nsteps):
    """CLS with the curve of the field fitted by fit_fn(samples) -> params.
    evaluate_fn(x) -> (E, F).  Returns (energies, x, F)."""
    x = np.array(x0, dtype=float)
    E, F = evaluate_fn(x)
    samples = [(x.copy(), F.copy())]
    energies = [E]
    s_prev = 0.0
    for _ in range(nsteps):
        params = fit_fn(samples)
        nodes = guided_curve(lattice, params, x)
        if len(nodes) < 2:
            fm = np.linalg.norm(F, axis=1).max()
            nodes = np.array([x, x + H_STEP * F / fm]) if fm > 0 else np.array([x, x])
        s_end = H_STEP * (len(nodes) - 1)
        _, t0 = curve_point(nodes, 0.0)
        g0 = -np.sum(F * t0)
        s1 = min(s_end, S_CAP)
        if s_prev > 0:
            s1 = min(s1, 2 * s_prev)
        x1, t1 = curve_point(nodes, s1)
        _, F1 = evaluate_fn(x1)
        g1 = -np.sum(F1 * t1)
        s2 = s1 * g0 / (g0 - g1) if g1 - g0 > 0 else 4 * s1
        s2 = min(4 * s1, max(0.1 * s1, s2))
        s2 = min(s2, s_end)
        s_prev = s2
        x, _ = curve_point(nodes, s2)
        E, F = evaluate_fn(x)
        samples.append((x.copy(), F.copy()))
        energies.append(E)
    return np.array(energies), x, F


def relax_cls(system, nsteps, **kw):
    lat = np.asarray(system["lattice"], dtype=float)

    def ev(x):
        return evaluate(system, x, **kw)

    return cls_core(ev, system["positions"], lambda smp: fit_morse(lat, smp), lat, nsteps)
