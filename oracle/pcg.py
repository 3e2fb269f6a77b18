"""Preconditioned CG relaxation with a force-fitted inverse-Hessian
preconditioner (oracle), the PCG option of Section 2.3.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 2.3: fit a classical force field to the DFT forces, take the Hessian
of the fitted energy by second-order finite differences, invert it on the
modes with non-zero eigenvalue, sum_j V_j V_j^T / tau_j (the three
translations have tau = 0), and use that as the preconditioner of a CG
relaxation; the fit may be renewed as the relaxation proceeds.

Readings (the paper names no force-field form or fit procedure):
  * force field: Morse pairs, E = sum_{i<j} D [(1 - e^{-a (r_ij - r0)})^2 - 1],
    minimum image over the 27 neighbouring cells, no cutoff;
  * fit: (D, a, r0) minimise the squared force error summed over every
    (positions, forces) sample of the relaxation so far; the forces are
    linear in D, so D is the least-squares optimum for each (a, r0) and must
    be positive; (a, r0) come from a grid, a = 0.5, 0.55, ..., 3.0 and
    r0 = r_min (0.80, 0.82, ..., 1.60) with r_min the smallest pair distance
    in the samples, refined by a compass search (moves of the current step
    along +-a, then +-r0, first improvement taken, steps halved when none
    improves, 30 halvings, starting from the grid spacing, moves that leave
    the grid's box not taken); defaults
    (0.1, 1.0, r_min) when no grid point gives D > 0;
  * Hessian: central second differences of the fitted energy with h = 1e-3
    bohr (diagonal: (E(+h) - 2E + E(-h)) / h^2; off-diagonal: the four-point
    formula / 4h^2);
  * preconditioner: modes with |tau| <= 1e-6 max|tau| (the translations)
    dropped; the others weighted 1 / max(|tau|, 0.1 max|tau|), so negative
    curvature counts by its magnitude and the preconditioner stays positive
    semi-definite (a CG preconditioner must not reverse a descent
    direction);
  * PCG step: d = P F + beta d_prev with beta = max(0, F_new.P(F_new - F) /
    F.P F); trial step alpha1 = min(1, 0.1 bohr / max_atom |d|) (the model's
    Newton step, capped by the trial displacement of the CG relaxation), at
    most twice the previous accepted step, then the
    secant step of the CG relaxation; the force field is refitted and P
    rebuilt every `refit` steps (0: only at the start).
"""
import copy
import math

import numpy as np

from .relax import evaluate


# ------------------------------------------------------------ force field
def _shifts(lattice):
    A = np.asarray(lattice, dtype=float)
    return np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)],
                    dtype=float) @ A


def _pairs(lattice, pos):
    """Minimum-image displacement r_i - r_j (+ shift) of every pair i < j."""
    sh = _shifts(lattice)
    pos = np.asarray(pos, dtype=float)
    out = []
    for i in range(len(pos)):
        for j in range(i + 1, len(pos)):
            d = pos[i] - pos[j] + sh
            k = int(np.argmin((d * d).sum(1)))
            out.append((i, j, d[k]))
    return out


def morse_energy(lattice, pos, D, a, r0):
    e = 0.0
    for _, _, d in _pairs(lattice, pos):
        r = math.sqrt(d @ d)
        x = 1.0 - math.exp(-a * (r - r0))
        e += D * (x * x - 1.0)
    return e


def morse_forces(lattice, pos, D, a, r0):
    """F_I = -dE/dR_I."""
    pos = np.asarray(pos, dtype=float)
    F = np.zeros_like(pos)
    for i, j, d in _pairs(lattice, pos):
        r = math.sqrt(d @ d)
        ex = math.exp(-a * (r - r0))
        dEdr = 2.0 * D * a * (1.0 - ex) * ex
        g = dEdr * d / r  # dE/dR_i
        F[i] -= g
        F[j] += g
    return F


# --------------------------------------------------------------------- fit
def _objective(samples, lattice, a, r0):
    """min over D of the squared force error; returns (value, D)."""
    gg = gf = ff = 0.0
    for pos, F in samples:
        g = morse_forces(lattice, pos, 1.0, a, r0)
        gg += float((g * g).sum())
        gf += float((g * F).sum())
        ff += float((np.asarray(F) ** 2).sum())
    if gg <= 0.0:
        return math.inf, 0.0
    D = gf / gg
    if D <= 0.0:
        return math.inf, D
    return ff - gf * gf / gg, D


def fit_morse(lattice, samples):
    """(D, a, r0) fitted to samples [(positions, forces)]."""
    rmin = min(min(math.sqrt(d @ d) for _, _, d in _pairs(lattice, p)) for p, _ in samples)
    best = (math.inf, None, None)
    for ia in range(51):
        a = 0.5 + 0.05 * ia
        for ir in range(41):
            r0 = rmin * (0.80 + 0.02 * ir)
            v, _ = _objective(samples, lattice, a, r0)
            if v < best[0]:
                best = (v, a, r0)
    if best[1] is None:
        return 0.1, 1.0, rmin
    v, a, r0 = best
    sa, sr = 0.05, 0.02 * rmin
    for _ in range(30):
        moved = True
        while moved:
            moved = False
            for da, dr in ((sa, 0.0), (-sa, 0.0), (0.0, sr), (0.0, -sr)):
                if not (0.5 <= a + da <= 3.0 and 0.8 * rmin <= r0 + dr <= 1.6 * rmin):
                    continue
                w, _ = _objective(samples, lattice, a + da, r0 + dr)
                if w < v:
                    v, a, r0 = w, a + da, r0 + dr
                    moved = True
                    break
        sa *= 0.5
        sr *= 0.5
    _, D = _objective(samples, lattice, a, r0)
    return D, a, r0


# ------------------------------------------------------ Hessian, preconditioner
def hessian_fd(lattice, pos, D, a, r0, h=1e-3):
    x0 = np.asarray(pos, dtype=float).reshape(-1)
    n = x0.size

    def E(x):
        return morse_energy(lattice, x.reshape(-1, 3), D, a, r0)

    H = np.zeros((n, n))
    e0 = E(x0)
    for i in range(n):
        ei = np.zeros(n)
        ei[i] = h
        H[i, i] = (E(x0 + ei) - 2.0 * e0 + E(x0 - ei)) / (h * h)
        for j in range(i + 1, n):
            ej = np.zeros(n)
            ej[j] = h
            v = (E(x0 + ei + ej) - E(x0 + ei - ej) - E(x0 - ei + ej) + E(x0 - ei - ej)) / (4 * h * h)
            H[i, j] = H[j, i] = v
    return H


def preconditioner(H, drop=1e-6, floor=0.1):
    tau, V = np.linalg.eigh(H)
    tmax = np.abs(tau).max()
    P = np.zeros_like(H)
    for j in range(len(tau)):
        if abs(tau[j]) <= drop * tmax:
            continue
        P += np.outer(V[:, j], V[:, j]) / max(abs(tau[j]), floor * tmax)
    return P


def build_preconditioner(lattice, samples, pos):
    D, a, r0 = fit_morse(lattice, samples)
    return preconditioner(hessian_fd(lattice, pos, D, a, r0)), (D, a, r0)


# ------------------------------------------------------------- relaxation
def pcg_beta(F_new, g_new, F_old, g_old):
    """Preconditioned Polak-Ribiere coefficient, g = P F:
    max(0, F_new.(g_new - g_old) / F_old.g_old) (0 when the denominator is
    not positive)."""
    den = float(np.sum(F_old * g_old))
    if den <= 0:
        return 0.0
    return max(0.0, float(np.sum(F_new * (g_new - g_old))) / den)


def pcg_core(evaluate_fn, x0, make_P, nsteps, refit=1):
    """PCG with the secant line search.  evaluate_fn(x) -> (E, F);
    make_P(samples, x) -> P [3n, 3n].  Returns (energies, x, F)."""
    x = np.array(x0, dtype=float)
    E, F = evaluate_fn(x)
    samples = [(x.copy(), F.copy())]
    P = make_P(samples, x)
    g = (P @ F.reshape(-1)).reshape(F.shape)
    d = g.copy()
    energies = [E]
    alpha_prev = 0.0
    for step in range(nsteps):
        dmax = np.linalg.norm(d, axis=1).max()
        a1 = min(1.0, 0.1 / dmax) if dmax > 0 else 0.0
        if alpha_prev > 0:
            a1 = min(a1, 2 * alpha_prev)
        s0 = -np.sum(F * d)
        _, F1 = evaluate_fn(x + a1 * d)
        s1 = -np.sum(F1 * d)
        a2 = a1 * s0 / (s0 - s1) if s1 - s0 > 0 else 4 * a1
        a2 = min(4 * a1, max(0.1 * a1, a2))
        alpha_prev = a2
        x = x + a2 * d
        E, F2 = evaluate_fn(x)
        samples.append((x.copy(), F2.copy()))
        if refit > 0 and (step + 1) % refit == 0:
            P = make_P(samples, x)
        g2 = (P @ F2.reshape(-1)).reshape(F2.shape)
        beta = pcg_beta(F2, g2, F, (P @ F.reshape(-1)).reshape(F.shape))
        d = g2 + beta * d
        F = F2
        energies.append(E)
    return np.array(energies), x, F


def relax_pcg(system, nsteps, refit=1, **kw):
    lat = np.asarray(system["lattice"], dtype=float)

    def ev(x):
        return evaluate(system, x, **kw)

    def make_P(samples, x):
        return build_preconditioner(lat, samples, x)[0]

    return pcg_core(ev, system["positions"], make_P, nsteps, refit)
