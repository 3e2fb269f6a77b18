"""Conventional conjugate-gradient relaxation (oracle), one of the local
relaxation options of Section 2.3.

Polak-Ribiere directions from the Hellmann-Feynman forces and a secant line
search on the directional derivative s(alpha) = -F(x + alpha d).d:
  trial step   alpha1 = 0.1 bohr / max_atom |d|, at most twice the previous
               accepted step
  secant step  alpha2 = alpha1 s(0) / (s(0) - s(alpha1)), clamped to
               [0.1 alpha1, 4 alpha1] (4 alpha1 when s does not increase)
  accept x + alpha2 d;  d <- F_new + max(0, F_new.(F_new - F) / F.F) d.
Each step costs two self-consistent evaluations.
"""
import copy

import numpy as np

from .scf import run_scf
from .forces import hf_forces


def evaluate(system, positions, **kw):
    s = copy.deepcopy(system)
    s["positions"] = np.asarray(positions).tolist()
    r = run_scf(s, **kw)
    F, _ = hf_forces(r)
    return r["energy"], F


def pr_beta(F_new, F_old):
    """Polak-Ribiere coefficient of the next direction, clipped at zero."""
    return max(0.0, np.sum(F_new * (F_new - F_old)) / np.sum(F_old * F_old))


def relax_cg(system, nsteps, **kw):
    x = np.array(system["positions"], dtype=float)
    E, F = evaluate(system, x, **kw)
    d = F.copy()
    energies = [E]
    alpha_prev = 0.0
    for _ in range(nsteps):
        dmax = np.linalg.norm(d, axis=1).max()
        a1 = 0.1 / dmax if dmax > 0 else 0.0
        if alpha_prev > 0:
            a1 = min(a1, 2 * alpha_prev)
        s0 = -np.sum(F * d)
        _, F1 = evaluate(system, x + a1 * d, **kw)
        s1 = -np.sum(F1 * d)
        a2 = a1 * s0 / (s0 - s1) if s1 - s0 > 0 else 4 * a1
        a2 = min(4 * a1, max(0.1 * a1, a2))
        alpha_prev = a2
        x = x + a2 * d
        E, F2 = evaluate(system, x, **kw)
        beta = pr_beta(F2, F)
        d = F2 + beta * d
        F = F2
        energies.append(E)
    return np.array(energies), x, F
