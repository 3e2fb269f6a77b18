"""Pins of the force-fitted PCG preconditioner of the oracle (Section 2.3):
Morse forces against finite differences of the energy, the dimer's Hessian
in closed form, translation invariance, recovery of known force-field
parameters, the spectral rules of the preconditioner, and the one-step
convergence of PCG on a quadratic with its exact inverse Hessian."""
import math

import numpy as np

from oracle import pcg

BOX = np.eye(3) * 30.0


def _cluster(n, seed, spread=2.2):
    rng = np.random.default_rng(seed)
    pts = [np.full(3, 15.0)]
    while len(pts) < n:
        p = 15.0 + rng.normal(size=3) * spread
        if min(np.linalg.norm(p - q) for q in pts) > 2.0:
            pts.append(p)
    return np.array(pts)


def test_forces_are_minus_energy_gradient():
    pos = _cluster(6, 1)
    prm = (0.3, 1.4, 2.6)
    F = pcg.morse_forces(BOX, pos, *prm)
    h = 1e-5
    for i in range(6):
        for k in range(3):
            p, m = pos.copy(), pos.copy()
            p[i, k] += h
            m[i, k] -= h
            g = (pcg.morse_energy(BOX, p, *prm) - pcg.morse_energy(BOX, m, *prm)) / (2 * h)
            assert abs(F[i, k] + g) < 1e-8
    assert np.abs(F.sum(0)).max() < 1e-12  # pair forces cancel


def test_dimer_hessian_closed_form():
    D, a, r0 = 0.25, 1.3, 2.8
    # at the minimum: one bond mode 2 V''(r0) = 4 D a^2, five zero modes
    pos = np.array([[14.0, 15.0, 15.0], [14.0 + r0, 15.0, 15.0]])
    tau = np.linalg.eigvalsh(pcg.hessian_fd(BOX, pos, D, a, r0))
    assert abs(tau[-1] - 4 * D * a * a) < 1e-5 * 4 * D * a * a
    assert np.abs(tau[:5]).max() < 1e-5
    # stretched to r: bond mode 2 V''(r), two rotations 2 V'(r)/r
    r = 3.4
    pos = np.array([[14.0, 15.0, 15.0], [14.0 + r, 15.0, 15.0]])
    e = math.exp(-a * (r - r0))
    v1 = 2 * D * a * (1 - e) * e
    v2 = 2 * D * a * a * e * (2 * e - 1)
    tau = np.sort(np.linalg.eigvalsh(pcg.hessian_fd(BOX, pos, D, a, r0)))
    want = np.sort([0, 0, 0, 2 * v1 / r, 2 * v1 / r, 2 * v2])
    assert np.abs(tau - want).max() < 1e-5


def test_hessian_translation_invariance():
    pos = _cluster(5, 2)
    H = pcg.hessian_fd(BOX, pos, 0.2, 1.2, 2.5)
    for k in range(3):
        t = np.zeros((5, 3))
        t[:, k] = 1.0
        assert np.abs(H @ t.reshape(-1)).max() < 1e-5 * np.abs(H).max()
    assert np.abs(H - H.T).max() == 0.0


def test_fit_recovers_known_parameters():
    prm = (0.17, 1.6, 2.9)
    samples = []
    for s in range(2):
        pos = _cluster(7, 10 + s)
        samples.append((pos, pcg.morse_forces(BOX, pos, *prm)))
    D, a, r0 = pcg.fit_morse(BOX, samples)
    assert abs(D - prm[0]) < 1e-6 and abs(a - prm[1]) < 1e-6 and abs(r0 - prm[2]) < 1e-6


def test_preconditioner_spectral_rules():
    # a symmetric matrix with exact translation modes (tau = 0), negative
    # curvature and modes below the floor
    n = 6
    rng = np.random.default_rng(4)
    T = np.zeros((3 * n, 3))
    for k in range(3):
        T[k::3, k] = 1.0 / math.sqrt(n)
    Q, _ = np.linalg.qr(np.hstack([T, rng.normal(size=(3 * n, 3 * n - 3))]))
    tau = np.concatenate([[0.0, 0.0, 0.0], [-0.4, -0.01, 0.001, 0.2, 0.25],
                          rng.uniform(0.1, 3.0, size=3 * n - 8)])
    H = Q @ np.diag(tau) @ Q.T
    P = pcg.preconditioner(H)
    tmax = np.abs(tau).max()
    for k in range(3):  # translations annihilated
        assert np.abs(P @ T[:, k]).max() < 1e-12 * np.abs(P).max()
    for j in range(3, 3 * n):  # kept modes scaled by 1 / max(|tau|, 0.1 max|tau|)
        v = Q[:, j]
        assert np.allclose(P @ v, v / max(abs(tau[j]), 0.1 * tmax), atol=1e-10 * np.abs(P).max())
    assert np.linalg.eigvalsh(P).min() > -1e-12 * np.abs(P).max()  # positive semi-definite


def test_pcg_is_exact_in_one_step_on_a_quadratic():
    rng = np.random.default_rng(5)
    n = 4
    Q, _ = np.linalg.qr(rng.normal(size=(3 * n, 3 * n)))
    K = Q @ np.diag(rng.uniform(0.5, 3.0, size=3 * n)) @ Q.T
    xs = rng.normal(size=(n, 3))

    def ev(x):
        dx = (x - xs).reshape(-1)
        return 0.5 * dx @ K @ dx, -(K @ dx).reshape(n, 3)

    x0 = xs + 0.02 * rng.normal(size=(n, 3))
    E, x, F = pcg.pcg_core(ev, x0, lambda samples, x: np.linalg.inv(K), 1, refit=0)
    assert np.abs(x - xs).max() < 1e-12
    assert E[-1] < 1e-20


def test_cg_secant_step_is_the_line_minimum_on_a_quadratic(monkeypatch):
    # On a quadratic the directional derivative is linear along d, so the
    # secant step of the CG relaxation lands on the exact line minimum:
    # F_new . d = 0 after each step (while the step stays inside its clamps).
    from oracle import relax
    rng = np.random.default_rng(6)
    n = 3
    Q, _ = np.linalg.qr(rng.normal(size=(3 * n, 3 * n)))
    K = Q @ np.diag(rng.uniform(2.0, 4.0, size=3 * n)) @ Q.T
    xs = rng.normal(size=(n, 3))
    seen = []

    def ev(system, x, **kw):
        dx = (np.asarray(x) - xs).reshape(-1)
        seen.append(np.array(x, dtype=float))
        return 0.5 * dx @ K @ dx, -(K @ dx).reshape(n, 3)

    monkeypatch.setattr(relax, "evaluate", ev)
    x0 = xs + 0.05 * rng.normal(size=(n, 3))
    E, x, F = relax.relax_cg({"positions": x0.tolist()}, 1)
    d = -(K @ (x0 - xs).reshape(-1)).reshape(n, 3)  # first direction = F(x0)
    a1 = 0.1 / np.linalg.norm(d, axis=1).max()
    astar = np.sum(d * d) / (d.reshape(-1) @ K @ d.reshape(-1))  # exact line minimum
    assert 0.1 * a1 < astar < 4 * a1  # inside the clamps
    assert np.abs(x - (x0 + astar * d)).max() < 1e-12
    assert abs(np.sum(F * d)) < 1e-10 * np.sum(d * d)
    assert E[1] < E[0]


def test_fit_stays_in_the_search_box():
    rng = np.random.default_rng(7)
    pos = _cluster(5, 8)
    rmin = min(np.linalg.norm(pos[i] - pos[j]) for i in range(5) for j in range(i + 1, 5))
    for trial in range(3):
        D, a, r0 = pcg.fit_morse(BOX, [(pos, 0.05 * rng.normal(size=pos.shape))])
        assert 0.5 <= a <= 3.0 and 0.8 * rmin - 1e-12 <= r0 <= 1.6 * rmin + 1e-12
        assert D > 0 or (D, a) == (0.1, 1.0)
