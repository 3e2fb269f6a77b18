"""Pins of oracle parts that the self-consistency checks (finite-difference
forces and stress, virial traces, rotation covariance) cannot see, because a
wrong constant there changes the functional and its derivatives together:

* the l = 1 real harmonics of the Kleinman-Bylander projectors: the
  addition theorem sum_m Y_1m^2 = 3/(4 pi) and unit norm on the sphere;
* the Perdew-Zunger correlation: the high-density coefficient A equals the
  exact (1 - ln 2)/pi^2, and the two branches meet with equal slope at
  r_s = 1 (the conditions that fixed C and D);
* the Hartree energy and potential: one Gaussian charge in a periodic cubic
  box against the closed form from the Ewald identity;
* the CG and PCG direction updates: n-step termination on an n-dimensional
  quadratic with exact line searches.

Each pin is written as a check that returns its error, and every check is
also run on a copy of the oracle with one constant or factor moved by 1 %,
which it must reject."""
import math

import numpy as np
import pytest

from oracle import lda, pseudo, relax, pcg
from oracle.hamiltonian import Setup
from oracle.scf import potentials, energy_terms
from workloads import make_system

# ---------------------------------------------------------------- Y_1m

def _sphere_quadrature(nmu=24, nphi=48):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi: exact
    for the polynomials of degree < 2 nmu in the direction cosines."""
    mu, wmu = np.polynomial.legendre.leggauss(nmu)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    s = np.sqrt(1 - M * M)
    dirs = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
    w = (wmu[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return dirs, w


def ylm_errors(ylm):
    """Largest errors of (addition theorem, orthonormality on the sphere) of
    ylm(1, G) over random and quadrature directions; lengths of G vary, so a
    dependence on |G| shows as well."""
    rng = np.random.default_rng(11)
    G = rng.normal(size=(200, 3)) * rng.uniform(0.2, 9.0, size=(200, 1))
    Y = ylm(1, G)
    add = np.abs((Y * Y).sum(0) - 3 / (4 * np.pi)).max()
    dirs, w = _sphere_quadrature()
    Yq = ylm(1, dirs * 2.7)
    gram = (Yq * w[None, :]) @ Yq.T
    Y0 = ylm(0, dirs)
    gram0 = (Y0 * w[None, :]) @ Y0.T
    orth = max(np.abs(gram - np.eye(3)).max(), abs(gram0[0, 0] - 1))
    return add, orth


def test_real_harmonics_addition_theorem_and_norm():
    add, orth = ylm_errors(pseudo.real_ylm)
    assert add < 1e-14 and orth < 1e-13


def test_real_harmonics_pin_rejects_a_one_percent_factor():
    bad = lambda l, G: pseudo.real_ylm(l, G) * (1.01 if l == 1 else 1.0)
    add, orth = ylm_errors(bad)
    assert add > 1e-3 and orth > 1e-3


def test_p_projectors_sum_to_the_radial_transform():
    # sum_m |beta_1m(G)|^2 = p_1(|G|)^2 (3/4pi) / Omega for the p channel of
    # one atom, as the oracle builds the projector columns (the radial part
    # p_1 is pinned by quadrature in test_oracle_lda_pseudo)
    lat = np.diag([9.0, 8.0, 10.0])
    s = make_system("p", lat, ["Si-G"], [[1.1, 2.0, 3.3]], 6.0, (24, 24, 24), 4,
                    {"kind": "fixed"})
    st = Setup(s)
    ch = [c for c in s["species"]["Si-G"]["kb"] if c["l"] == 1][0]
    cols = [k for k in range(st.beta.shape[1]) if k >= 1]  # s first, then p (x, y, z)
    assert len(cols) == 3
    lhs = (np.abs(st.beta[:, cols]) ** 2).sum(1)
    g = np.sqrt(st.g2)
    rhs = pseudo.projector_ft(1, ch["r"], g) ** 2 * 3 / (4 * np.pi) / st.omega
    assert np.abs(lhs - rhs).max() < 1e-12 * rhs.max()


# ---------------------------------------------------------------- PZ-81

EXCH = -0.75 * (3 / np.pi) ** (1 / 3)  # Dirac exchange: eps_x = EXCH rho^(1/3)


def _eps_c(rs):
    rho = 3 / (4 * np.pi * np.asarray(rs, dtype=float) ** 3)
    eps, _ = lda.pz81(rho)
    return eps - EXCH * rho ** (1 / 3)


def pz_errors():
    """(error of A against (1 - ln 2)/pi^2, slope step at r_s = 1, value
    step at r_s = 1).  A is read from the r_s < 1 branch of the oracle's
    eps_c by its limit: eps_c(r) - eps_c(r/e) -> A as r -> 0 (the other
    terms vanish with r)."""
    r = np.array([1e-7])
    a_est = float(_eps_c(r)[0] - _eps_c(r / np.e)[0])
    err_a = abs(a_est - (1 - math.log(2)) / math.pi ** 2)
    d, h = 1e-5, 1e-7
    lo = (_eps_c([1 - d + h])[0] - _eps_c([1 - d - h])[0]) / (2 * h)
    hi = (_eps_c([1 + d + h])[0] - _eps_c([1 + d - h])[0]) / (2 * h)
    slope = abs(lo - hi)
    value = abs(_eps_c([1 - 1e-12])[0] - _eps_c([1.0])[0])
    return err_a, slope, value


def test_pz_high_density_coefficient_and_continuity():
    err_a, slope, value = pz_errors()
    assert err_a < 1e-5
    # continuity of eps_c and d eps_c / d r_s at r_s = 1 is what fixed C and
    # D; the published four-digit rounding leaves a 1.3e-5 slope step and the
    # 3.2e-5 value step pinned in test_oracle_lda_pseudo
    assert slope < 2e-5
    assert abs(value - 3.2e-5) < 2e-7


@pytest.mark.parametrize("name,factor", [
    ("A_", 1.01), ("A_", 0.99), ("B_", 1.01), ("B_", 0.99), ("C_", 1.01),
    ("D_", 1.01), ("D_", 0.99), ("GAMMA", 1.01), ("BETA1", 0.99), ("BETA2", 1.01)])
def test_pz_pins_reject_a_one_percent_constant(monkeypatch, name, factor):
    # C - 1 % stays inside the slope pin: continuity fixes C only to the
    # published rounding (C in [0.001967, 0.002007])
    monkeypatch.setattr(lda, name, getattr(lda, name) * factor)
    err_a, slope, value = pz_errors()
    assert err_a >= 1e-5 or slope >= 2e-5 or abs(value - 3.2e-5) >= 2e-7


# ---------------------------------------------------------------- Hartree

SC_MADELUNG = -0.880059  # point charge in a neutralising background, simple cubic, per ion / r_s


def _gaussian_box(Q, sigma, L, N):
    s = make_system("gauss", np.eye(3) * L, [], np.zeros((0, 3)), 1.0, (N, N, N), 1,
                    {"kind": "fixed"})
    s["nelec"] = 0.0
    st = Setup(s)
    x = np.arange(N) * L / N
    X, Y, Zc = np.meshgrid(x, x, x, indexing="ij")
    c = np.array([0.37, 0.52, 0.61]) * L
    rho = np.zeros((N, N, N))
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                r2 = ((X - c[0] + i * L) ** 2 + (Y - c[1] + j * L) ** 2
                      + (Zc - c[2] + k * L) ** 2)
                rho += np.exp(-0.5 * r2 / sigma ** 2)
    rho *= Q / (2 * np.pi * sigma ** 2) ** 1.5
    return st, rho


def hartree_errors(st, rho, Q, sigma, L):
    """E_H of the periodic Gaussian charge from the oracle's energy terms
    and from its potential, against the closed form
    E_H = Q^2/(2 sqrt(pi) sigma) + M_sc Q^2/r_s + 2 pi Q^2 sigma^2 / Omega
    (the Ewald identity at eta = 1/(2 sigma); the real-space sum vanishes
    for L >> sigma)."""
    omega = L ** 3
    rs = (3 * omega / (4 * np.pi)) ** (1 / 3)
    exact = (Q * Q / (2 * math.sqrt(math.pi) * sigma) + SC_MADELUNG * Q * Q / rs
             + 2 * math.pi * Q * Q * sigma ** 2 / omega)
    terms = energy_terms(st, np.zeros((st.npw, 0), complex), np.zeros(0), rho)
    _, parts = potentials(st, rho)
    e_pot = 0.5 * omega / st.ntot * float((parts["vh"] * rho).sum())
    return abs(terms["hartree"] - exact), abs(e_pot - exact), exact


@pytest.fixture(scope="module")
def gauss_box():
    Q, sigma, L = 2.0, 0.7, 12.0
    st, rho = _gaussian_box(Q, sigma, L, 40)
    return st, rho, Q, sigma, L


def test_hartree_of_a_gaussian_charge(gauss_box):
    st, rho, Q, sigma, L = gauss_box
    # the charge integrates to Q on the grid (rho sampled, not projected)
    assert abs(rho.sum() * L ** 3 / st.ntot - Q) < 1e-12
    e1, e2, exact = hartree_errors(st, rho, Q, sigma, L)
    assert exact > 1.0
    assert e1 < 2e-6 and e2 < 2e-6  # the constant M_sc is known to 6 digits


def test_hartree_pin_rejects_a_one_percent_prefactor(gauss_box, monkeypatch):
    st, rho, Q, sigma, L = gauss_box
    # the oracle's 4 pi / G^2 kernel scaled by 1.01: the Coulomb kernel lives
    # in the G^2 grid that potentials() and energy_terms() divide by
    monkeypatch.setattr(st, "g2grid", st.g2grid / 1.01)
    e1, e2, _ = hartree_errors(st, rho, Q, sigma, L)
    assert e1 > 1e-3 and e2 > 1e-3


# ---------------------------------------------------------------- CG / PCG

def _quadratic(seed, n_atoms, lo, hi):
    rng = np.random.default_rng(seed)
    m = 3 * n_atoms
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)))
    lam = np.linspace(lo, hi, m)
    K = Q @ np.diag(lam) @ Q.T
    xs = rng.normal(size=(n_atoms, 3))
    x0 = xs + 0.08 * rng.normal(size=(n_atoms, 3))
    return K, xs, x0


def cg_termination_error(monkeypatch, beta_scale=1.0):
    """|x_n - x*| / |x_0 - x*| after n = 3 n_atoms steps of the oracle's CG
    relaxation on E = (x - x*)^T K (x - x*)/2 (distinct eigenvalues, so the
    Krylov space needs all n steps).  The secant step is exact on a
    quadratic and the clamps stay inactive for these sizes, so Polak-Ribiere
    CG (= Fletcher-Reeves here) terminates in n steps."""
    K, xs, x0 = _quadratic(21, 2, 1.0, 3.0)
    n = K.shape[0]

    def ev(system, x, **kw):
        dx = (np.asarray(x) - xs).reshape(-1)
        return 0.5 * dx @ K @ dx, -(K @ dx).reshape(xs.shape)

    monkeypatch.setattr(relax, "evaluate", ev)
    if beta_scale != 1.0:
        beta = relax.pr_beta
        monkeypatch.setattr(relax, "pr_beta", lambda a, b: beta_scale * beta(a, b))
    E, x, F = relax.relax_cg({"positions": x0.tolist()}, n)
    return np.linalg.norm(x - xs) / np.linalg.norm(x0 - xs)


def test_cg_relaxation_terminates_in_n_steps(monkeypatch):
    assert cg_termination_error(monkeypatch) < 1e-9


def test_cg_pin_rejects_a_one_percent_beta(monkeypatch):
    assert cg_termination_error(monkeypatch, 1.01) > 1e-6


def pcg_termination_error(monkeypatch, beta_scale=1.0):
    """Same for the PCG core with a fixed SPD preconditioner P that is not
    K^-1: preconditioned CG with exact line searches terminates in n steps."""
    K, xs, x0 = _quadratic(22, 2, 1.0, 3.0)
    n = K.shape[0]
    rng = np.random.default_rng(23)
    Qp, _ = np.linalg.qr(rng.normal(size=(n, n)))
    P = Qp @ np.diag(np.linspace(0.6, 1.2, n)) @ Qp.T

    def ev(x):
        dx = (np.asarray(x) - xs).reshape(-1)
        return 0.5 * dx @ K @ dx, -(K @ dx).reshape(xs.shape)

    if beta_scale != 1.0:
        beta = pcg.pcg_beta
        monkeypatch.setattr(pcg, "pcg_beta", lambda *a: beta_scale * beta(*a))
    E, x, F = pcg.pcg_core(ev, x0, lambda samples, x: P, n, refit=0)
    return np.linalg.norm(x - xs) / np.linalg.norm(x0 - xs)


def test_pcg_relaxation_terminates_in_n_steps(monkeypatch):
    assert pcg_termination_error(monkeypatch) < 1e-9


def test_pcg_pin_rejects_a_one_percent_beta(monkeypatch):
    assert pcg_termination_error(monkeypatch, 1.01) > 1e-6
