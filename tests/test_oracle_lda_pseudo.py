"""Pins of the LDA and analytic pseudopotential transforms: closed-form
exchange constant, v_xc = d(rho eps)/d rho by differences, branch continuity,
and every transform against independent radial quadrature."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import spherical_jn, erf

from oracle.lda import pz81
from oracle.pseudo import (local_ft, local_short_ft, local_g0, projector_ft,
                           projector_real, local_real)
from workloads import SPECIES


def test_exchange_constant():
    rs = np.array([0.5, 1.0, 2.0, 4.7])
    rho = 3 / (4 * np.pi * rs ** 3)
    eps, _ = pz81(rho)
    # Hartree units: eps_x = -0.4581652932831429 / r_s; correlation at high
    # density is a small correction, so isolate exchange via rho -> large r_s?
    # Instead evaluate the exchange part directly as eps - eps_c.
    from oracle.lda import GAMMA, BETA1, BETA2, A_, B_, C_, D_
    ec = np.where(rs >= 1, GAMMA / (1 + BETA1 * np.sqrt(rs) + BETA2 * rs),
                  A_ * np.log(rs) + B_ + C_ * rs * np.log(rs) + D_ * rs)
    assert np.allclose((eps - ec) * rs, -0.4581652932831429, atol=1e-13)


@pytest.mark.parametrize("rs", [0.3, 0.8, 1.5, 3.0, 8.0])
def test_potential_is_derivative(rs):
    rho = 3 / (4 * np.pi * rs ** 3)
    h = rho * 1e-5
    e_p, _ = pz81(np.array([rho + h]))
    e_m, _ = pz81(np.array([rho - h]))
    dfd = ((rho + h) * e_p[0] - (rho - h) * e_m[0]) / (2 * h)
    _, v = pz81(np.array([rho]))
    assert abs(dfd - v[0]) < 1e-8


def test_correlation_branches_meet():
    rho1 = 3 / (4 * np.pi)
    e_hi, _ = pz81(np.array([rho1 * (1 - 1e-12)]))
    e_lo, _ = pz81(np.array([rho1 * (1 + 1e-12)]))
    # the published four-digit constants leave a 3.2e-5 Ha step at r_s = 1:
    # B + D = -0.0596 against gamma / (1 + beta1 + beta2) = -0.0596323
    assert abs(abs(e_hi[0] - e_lo[0]) - 3.2e-5) < 2e-7


def test_zero_density():
    eps, v = pz81(np.array([0.0, 1e-31]))
    assert np.all(eps == 0) and np.all(v == 0)


@pytest.mark.parametrize("name", ["Si-AH", "C-G", "Si-G"])
@pytest.mark.parametrize("G", [0.0, 0.7, 2.3, 5.1])
def test_local_transform_quadrature(name, G):
    sp = SPECIES[name]
    Z = sp["Z"]
    # short-range part v(r) + Z/r, transformed radially
    f = lambda r: local_real(sp["local"], Z, r) + Z / r
    if G == 0:
        val = 4 * np.pi * quad(lambda r: r * r * f(r), 1e-12, 30, limit=400)[0]
    else:
        val = 4 * np.pi / G * quad(lambda r: r * f(r) * np.sin(G * r), 1e-12, 30, limit=400)[0]
    assert abs(val - local_short_ft(sp["local"], Z, np.array([G]))[0]) < 1e-9
    if G > 0:
        assert abs(local_ft(sp["local"], Z, np.array([G]))[0] + 4 * np.pi * Z / G ** 2 - val) < 1e-9
    else:
        assert abs(local_g0(sp["local"], Z) - val) < 1e-9


@pytest.mark.parametrize("l,rl", [(0, 0.303), (0, 0.423), (1, 0.484)])
def test_projector_norm_and_transform(l, rl):
    norm = quad(lambda r: (projector_real(l, rl, r) * r) ** 2, 0, 20)[0]
    assert abs(norm - 1) < 1e-12
    for G in [0.0, 1.0, 3.7, 9.0]:
        val = 4 * np.pi * quad(lambda r: r * r * projector_real(l, rl, r) * spherical_jn(l, G * r),
                               0, 20, limit=400)[0]
        assert abs(val - projector_ft(l, rl, np.array([G]))[0]) < 1e-10
