"""Pins for the oracle's quadrature rules against closed forms and library
routines (no GPU)."""
import math

import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import quadrature as q
from oracle import grid


@pytest.mark.parametrize("n,a,b", [(4, 0.0, 3.0), (8, 0.0, 3.52), (16, 0.0, 4.0), (5, 1.5, 0.5)])
def test_gauss_jacobi_matches_scipy(n, a, b):
    x, w = q.gauss_jacobi(n, a, b)
    xr, wr = roots_jacobi(n, a, b)
    np.testing.assert_allclose(np.sort(x), np.sort(xr), rtol=0, atol=1e-13)
    np.testing.assert_allclose(w[np.argsort(x)], wr[np.argsort(xr)], rtol=1e-12)


@pytest.mark.parametrize("J", [2, 3, 5, 9, 17, 33])
@pytest.mark.parametrize("omega", [0.5, 0.74, 1.0])
def test_g_rule_monomial_exactness(J, omega):
    # sum_j W_j g_j^p = C int_0^R g^(4-2 omega) g^p dg = C R^(p+5-2w)/(p+5-2w)
    # for p = 0 .. 2J-2 (Radau exactness, Sec. 4.1 asks for degree 2N = n).
    R, C = 7.2492, 1.0 / (4.0 * math.pi)
    g, W = q.g_rule(J, R, omega, C=C)
    assert g[0] == 0.0
    assert np.all(W > 0)
    assert np.all(np.diff(g) > 0) and g[-1] < R
    for p in range(2 * J - 1):
        e = p + 5.0 - 2.0 * omega
        exact = C * R ** e / e
        got = np.sum(W * g ** p)
        assert abs(got - exact) <= 1e-12 * exact, (p, got, exact)
    if J <= 5:   # one degree higher is not exact (visible at small J)
        p = 2 * J - 1
        e = p + 5.0 - 2.0 * omega
        assert abs(np.sum(W * g ** p) - C * R ** e / e) > 1e-7 * C * R ** e / e


@pytest.mark.parametrize("J", [9, 17, 33])
@pytest.mark.parametrize("omega", [0.5, 0.74])
def test_g_rule_chebyshev_exactness(J, omega):
    # Monomials are dominated by g ~ R at high degree; Chebyshev polynomials
    # in x = 2g/R - 1 test every degree up to 2J-2 evenly.  Exact integrals
    # by adaptive quadrature (library routine).
    from scipy.integrate import quad
    R, C = 9.0612, 1.0 / (4.0 * math.pi)
    beta = 4.0 - 2.0 * omega
    g, W = q.g_rule(J, R, omega, C=C)
    x = 2.0 * g / R - 1.0
    for p in range(0, 2 * J - 1, 3):
        f = lambda t: (1.0 + t) ** beta * math.cos(p * math.acos(max(-1.0, min(1.0, t))))
        exact = C * (R / 2.0) ** (beta + 1) * quad(f, -1.0, 1.0, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
        got = np.sum(W * np.cos(p * np.arccos(np.clip(x, -1, 1))))
        scale = C * (R / 2.0) ** (beta + 1) * 2.0 ** (beta + 1) / (beta + 1)
        assert abs(got - exact) <= 1e-12 * scale, (p, got, exact)


def test_g_rule_alternative_weight():
    # rule 1: Radau for the plain g^2 weight, B(g_j) multiplied in; for
    # Maxwell molecules (B constant) it is exact to degree 2J-2 as well.
    R, C, J = 6.0, 1.0 / (4.0 * math.pi), 9
    g, W = q.g_rule(J, R, 1.0, C=C, rule=1)
    for p in range(2 * J - 1):
        assert abs(np.sum(W * g ** p) - C * R ** (p + 3) / (p + 3)) <= 1e-12 * C * R ** (p + 3)


def test_hemisphere_rule_moments():
    sig, w = q.hemisphere_product_rule()
    assert sig.shape == (64, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.linalg.norm(sig, axis=1), 1.0, atol=1e-15)
    assert np.all(sig[:, 2] > 0)
    # (1/2pi) int_{S^2_+} mu^(2p) dsigma = 1/(2p+1), exact while 2p <= 15
    for p in range(8):
        assert abs(np.sum(w * sig[:, 2] ** (2 * p)) - 1.0 / (2 * p + 1)) < 1e-14
    # azimuthal harmonics vanish below the azimuth count
    phi = np.arctan2(sig[:, 1], sig[:, 0])
    for k in range(1, 16):
        assert abs(np.sum(w * np.cos(k * phi))) < 1e-14


def test_sphere_sinc_estimate_converges():
    # eq. (16): (1/2pi) int_{S^2_+} cos(a sigma.e) dsigma = sinc(a) for unit e
    e = np.array([0.3, -0.5, 0.81])
    e /= np.linalg.norm(e)
    errs = []
    for npol, naz in [(4, 8), (8, 16), (16, 32), (24, 48)]:
        sig, w = q.hemisphere_product_rule(npol, naz)
        a = 6.0
        est = np.sum(w * np.cos(a * sig @ e))
        errs.append(abs(est - grid.sinc(a)))
    assert errs[-1] < 1e-12
    assert errs[0] > errs[1] > errs[2]
