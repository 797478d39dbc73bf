"""Quadrature rules used by the oracle (test infrastructure only).

* ``gauss_jacobi``        Gauss-Jacobi rule by the Golub-Welsch eigenvalue
                          method (numpy symmetric eigensolver).
* ``gauss_jacobi_radau``  Radau variant with the node fixed at x = -1.
* ``g_rule``              The rule in the relative speed g on [0, R] that
                          discretises  int_0^R g^2 B(g) chi(g) dg  (Sec. 2.3,
                          eq. (13); Sec. 4.1 asks for a Jacobi-Gauss-Radau
                          rule exact to polynomial degree 2N).
* ``hemisphere_product_rule``  A product rule on the unit hemisphere in the
                          normalisation of eq. (13): int_{S^2_+} f dsigma
                          ~= 2 pi sum_m w_m f(sigma_m), sum_m w_m = 1.
"""
import math

import numpy as np


def jacobi_recurrence(n, a, b):
    """Monic three-term recurrence coefficients of the Jacobi polynomials
    for the weight (1-x)^a (1+x)^b on [-1, 1]:
        p_{k+1} = (x - alpha_k) p_k - beta_k p_{k-1}.
    Returns (alpha[0:n], beta[0:n]) with beta[0] = mu_0 = int w dx."""
    alpha = np.zeros(n)
    beta = np.zeros(n)
    for k in range(n):
        s = 2 * k + a + b
        if k == 0 and abs(a + b) < 1e-300:
            alpha[k] = (b - a) / (a + b + 2)
        else:
            alpha[k] = (b * b - a * a) / (s * (s + 2))
        if k == 0:
            beta[k] = 2.0 ** (a + b + 1) * math.gamma(a + 1) * math.gamma(b + 1) / math.gamma(a + b + 2)
        else:
            beta[k] = 4.0 * k * (k + a) * (k + b) * (k + a + b) / (s * s * (s + 1) * (s - 1))
    return alpha, beta


def gauss_jacobi(n, a, b):
    """n-point Gauss-Jacobi nodes/weights (Golub-Welsch)."""
    alpha, beta = jacobi_recurrence(n, a, b)
    T = np.diag(alpha) + np.diag(np.sqrt(beta[1:]), 1) + np.diag(np.sqrt(beta[1:]), -1)
    x, V = np.linalg.eigh(T)
    w = beta[0] * V[0, :] ** 2
    return x, w


def gauss_jacobi_radau(n, b):
    """n-point Gauss-Radau rule for the weight (1+x)^b on [-1, 1] with the
    node x = -1 fixed.  Exact for polynomials of degree <= 2n - 2.

    Writing p(x) = p(-1) + (1+x) q(x), the (n-1)-point Gauss-Jacobi rule for
    the weight (1+x)^(b+1) integrates (1+x)^b (1+x) q exactly; the fixed
    node then carries the remaining mass."""
    mu0 = 2.0 ** (b + 1) / (b + 1)
    if n == 1:
        return np.array([-1.0]), np.array([mu0])
    xi, wi = gauss_jacobi(n - 1, 0.0, b + 1.0)
    lam = wi / (1.0 + xi)
    x = np.concatenate(([-1.0], xi))
    w = np.concatenate(([mu0 - lam.sum()], lam))
    return x, w


def g_rule(J, R, omega, C=1.0 / (4.0 * math.pi), rule=0):
    """Nodes g_j and combined weights W_j = w_j^g B(g_j) such that
        sum_j W_j chi(g_j) ~= int_0^R g^2 B(g) chi(g) dg,   B(g) = C g^(2(1-omega)).

    rule 0 (default): Radau weight (1+x)^beta with beta = 4 - 2 omega
        absorbs g^2 B(g), so W_j = C (R/2)^(beta+1) lambda_j.
    rule 1: Radau weight (1+x)^2 (the g^2 of eq. (13)) and B(g_j)
        multiplied in afterwards.
    The fixed node is g = 0 in both cases."""
    if rule == 0:
        beta = 4.0 - 2.0 * omega
        x, lam = gauss_jacobi_radau(J, beta)
        g = 0.5 * R * (1.0 + x)
        W = C * (0.5 * R) ** (beta + 1.0) * lam
    elif rule == 1:
        x, lam = gauss_jacobi_radau(J, 2.0)
        g = 0.5 * R * (1.0 + x)
        wg = (0.5 * R) ** 3 * lam
        W = wg * C * np.power(g, 2.0 * (1.0 - omega))
    else:
        raise ValueError("rule must be 0 or 1")
    return g, W


def hemisphere_product_rule(n_polar=8, n_azimuth=16):
    """Product rule on S^2_+ (sigma_3 >= 0 half) in the normalisation of
    eq. (13): nodes are the positive Gauss-Legendre nodes mu_i of the
    n_polar-point rule on [-1, 1] (polar cosines) times n_azimuth equispaced
    azimuths; weights w_i^GL / n_azimuth, summing to 1.  The default gives
    4 x 16 = 64 points.  Returns (sigma[M, 3], w[M])."""
    mu, wmu = np.polynomial.legendre.leggauss(n_polar)
    keep = mu > 0
    mu, wmu = mu[keep], wmu[keep]
    phi = 2.0 * math.pi * np.arange(n_azimuth) / n_azimuth
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    W = np.repeat(wmu[:, None], n_azimuth, axis=1) / n_azimuth
    st = np.sqrt(1.0 - MU ** 2)
    sigma = np.stack([st * np.cos(PHI), st * np.sin(PHI), MU], axis=-1).reshape(-1, 3)
    return sigma, W.reshape(-1)
