"""O1: the fast spectral method for the linearized operator, by direct sums.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Computes L[h] = Q(M,h) + Q(h,M) = L+[h] - L-[h] as the paper discretises it
(Sec. 3.2 and Algorithm 1), with every transform a dense per-axis DFT matrix
(``grid.dft3``) and the convolution that defines psi_j (eq. (24)) evaluated
as an explicit cyclic sum -- the "naive convolution" that Sec. 3.3 calls the
accurate one.  FP64 throughout.

Discrete definitions (n = 2N points per axis, h_v = 2L/n, k, l in -N..N-1):
  plan (Algorithm 1, precomputation; eq. (13)):
    s_j(k)     = sinc(pi g_j |k| / (2L))
    sigma_j(k) = s_j(k) * prod_d (2 if k_d = -N else 1)      [reading R4]
    phi_j      = iDFT[sigma_j]                                (real, even)
    Phi_j(k)   = 4 pi^2 W_j s_j(k)                            [reading R3]
    Omega(k)   = 16 pi^2 sum_j W_j sinc(pi g_j |k| / L)
  per Maxwellian (rho, u, theta) (Algorithm 1, first loop):
    M   = rho (2 pi theta)^(-3/2) exp(-|v-u|^2 / (2 theta))
    M^h = rho (pi theta)^(-3/2)   exp(-|v-u|^2 / theta)
    G   = rho (pi theta)^(-3/2)   exp(-|v|^2 / theta)   (centred at 0)
    chi = [M / rho >= eps]                                  (eq. (25))
  apply:
    r      = chi h / M                                       (eq. (17), (25))
    psi_j(l) = sum_d G(d) phi_j(d) r(l - d)   (cyclic; eq. (24), its
               constant (pi/N)^3 n^3 = 8 pi^3 moved into Phi_j)
    L+     = iDFT[ sum_j Phi_j DFT[M^h psi_j] ]              (eq. (23))
    L-     = M iDFT[Omega DFT[h]] + h iDFT[Omega DFT[M]]     (eq. (20) in
               collocation form, as in Algorithm 1)
    L      = L+ - L-

Why 4 pi^2: eq. (22)-(24) give psi = (pi/N)^3 * sum_k r G [sum_m s e^{..}]
= 8 pi^3 (r conv G phi_j); eq. (23) contributes (L/N)^3 / (2 pi) and the
return to point values (2L)^-3 n^3 = (N/L)^3, so the total factor on
iDFT[sum_j W_j s_j DFT[M^h (r conv G phi_j)]] is 8 pi^3 / (2 pi) = 4 pi^2.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import grid
from .quadrature import g_rule


@dataclass
class Plan:
    n: int
    L: float
    omega: float
    C: float
    R: float
    J: int
    eps: float
    rule: int
    g: np.ndarray          # [J]
    W: np.ndarray          # [J]
    s: np.ndarray          # [J, n, n, n]
    sigma: np.ndarray      # [J, n, n, n]
    phi: np.ndarray        # [J, n, n, n]  real
    Phi: np.ndarray        # [J, n, n, n]
    Omega: np.ndarray      # [n, n, n]


def default_R(L):
    """Largest kernel cutoff allowed by the de-aliasing condition
    L >= (3 + sqrt 2) R / 4 (Sec. 2.3)."""
    return 4.0 * L / (3.0 + math.sqrt(2.0))


def make_plan(n, L, omega, C=1.0 / (4.0 * math.pi), R=None, J=None, eps=1e-9, rule=0):
    """Precomputation of Algorithm 1 (tables s, sigma, phi, Phi, Omega)."""
    if n % 2:
        raise ValueError("n must be even")
    R = default_R(L) if R is None or R <= 0 else R
    J = n // 2 + 1 if J is None or J <= 0 else J
    g, W = g_rule(J, R, omega, C=C, rule=rule)
    kk = np.sqrt(grid.kabs2(n))
    s = np.stack([grid.sinc(math.pi * gj * kk / (2.0 * L)) for gj in g])
    nyq = (grid.signed_index(n) == -(n // 2)).astype(np.float64) + 1.0
    dbl = nyq[:, None, None] * nyq[None, :, None] * nyq[None, None, :]
    sigma = s * dbl[None]
    phi = np.stack([grid.idft3(sj) for sj in sigma])
    assert np.max(np.abs(phi.imag)) < 1e-12 * max(1.0, np.max(np.abs(phi.real)))
    phi = phi.real.copy()
    Phi = 4.0 * math.pi ** 2 * W[:, None, None, None] * s
    Omega = 16.0 * math.pi ** 2 * np.tensordot(
        W, np.stack([grid.sinc(math.pi * gj * kk / L) for gj in g]), axes=1)
    return Plan(n, L, omega, C, R, J, eps, rule, g, W, s, sigma, phi, Phi, Omega)


def maxwellian_fields(plan, rho, u, theta):
    """M, M^h, G and the cutoff mask chi on the grid (Algorithm 1)."""
    v = grid.velocities(plan.n, plan.L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    d2u = (VX - u[0]) ** 2 + (VY - u[1]) ** 2 + (VZ - u[2]) ** 2
    d20 = VX ** 2 + VY ** 2 + VZ ** 2
    M = rho * (2.0 * math.pi * theta) ** -1.5 * np.exp(-d2u / (2.0 * theta))
    Mh = rho * (math.pi * theta) ** -1.5 * np.exp(-d2u / theta)
    G = rho * (math.pi * theta) ** -1.5 * np.exp(-d20 / theta)
    if plan.eps > 0.0:
        chi = (M / rho) >= plan.eps
    else:
        chi = np.ones_like(M, dtype=bool)
    return M, Mh, G, chi


def cyclic_convolve_direct(r, kernels):
    """psi[c](l) = sum_{d} kernels[c](d) r(l - d) over the cyclic signed index
    set, by explicit summation.  r: [n,n,n]; kernels: [C,n,n,n] indexed by
    the signed displacement d (storage index d + N).  Returns [C,n,n,n]."""
    n = r.shape[0]
    N = n // 2
    i = np.arange(n)
    # storage index of the signed value (l - d) reduced into -N..N-1
    idx = (i[:, None] - i[None, :] + N) % n           # [i, e]
    Kmat = kernels.reshape(kernels.shape[0], -1).T    # [n^3, C]
    out = np.empty((n, n * n, kernels.shape[0]))
    ax2 = idx.reshape(n, 1, 1, n, 1)                   # (i2, ., ., e2, .)
    ax3 = idx.reshape(1, n, 1, 1, n)                   # (., i3, ., ., e3)
    for i1 in range(n):
        ax1 = idx[i1].reshape(1, 1, n, 1, 1)           # (., ., e1, ., .)
        g = r[ax1, ax2, ax3]                           # (i2, i3, e1, e2, e3)
        out[i1] = g.reshape(n * n, n ** 3) @ Kmat
    return out.reshape(n, n, n, -1).transpose(3, 0, 1, 2)


def apply(plan, h, rho=1.0, u=(0.0, 0.0, 0.0), theta=1.0, parts=False):
    """L[h] for one cell with Maxwellian (rho, u, theta), FP64, direct sums."""
    h = np.asarray(h, dtype=np.float64)
    M, Mh, G, chi = maxwellian_fields(plan, rho, u, theta)
    r = np.zeros_like(h)
    r[chi] = h[chi] / M[chi]
    # gain term: psi_j by naive convolution, then eq. (23)
    K = G[None] * plan.phi                             # G(d) phi_j(d)
    psi = cyclic_convolve_direct(r, K)
    Lhat = np.zeros((plan.n,) * 3, dtype=np.complex128)
    for j in range(plan.J):
        Lhat += plan.Phi[j] * grid.dft3(Mh * psi[j])
    Lp = grid.idft3(Lhat).real
    # loss term, eq. (20) in collocation form
    U = grid.idft3(plan.Omega * grid.dft3(h)).real
    nu = grid.idft3(plan.Omega * grid.dft3(M)).real
    Lm = M * U + nu * h
    if parts:
        return Lp - Lm, Lp, Lm
    return Lp - Lm
