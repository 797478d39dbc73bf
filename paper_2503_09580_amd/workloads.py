"""Seeded synthetic inputs for the linearized collision operator.

This module only builds input distributions and per-cell Maxwellian
parameters; it contains none of the operator's arithmetic.  It is the one
module shared by the GPU tests/benchmark and the CPU oracle tests.  NumPy
only, FP64.

Grid: n points per axis, v_i = -L + i (2L/n), i = 0..n-1, row-major
[x][y][z] with z fastest.  Parameters per cell: (rho, u1, u2, u3, theta).

The paper measures on closed-form distributions only (Sec. 4: f^(1), f^(2));
the configurations below are synthetic stand-ins of the same kind:
  C1  n=16, L=8,  omega=0.5,  1 cell, M=(1,0,1), h = M p(v)
  C2  n=32, L=8,  omega=0.74, 64 cells, M=(1,0,1), h = f_b - M with f_b a
      drifting anisotropic (bi-)Maxwellian; also Burnett functions (omega=1)
  C3  n=32, L=8,  omega=0.74, 4096 cells along a 1-D grid with sinusoidal
      rho, u, theta (amplitude 0.2), h_i = M_i p_i((v-u_i)/sqrt(theta_i))
  C4  n=32, L=8,  omega=0.74, the steady 1-D slab x in [-0.5, 0.5] on 256
      cells, wall temperatures 1 and 1.5, Kn = 0.1, total mass 1 (Sec. 5.3.2,
      the heat-transfer case); states from the solver, test states from
      slab_state
  C5  n=64, L=10, omega=0.74, 512 cells, rho=1, u=0, theta log-uniform in
      [0.5, 2], h_i = M_i p_i(v/sqrt(theta_i))
p is a polynomial of total degree <= 4 (35 monomials) with coefficients
drawn N(0, 0.1^2).
"""
import math

import numpy as np

CONFIGS = {
    "C1": dict(n=16, L=8.0, omega=0.5, batch=1, seed=101),
    "C2": dict(n=32, L=8.0, omega=0.74, batch=64, seed=202),
    "C3": dict(n=32, L=8.0, omega=0.74, batch=4096, seed=303),
    "C5": dict(n=64, L=10.0, omega=0.74, batch=512, seed=505),
    "C4": dict(n=32, L=8.0, omega=0.74, nx=256, kn=0.1, theta_l=1.0, theta_r=1.5, mass=1.0),
}

MONOMIALS = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]


def axis(n, L):
    return -L + np.arange(n) * (2.0 * L / n)


def maxwellian(n, L, rho, u, theta):
    """rho (2 pi theta)^-3/2 exp(-|v-u|^2/(2 theta)) on the grid (input
    construction only)."""
    v = axis(n, L)
    ex = np.exp(-(v - u[0]) ** 2 / (2.0 * theta))
    ey = np.exp(-(v - u[1]) ** 2 / (2.0 * theta))
    ez = np.exp(-(v - u[2]) ** 2 / (2.0 * theta))
    return rho * (2.0 * math.pi * theta) ** -1.5 * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]


def poly_eval(n, L, coeffs, shift=(0.0, 0.0, 0.0), scale=1.0):
    """sum_abc c_abc w1^a w2^b w3^c with w = (v - shift) / scale."""
    v = axis(n, L)
    w = [(v - shift[d]) / scale for d in range(3)]
    pw = [np.stack([wd ** e for e in range(5)]) for wd in w]
    out = np.zeros((n, n, n))
    for c, (a, b, e) in zip(coeffs, MONOMIALS):
        out += c * pw[0][a][:, None, None] * pw[1][b][None, :, None] * pw[2][e][None, None, :]
    return out


def poly_coeffs(rng, std=0.1):
    return rng.normal(0.0, std, size=len(MONOMIALS))


def bimaxwellian(n, L, tau, u):
    """Unit-density anisotropic Maxwellian with T_par = tau T_perp along e1,
    trace temperature 1, drift u."""
    tperp = 3.0 / (2.0 + tau)
    tpar = tau * tperp
    v = axis(n, L)
    ex = np.exp(-(v - u[0]) ** 2 / (2.0 * tpar))
    ey = np.exp(-(v - u[1]) ** 2 / (2.0 * tperp))
    ez = np.exp(-(v - u[2]) ** 2 / (2.0 * tperp))
    pre = (2.0 * math.pi) ** -1.5 / math.sqrt(tpar * tperp * tperp)
    return pre * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]


def _ball(rng, radius):
    while True:
        u = rng.uniform(-radius, radius, size=3)
        if u @ u <= radius * radius:
            return u


def c1(seed=101):
    cfg = CONFIGS["C1"]
    n, L = cfg["n"], cfg["L"]
    rng = np.random.default_rng(seed)
    M = maxwellian(n, L, 1.0, (0, 0, 0), 1.0)
    h = M * poly_eval(n, L, poly_coeffs(rng))
    params = np.array([[1.0, 0.0, 0.0, 0.0, 1.0]])
    return h[None], params


def c2(batch=64, seed=202, n=32, L=8.0):
    rng = np.random.default_rng(seed)
    M = maxwellian(n, L, 1.0, (0, 0, 0), 1.0)
    h = np.empty((batch, n, n, n))
    for b in range(batch):
        tau = rng.uniform(0.8, 1.25)
        u = _ball(rng, 0.3)
        h[b] = bimaxwellian(n, L, tau, u) - M
    params = np.array([[1.0, 0.0, 0.0, 0.0, 1.0]])
    return h, params


def c3_params(batch=4096, seed=303):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=5)        # rho, u1, u2, u3, theta
    x = (np.arange(batch) + 0.5) / batch
    p = np.empty((batch, 5))
    p[:, 0] = 1.0 + 0.2 * np.sin(2 * math.pi * x + ph[0])
    for d in range(3):
        p[:, 1 + d] = 0.2 * np.sin(2 * math.pi * x + ph[1 + d])
    p[:, 4] = 1.0 + 0.2 * np.sin(2 * math.pi * x + ph[4])
    return p, rng


def c3(batch=4096, seed=303, n=32, L=8.0, cells=None):
    """Returns (h[len(cells)], params[len(cells)]); `cells` selects a subset
    of the full batch (default: all) without changing any cell's data."""
    p, rng = c3_params(batch, seed)
    coeffs = np.stack([poly_coeffs(rng) for _ in range(batch)])
    cells = np.arange(batch) if cells is None else np.asarray(cells, dtype=np.int64)
    h = np.empty((len(cells), n, n, n))
    for i, c in enumerate(cells):
        rho, u, th = p[c, 0], p[c, 1:4], p[c, 4]
        h[i] = maxwellian(n, L, rho, u, th) * poly_eval(n, L, coeffs[c], u, math.sqrt(th))
    return h, p[cells].copy()


def c5(batch=512, seed=505, n=64, L=10.0, cells=None):
    rng = np.random.default_rng(seed)
    th = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=batch))
    coeffs = np.stack([poly_coeffs(rng) for _ in range(batch)])
    p = np.zeros((batch, 5))
    p[:, 0] = 1.0
    p[:, 4] = th
    cells = np.arange(batch) if cells is None else np.asarray(cells, dtype=np.int64)
    h = np.empty((len(cells), n, n, n))
    for i, c in enumerate(cells):
        h[i] = maxwellian(n, L, 1.0, (0, 0, 0), th[c]) * poly_eval(n, L, coeffs[c], (0, 0, 0), math.sqrt(th[c]))
    return h, p[cells].copy()


def invariant_inputs(n, L, rho=1.0, u=(0.0, 0.0, 0.0), theta=1.0):
    """[5, n, n, n]: M, v1 M, v2 M, v3 M, |v|^2 M."""
    v = axis(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    M = maxwellian(n, L, rho, u, theta)
    return np.stack([M, VX * M, VY * M, VZ * M, (VX ** 2 + VY ** 2 + VZ ** 2) * M])


BURNETT_NL = [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0), (0, 3), (1, 2), (0, 4)]


def burnett(n, L, nn, l):
    """h_nl = M(v) L_n^(l+1/2)(|v|^2/2) |v|^l P_l(v3/|v|) for the unit
    Maxwellian (the m = 0 Burnett functions)."""
    from scipy.special import eval_genlaguerre, eval_legendre
    v = axis(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    r2 = VX ** 2 + VY ** 2 + VZ ** 2
    r = np.sqrt(r2)
    c = np.where(r > 0, VZ / np.where(r > 0, r, 1.0), 0.0)
    rad = eval_genlaguerre(nn, l + 0.5, r2 / 2.0) * r ** l
    ang = eval_legendre(l, c) if l > 0 else np.ones_like(c)
    return maxwellian(n, L, 1.0, (0, 0, 0), 1.0) * rad * ang


def paper_f1(n, L, unit_mass=False):
    """Initial/test distribution f^(1) of Sec. 4 (Cases of Sec. 4.1-4.2):
    four shifted Gaussians, u = sqrt 2, theta = 1/3.  With the printed
    prefactor 1/(4 pi^(3/2)) its mass is (2/3)^(3/2); unit_mass=True uses
    (3/(2 pi))^(3/2)/4 instead, the mass-1 form that relaxes to the standard
    Maxwellian (as the time-stepping experiments of Sec. 4.2 need)."""
    v = axis(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    u, th = math.sqrt(2.0), 1.0 / 3.0

    def e(a, b):
        return np.exp(-((VX + a) ** 2 + (VY + b) ** 2 + VZ ** 2) / (2 * th))

    pref = (3.0 / (2.0 * math.pi)) ** 1.5 / 4.0 if unit_mass else 1.0 / (4 * math.pi ** 1.5)
    return (e(u, 0) + e(-u, 0) + e(0, u) + e(0, -u)) * pref


def paper_f2(n, L):
    """The discontinuous distribution f^(2) of Sec. 4: a narrow Gaussian
    (variance 1/sqrt 2 per axis) for v1 > 0 and a wide one (variance sqrt 2)
    at a quarter of the prefactor for v1 < 0, prefactor
    2^(1/4) (2 - sqrt 2) / pi^(3/2); mass 1, velocity 0, temperature 1.  On
    the grid plane v1 = 0 it takes the mean of the two one-sided values."""
    v = axis(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    r2 = VX ** 2 + VY ** 2 + VZ ** 2
    a = 2.0 ** 0.25 * (2.0 - math.sqrt(2.0)) / math.pi ** 1.5
    pos = a * np.exp(-r2 / math.sqrt(2.0))
    neg = 0.25 * a * np.exp(-r2 / (2.0 * math.sqrt(2.0)))
    return np.where(VX > 0, pos, np.where(VX < 0, neg, 0.5 * (pos + neg)))


def slab_state(n, L, nx, theta_l=1.0, theta_r=1.5, seed=404, amp=0.05):
    """Seeded non-equilibrium states of the 1-D slab on nx cells: per cell a
    Maxwellian whose temperature runs linearly from theta_l to theta_r, with
    density and drift perturbed by amp-sized seeded values, times
    (1 + p((v-u)/sqrt(theta))) with a small seeded polynomial p; and a
    seeded perturbation g of the same shape (M_c times a polynomial).
    Returns (f, g), each [nx][n][n][n]."""
    rng = np.random.default_rng(seed)
    f = np.empty((nx, n, n, n))
    g = np.empty((nx, n, n, n))
    for c in range(nx):
        x = (c + 0.5) / nx
        th = theta_l + (theta_r - theta_l) * x
        rho = 1.0 + amp * rng.uniform(-1.0, 1.0)
        u = amp * rng.uniform(-1.0, 1.0, size=3)
        M = maxwellian(n, L, rho, u, th)
        f[c] = M * (1.0 + poly_eval(n, L, poly_coeffs(rng, std=0.2 * amp), u, math.sqrt(th)))
        g[c] = M * poly_eval(n, L, poly_coeffs(rng), u, math.sqrt(th))
    return f, g
