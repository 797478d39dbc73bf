"""Algorithm 1 of the paper, step by step, with a library FFT as the
transform primitive.  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is the CPU
throughput baseline; its agreement with the direct-sum evaluation in
``fast_direct`` (which shares only the plan tables' definitions, not this
code path) is pinned in the tests.

Algorithm 1 (Sec. 3.5) with the readings R3 (gain constant 4 pi^2 instead
of the printed 32 pi^2), R4 (phi_j from the Nyquist-doubled s_j) and R5 (the
product of line "psi <- InvFFT(u_hat r_hat)" is a plain cyclic convolution,
i.e. FFT and InvFFT without the c_k halving).  FFT/InvFFT use the paper's
index sets -N..N-1 for both l and k; ``fft3``/``ifft3`` realise that with
fftshift bookkeeping around numpy's transforms.
"""
import math

import numpy as np

from . import grid
from .fast_direct import make_plan  # plan tables: same definitions


def fft3(x):
    """sum_l x(l) exp(-i pi k.l/N) for k, l in -N..N-1 (storage k + N)."""
    return np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(x)))


def ifft3(X):
    """n^-3 sum_k X(k) exp(+i pi k.l/N)."""
    return np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(X)))


def collision_operator(plan, rho, u, theta, f, cutoff=True):
    """LinearizedCollisionOperator(rho, u, theta, f, cutoff) of Algorithm 1
    for one cell; f and the result are point values on the grid."""
    n, L = plan.n, plan.L
    v = grid.velocities(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    d2u = (VX - u[0]) ** 2 + (VY - u[1]) ** 2 + (VZ - u[2]) ** 2
    d20 = VX ** 2 + VY ** 2 + VZ ** 2
    # first loop: Maxwellians and r = f / M with the cutoff (eq. (25))
    M = rho / (2.0 * math.pi * theta) ** 1.5 * np.exp(-d2u / (2.0 * theta))
    Mg = rho / (math.pi * theta) ** 1.5 * np.exp(-d20 / theta)
    Mh = rho / (math.pi * theta) ** 1.5 * np.exp(-d2u / theta)
    if cutoff and plan.eps > 0.0:
        keep = (M / rho) >= plan.eps
        r = np.where(keep, f / np.where(keep, M, 1.0), 0.0)
    else:
        r = f / M
    # gain term
    rhat = fft3(r)
    Lhat = np.zeros((n, n, n), dtype=np.complex128)
    for j in range(plan.J):
        uj = Mg * plan.phi[j]
        uhat = fft3(uj)
        psi = ifft3(uhat * rhat).real
        psi = Mh * psi
        psihat = fft3(psi)
        Lhat += plan.Phi[j] * psihat
    Lplus = ifft3(Lhat).real
    # loss term
    fhat = fft3(f)
    Mhat = fft3(M)
    uu = ifft3(fhat * plan.Omega).real
    ww = ifft3(Mhat * plan.Omega).real
    return Lplus - uu * M - ww * f


def apply_batch(plan, h, params, cutoff=True):
    """Cells b = 0..B-1 with Maxwellians params[b] = (rho, u1, u2, u3, theta)
    (a single row is broadcast).  h: [B, n, n, n]."""
    h = np.asarray(h, dtype=np.float64)
    params = np.atleast_2d(np.asarray(params, dtype=np.float64))
    out = np.empty_like(h)
    for b in range(h.shape[0]):
        p = params[b if params.shape[0] > 1 else 0]
        out[b] = collision_operator(plan, p[0], p[1:4], p[4], h[b], cutoff)
    return out


def threads_used():
    """numpy's pocketfft runs single-threaded."""
    return 1


__all__ = ["make_plan", "collision_operator", "apply_batch", "fft3", "ifft3",
           "threads_used"]
