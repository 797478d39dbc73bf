"""The paper's fast method for the linearized operator with a library FFT as
the transform primitive (the route of Algorithm 1).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is the CPU
throughput baseline; its agreement with the direct-sum evaluation in
``fast_direct`` (which shares only the plan tables' definitions, not this
code path) is pinned in the tests.

What is computed, per cell with Maxwellian (rho, u, theta), written from
eq. (20) (loss), eqs. (23)-(24) (gain) and the cutoff of Sec. 3.4:
    r      = h / M where M / rho >= eps, else 0
    K_j    = DFT[G phi_j]                 (G the Gaussian of eq. (24), centred at 0)
    psi_j  = iDFT[K_j DFT[r]]             (the cyclic convolution of eq. (24))
    L+     = iDFT[ sum_j Phi_j DFT[M^h psi_j] ]
    L-     = M iDFT[Omega DFT[h]] + h iDFT[Omega DFT[M]]
    L      = L+ - L-
with the readings R3 (gain constant 4 pi^2 rather than the printed 32 pi^2,
carried by Phi_j), R4 (phi_j from the Nyquist-doubled s_j) and R5 (the
product of eq. (24) is a plain cyclic convolution: unhalved DFT and inverse).
The transforms run over the signed index sets -N..N-1 of Sec. 2.3; ``fft3``
and ``ifft3`` realise them with shift bookkeeping around numpy's transforms.
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


def _gaussians(plan, rho, u, theta):
    """The three Gaussians of Sec. 3.2 on the grid: the Maxwellian M, the
    factor M^h of the gain (half the variance, centred at u) and G of
    eq. (24) (half the variance, centred at 0)."""
    v = grid.velocities(plan.n, plan.L)
    X, Y, Z = np.meshgrid(v, v, v, indexing="ij")
    du = (X - u[0]) ** 2 + (Y - u[1]) ** 2 + (Z - u[2]) ** 2
    d0 = X ** 2 + Y ** 2 + Z ** 2
    maxw = rho * (2.0 * math.pi * theta) ** -1.5 * np.exp(-du / (2.0 * theta))
    half = rho * (math.pi * theta) ** -1.5 * np.exp(-du / theta)
    gauss0 = rho * (math.pi * theta) ** -1.5 * np.exp(-d0 / theta)
    return maxw, half, gauss0


def collision_operator(plan, rho, u, theta, f, cutoff=True):
    """L[f] for one cell about the Maxwellian (rho, u, theta); f and the
    result are point values on the grid."""
    maxw, half, gauss0 = _gaussians(plan, rho, u, theta)
    # the cutoff of Sec. 3.4 decides where r is kept, relative to rho
    if cutoff and plan.eps > 0.0:
        kept = maxw / rho >= plan.eps
        r = np.zeros_like(f)
        r[kept] = f[kept] / maxw[kept]
    else:
        r = f / maxw
    # gain, eqs. (23)-(24): one convolution and one spectral weight per g-node
    r_spec = fft3(r)
    acc = np.zeros(f.shape, dtype=np.complex128)
    for weight, phi in zip(plan.Phi, plan.phi):
        kernel_spec = fft3(gauss0 * phi)
        psi = ifft3(kernel_spec * r_spec).real
        acc += weight * fft3(half * psi)
    l_plus = ifft3(acc).real
    # loss, eq. (20) at the grid points: the collision frequency nu = Omega * M
    # applied to f, and f's own convolution with Omega times M
    nu = ifft3(plan.Omega * fft3(maxw)).real
    conv_f = ifft3(plan.Omega * fft3(f)).real
    l_minus = maxw * conv_f + nu * f
    return l_plus - l_minus


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
