"""Time stepping of the spatially homogeneous linearized equation
df/dt = L[f] (Sec. 4.2) with the classical fourth-order Runge-Kutta scheme
and a fixed step, as the paper integrates it.  FP64, one cell at a time,
the operator by Algorithm 1 (``alg1``).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from . import alg1


def _L(plan, f, params, cutoff=True):
    return alg1.apply_batch(plan, f, params, cutoff)


def rk4(plan, f, params, dt, steps, cutoff=True):
    """f: [batch, n, n, n]; params: [batch or 1, 5].  Returns f after
    `steps` steps: k1 = L f, k2 = L(f + dt/2 k1), k3 = L(f + dt/2 k2),
    k4 = L(f + dt k3), f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    f = np.array(f, dtype=np.float64, copy=True)
    for _ in range(steps):
        k1 = _L(plan, f, params, cutoff)
        k2 = _L(plan, f + 0.5 * dt * k1, params, cutoff)
        k3 = _L(plan, f + 0.5 * dt * k2, params, cutoff)
        k4 = _L(plan, f + dt * k3, params, cutoff)
        f = f + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return f
