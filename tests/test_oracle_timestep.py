"""Pins of the oracle's RK4 for df/dt = L[f] (Sec. 4.2).

1. On a linear operator one RK4 step equals the degree-4 Taylor polynomial
   of exp(dt L) applied to f; here evaluated by repeated applications of L
   (a different evaluation order than the stages), so a wrong stage weight or
   argument fails.
2. Global error against the exact exp(t L) f of the discrete operator (its
   n^3 x n^3 matrix assembled from unit vectors at n = 8, exponentiated by
   scipy) falls by 2^4 when dt is halved: fourth order."""
import math

import numpy as np
import scipy.linalg

from oracle import alg1, fast_direct as fd, timestep
from paper_2503_09580_amd import workloads as wl


def _inputs(n, L, seed):
    rng = np.random.default_rng(seed)
    keep = np.array([a + b + c <= 2 for a, b, c in wl.MONOMIALS])
    M = wl.maxwellian(n, L, 1.0, (0, 0, 0), 1.0)
    f = M * (1.0 + wl.poly_eval(n, L, wl.poly_coeffs(rng) * keep, (0, 0, 0), 1.0))
    return f[None], np.array([[1.0, 0, 0, 0, 1.0]])


def test_one_step_is_the_taylor_polynomial():
    n, L, om, dt = 8, 4.0, 0.74, 0.1
    plan = fd.make_plan(n, L, om)
    f, p = _inputs(n, L, 1)
    step = timestep.rk4(plan, f, p, dt, 1)
    term, taylor = f.copy(), f.copy()
    for m in range(1, 5):
        term = dt / m * alg1.apply_batch(plan, term, p)
        taylor = taylor + term
    assert np.linalg.norm(step - taylor) <= 1e-13 * np.linalg.norm(taylor)


def test_fourth_order_against_matrix_exponential():
    n, L, om, T = 8, 4.0, 0.74, 0.8
    plan = fd.make_plan(n, L, om)
    p = np.array([[1.0, 0, 0, 0, 1.0]])
    N3 = n ** 3
    A = np.empty((N3, N3))
    eye = np.eye(N3).reshape(N3, n, n, n)
    for i in range(0, N3, 64):
        A[:, i:i + 64] = alg1.apply_batch(plan, eye[i:i + 64], np.repeat(p, 64, 0)).reshape(64, N3).T
    f, _ = _inputs(n, L, 2)
    exact = (scipy.linalg.expm(T * A) @ f.reshape(-1)).reshape(f.shape)
    errs = []
    for steps in (4, 8, 16):
        errs.append(np.linalg.norm(timestep.rk4(plan, f, p, T / steps, steps) - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, (errs, r1, r2)
