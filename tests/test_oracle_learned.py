"""Pins of the oracle's learned-correction pieces (network, training step,
features, Hermite moments and correction).

1. Backward pass against central finite differences of the loss.
2. Forward pass of a network with one live path against its closed form.
3. The first Adam step moves every weight by lr * sign(gradient) (bias
   correction makes m/sqrt(v) = g/|g| at t = 1; Kingma & Ba, 2015).
4. Features of a constant moment field against their closed forms
   (x_c ms, (1 - x_c) ms, (c+1)^2/(2 nx^2) ms, ...).
5. Hermite moments invert the correction: psi_a are orthonormal under M/rho,
   so moments(correction(y)) = s y up to the quadrature error of a resolved
   Maxwellian."""
import math

import numpy as np

from oracle import learned as lr_


def _weights(seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(0, 0.3, (lr_.N_IN, lr_.N_HID)), rng.normal(0, 0.1, lr_.N_HID),
            rng.normal(0, 0.3, (lr_.N_HID, lr_.N_OUT)), rng.normal(0, 0.1, lr_.N_OUT)]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = _weights(2)
    X = rng.normal(size=(7, lr_.N_IN))
    T = rng.normal(size=(7, lr_.N_OUT))
    _, g = lr_.loss_grad(w, X, T)
    for k, idx in [(0, (3, 17)), (1, (40,)), (2, (100, 4)), (3, (2,)), (0, (25, 127))]:
        h = 1e-6
        wp = [a.copy() for a in w]
        wm = [a.copy() for a in w]
        wp[k][idx] += h
        wm[k][idx] -= h
        fd = (lr_.loss_grad(wp, X, T)[0] - lr_.loss_grad(wm, X, T)[0]) / (2 * h)
        assert abs(fd - g[k][idx]) <= 1e-7 * max(abs(fd), 1e-3), (k, idx, fd, g[k][idx])


def test_forward_single_path_closed_form():
    W1 = np.zeros((lr_.N_IN, lr_.N_HID))
    W1[4, 9] = 0.7
    b1 = np.zeros(lr_.N_HID)
    b1[9] = -0.2
    W2 = np.zeros((lr_.N_HID, lr_.N_OUT))
    W2[9, 3] = 1.5
    b2 = np.array([0.1, 0.0, 0.0, -0.4, 0.0])
    X = np.zeros((2, lr_.N_IN))
    X[:, 4] = [0.5, -1.0]
    Y, _ = lr_.forward([W1, b1, W2, b2], X)
    for i, x in enumerate([0.5, -1.0]):
        want = b2.copy()
        want[3] += 1.5 * math.tanh(0.7 * x - 0.2)
        assert np.allclose(Y[i], want, rtol=0, atol=1e-15)


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.default_rng(3)
    w = _weights(4)
    X = rng.normal(size=(5, lr_.N_IN))
    T = rng.normal(size=(5, lr_.N_OUT))
    _, g = lr_.loss_grad(w, X, T)
    m = [np.zeros_like(a) for a in w]
    v = [np.zeros_like(a) for a in w]
    w0 = [a.copy() for a in w]
    lr = 1e-3
    lr_.adam_step(w, list(g), m, v, 1, lr)
    for a0, a1, ga in zip(w0, w, g):
        big = np.abs(ga) > 1e-4
        step = (a1 - a0)[big]
        assert np.allclose(step, -lr * np.sign(ga[big]), rtol=1e-3, atol=0)


def test_features_of_a_constant_field():
    nx = 6
    m = np.tile(np.array([1.0, -2.0, 0.5, 0.0, 3.0]), (nx, 1))
    X, s = lr_.features(m)
    assert abs(s - math.sqrt(np.mean(m * m))) < 1e-15
    ms = m[0] / s
    for c in range(nx):
        x = (c + 0.5) / nx
        assert np.allclose(X[c, 0:5], ms, atol=1e-15)
        assert np.allclose(X[c, 5:10], x * ms, atol=1e-15)
        assert np.allclose(X[c, 10:15], (1 - x) * ms, atol=1e-15)
        assert np.allclose(X[c, 15:20], (c + 1) ** 2 / (2 * nx * nx) * ms, atol=1e-15)
        assert np.allclose(X[c, 20:25], (nx * nx - c * c) / (2 * nx * nx) * ms, atol=1e-15)
        assert X[c, 25] == x
    X0, s0 = lr_.features(np.zeros((3, 5)))
    assert s0 == 1.0 and np.all(X0[:, :25] == 0)


def test_moments_invert_the_correction():
    n, L = 32, 8.0
    params = np.array([[1.1, 0.1, -0.05, 0.02, 1.2], [0.8, 0.0, 0.1, 0.0, 0.9]])
    Y = np.array([[0.3, -0.2, 0.1, 0.05, 0.4], [-0.1, 0.2, 0.0, 0.3, -0.25]])
    s = 0.7
    d = lr_.correction(Y, s, params, n, L)
    m = lr_.moments(d, params, n, L)
    # the box edge truncates the theta = 1.2 tail of |v - u|^4 M at about 1e-10
    assert np.max(np.abs(m - s * Y)) < 1e-9


def test_adam_bias_correction_beyond_the_first_step():
    """Pins Adam's bias correction at t > 1 against two closed forms
    (Kingma & Ba, 2015, Algorithm 1):
    - a constant gradient g for t = 1..5 gives m_t = (1 - b1^t) g and
      v_t = (1 - b2^t) g^2, so the corrected ratio is g/|g| at every step
      and each step moves the weight by lr * sign(g);
    - g at t = 1 and -g at t = 2 gives m_2 = -(1 - b1)^2 g and
      v_2 = (1 - b2^2) g^2; corrected, m_2/(1 - b1^2) = -(1 - b1)/(1 + b1) g
      and v_2/(1 - b2^2) = g^2, so the second step is
      +lr (1 - b1)/(1 + b1) sign(g).
    A bias correction with the wrong power of b1 or b2 fails both."""
    lr, b1 = 1e-2, 0.9
    g = np.array([0.3, -2.0, 5e-3, -1e-2, 7.0])
    w = [np.zeros(5)]
    m, v = [np.zeros(5)], [np.zeros(5)]
    for t in range(1, 6):
        before = w[0].copy()
        lr_.adam_step(w, [g], m, v, t, lr)
        assert np.allclose(w[0] - before, -lr * np.sign(g), rtol=1e-5, atol=0), t
    w = [np.zeros(5)]
    m, v = [np.zeros(5)], [np.zeros(5)]
    lr_.adam_step(w, [g], m, v, 1, lr)
    first = w[0].copy()
    lr_.adam_step(w, [-g], m, v, 2, lr)
    want = lr * (1 - b1) / (1 + b1) * np.sign(g)
    assert np.allclose(w[0] - first, want, rtol=1e-5, atol=0)
