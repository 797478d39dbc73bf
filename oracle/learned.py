"""Learned correction for the inner solves of the steady problem: the fixed
(non-learned) maps around the network, and the network itself with its
training step, in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Newton correction g of eq. (modified_Newton) is split as
g = z + (macroscopic rest) with z one transport sweep of the residual.  The
rest is modelled per cell by five Hermite coefficients predicted from
per-cell features of z (a small network; trained on (residual, Newton
correction) pairs of converged solves).

Per cell c with local Maxwellian parameters (rho, u, theta):
    psi_0 = 1, psi_d = (v_d - u_d)/sqrt(theta) (d = 1..3),
    psi_4 = (|v - u|^2/theta - 3)/sqrt(6)
(orthonormal under M/rho), and the moments of a field z
    m_a(c) = h_v^3 sum_v z_c(v) psi_a(v) / rho_c.
Features (26 per cell): with s = sqrt(mean_{c,a} m_a(c)^2) (s = 1 if zero),
ms = m / s and x_c = (c + 1/2)/nx,
    ms (5) | left (5): (sum_{c'<=c} ms - ms/2)/nx | right (5): (sum_{c'>=c} ms - ms/2)/nx
    | lx (5): sum_{c'<=c} ms x_c' / nx | rx (5): sum_{c'>=c} ms x_c' / nx | x_c.
Training target: m(g - z)/s.  The correction for predicted y:
    Delta_c(v) = sum_a s y_a(c) M_c(v) psi_a(v),
    M_c = rho (2 pi theta)^(-3/2) exp(-|v - u|^2/(2 theta)).

Network: Y = tanh(X W1 + b1) W2 + b2 (W1: 26 x 128, W2: 128 x 5); loss
mean((Y - T)^2) over all entries; Adam (Kingma & Ba, 2015) with bias
correction.
"""
import math

import numpy as np

from . import grid

N_IN, N_HID, N_OUT = 26, 128, 5


def _basis(n, L, params_c):
    v = grid.velocities(n, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    rho, u, th = params_c[0], params_c[1:4], params_c[4]
    w = [(V[d] - u[d]) / math.sqrt(th) for d in range(3)]
    q = (sum(x * x for x in w) - 3.0) / math.sqrt(6.0)
    d2 = sum((V[d] - u[d]) ** 2 for d in range(3))
    M = rho * (2 * math.pi * th) ** -1.5 * np.exp(-d2 / (2 * th))
    return M, [np.ones_like(M), *w, q]


def moments(z, params, n, L):
    """m[c][a] = h^3 sum z_c psi_a / rho_c."""
    h3 = (2.0 * L / n) ** 3
    out = np.empty((z.shape[0], 5))
    for c in range(z.shape[0]):
        _, psi = _basis(n, L, params[c])
        out[c] = [h3 * np.sum(z[c] * psi[a]) / params[c, 0] for a in range(5)]
    return out


def features(m):
    """(X [nx][26], s) from the moments m [nx][5]."""
    nx = m.shape[0]
    s = math.sqrt(np.mean(m * m))
    if s == 0.0:
        s = 1.0
    ms = m / s
    x = (np.arange(nx) + 0.5) / nx
    X = np.empty((nx, N_IN))
    for c in range(nx):
        X[c, 0:5] = ms[c]
        X[c, 5:10] = (ms[:c + 1].sum(0) - ms[c] / 2) / nx
        X[c, 10:15] = (ms[c:].sum(0) - ms[c] / 2) / nx
        X[c, 15:20] = (ms[:c + 1] * x[:c + 1, None]).sum(0) / nx
        X[c, 20:25] = (ms[c:] * x[c:, None]).sum(0) / nx
        X[c, 25] = x[c]
    return X, s


def correction(Y, s, params, n, L):
    """Delta[c] = sum_a s Y[c][a] M_c psi_a."""
    out = np.empty((Y.shape[0], n, n, n))
    for c in range(Y.shape[0]):
        M, psi = _basis(n, L, params[c])
        out[c] = M * sum(s * Y[c, a] * psi[a] for a in range(5))
    return out


# ---- network ------------------------------------------------------------------

def forward(w, X):
    """w = (W1, b1, W2, b2).  Returns (Y, H)."""
    W1, b1, W2, b2 = w
    H = np.tanh(X @ W1 + b1)
    return H @ W2 + b2, H


def loss_grad(w, X, T):
    """(loss, (dW1, db1, dW2, db2)) of loss = mean((Y - T)^2)."""
    W1, b1, W2, b2 = w
    Y, H = forward(w, X)
    E = Y - T
    loss = np.mean(E * E)
    dY = 2.0 * E / E.size
    dW2 = H.T @ dY
    db2 = dY.sum(0)
    dH = (dY @ W2.T) * (1.0 - H * H)
    dW1 = X.T @ dH
    db1 = dH.sum(0)
    return loss, (dW1, db1, dW2, db2)


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (in place on lists w, m, v)."""
    for i in range(len(w)):
        m[i] = b1 * m[i] + (1 - b1) * g[i]
        v[i] = b2 * v[i] + (1 - b2) * g[i] * g[i]
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        w[i] = w[i] - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v


def pack(w):
    return np.concatenate([a.reshape(-1) for a in w])


def unpack(flat):
    sizes = [(N_IN, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,)]
    out, o = [], 0
    for sh in sizes:
        k = int(np.prod(sh))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(sh))
        o += k
    return out


N_WEIGHTS = N_IN * N_HID + N_HID + N_HID * N_OUT + N_OUT
