"""O2: the spectral method for the binary collision operator (Sec. 2.3,
eq. (14)) with an explicit hemisphere quadrature, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a bilinear pair (F, G) with coefficients
    F^_k = h_v^3 sum_l F(l) exp(-i pi k.l / N)   (no c_k halving; reading R6)
the discrete operator of eq. (14) is
    Q^_k = (2 pi^2 / L^3) [ sum_j sum_m W_j w_m s_j(k) I_{j,k,m}
                            - sum_l F^_{k-l} G^_l Omega'_l ]
    I_{j,k,m} = sum_l F^_{k-l} G^_l cos(pi g_j sigma_m.((k-l) - l) / (2L))
    Omega'_l  = sum_j W_j sinc(pi g_j |l| / L)
where k-l is reduced cyclically into -N..N-1 before it enters the cosine
(the cos*cos + sin*sin bracket of eq. (14) written as one cosine), and point
values are Q(v_l) = (2L)^-3 sum_k Q^_k exp(i pi k.l / N) = iDFT[Q^] / h_v^3.
The linearized operator of this method is L_bin[h] = Q(M,h) + Q(h,M)
(Sec. 4.1, second method).

Two evaluations are provided: ``brute`` sums over (k, l) explicitly (small
n only) and ``fast`` uses the exact identity
    sum_l A(k-l) B(l) = n^3 DFT[iDFT[A] iDFT[B]](k)
with a library FFT; the tests pin one against the other.

Mass-conservation fixes of Sec. 2.3 (eq. (15)-(16)) are options:
    fix=1  set Q^_0 = 0
    fix=2  replace the sinc in the loss weight by its hemisphere estimate
           sum_m w_m cos(pi g_j sigma_m.l / L)
"""
import math

import numpy as np

from . import grid
from .alg1 import fft3, ifft3


def coefficients(x, L):
    """F^_k = h_v^3 DFT[x](k)."""
    n = x.shape[0]
    hv = 2.0 * L / n
    return hv ** 3 * fft3(x)


def _signed_grid(n):
    k = grid.signed_index(n).astype(np.float64)
    K = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1)   # [n,n,n,3]
    return K


def _loss_weight(plan, sphere, fix):
    n, L = plan.n, plan.L
    if fix == 2:
        sig, wm = sphere
        K = _signed_grid(n)
        out = np.zeros((n, n, n))
        for j in range(plan.J):
            c = np.cos(math.pi * plan.g[j] * np.tensordot(K, sig.T, axes=1) / L)  # [n,n,n,M]
            out += plan.W[j] * (c @ wm)
        return out
    kk = np.sqrt(grid.kabs2(n))
    return sum(plan.W[j] * grid.sinc(math.pi * plan.g[j] * kk / L) for j in range(plan.J))


def q_hat_fast(plan, sphere, Fh, Gh, fix=0):
    """Coefficients Q^_k(F, G) by the FFT identity."""
    n, L = plan.n, plan.L
    sig, wm = sphere
    K = _signed_grid(n)
    gain = np.zeros((n, n, n), dtype=np.complex128)
    for j in range(plan.J):
        acc = np.zeros((n, n, n), dtype=np.complex128)
        for m in range(len(wm)):
            a = math.pi * plan.g[j] * (K @ sig[m]) / (2.0 * L)      # a(p), p signed
            ca, sa = np.cos(a), np.sin(a)
            conv = (ifft3(Fh * ca) * ifft3(Gh * ca) + ifft3(Fh * sa) * ifft3(Gh * sa))
            acc += wm[m] * conv
        gain += plan.W[j] * plan.s[j] * n ** 3 * fft3(acc)
    wl = _loss_weight(plan, sphere, fix)
    loss = n ** 3 * fft3(ifft3(Fh) * ifft3(Gh * wl))
    Q = (2.0 * math.pi ** 2 / L ** 3) * (gain - loss)
    if fix == 1:
        Q[n // 2, n // 2, n // 2] = 0.0
    return Q


def q_hat_brute(plan, sphere, Fh, Gh, fix=0):
    """Coefficients Q^_k(F, G) by explicit double sums over k and l."""
    n, L = plan.n, plan.L
    sig, wm = sphere
    N = n // 2
    Kf = _signed_grid(n).reshape(-1, 3)                   # signed vectors
    # storage index of (k - l) reduced into -N..N-1, per axis
    dif = Kf[:, None, :] - Kf[None, :, :]
    red = (dif + N) % n - N                                # reduced signed k-l
    flat = ((red[..., 0] + N) * n + (red[..., 1] + N)) * n + (red[..., 2] + N)
    flat = flat.astype(np.int64)
    F = Fh.reshape(-1)
    G = Gh.reshape(-1)
    FG = F[flat] * G[None, :]                              # [k, l]
    arg = red - Kf[None, :, :]                             # (k-l) - l
    gain = np.zeros(n ** 3, dtype=np.complex128)
    s = plan.s.reshape(plan.J, -1)
    for j in range(plan.J):
        for m in range(len(wm)):
            c = np.cos(math.pi * plan.g[j] * (arg @ sig[m]) / (2.0 * L))
            gain += plan.W[j] * wm[m] * s[j] * np.sum(FG * c, axis=1)
    wl = _loss_weight(plan, sphere, fix).reshape(-1)
    loss = np.sum(FG * wl[None, :], axis=1)
    Q = (2.0 * math.pi ** 2 / L ** 3) * (gain - loss)
    Q = Q.reshape(n, n, n)
    if fix == 1:
        Q[N, N, N] = 0.0
    return Q


def q_binary(plan, sphere, F, G, method="fast", fix=0, parts=False):
    """Point values of Q(F, G) by eq. (14)."""
    L, n = plan.L, plan.n
    hv = 2.0 * L / n
    Fh, Gh = coefficients(F, L), coefficients(G, L)
    qf = q_hat_fast if method == "fast" else q_hat_brute
    Q = qf(plan, sphere, Fh, Gh, fix)
    return (ifft3(Q) / hv ** 3).real


def loss_only(plan, F, G):
    """Point values of the loss part of Q(F, G) (eq. (14), second line),
    returned with a positive sign."""
    L, n = plan.L, plan.n
    hv = 2.0 * L / n
    Fh, Gh = coefficients(F, L), coefficients(G, L)
    wl = _loss_weight(plan, None, 0)
    loss = (2.0 * math.pi ** 2 / L ** 3) * n ** 3 * fft3(ifft3(Fh) * ifft3(Gh * wl))
    return (ifft3(loss) / hv ** 3).real


def linearized_binary(plan, sphere, h, M, method="fast", fix=0):
    """L_bin[h] = Q(M, h) + Q(h, M) by the binary method."""
    return (q_binary(plan, sphere, M, h, method, fix)
            + q_binary(plan, sphere, h, M, method, fix))
