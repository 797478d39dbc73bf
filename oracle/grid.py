"""Collocation grid and discrete Fourier conventions (Sec. 2.3).

The paper's N is half the number of points per axis; here n = 2N is the
number of points (and Fourier modes) per axis.  Storage index i in [0, n)
corresponds to the signed index l = i - N and the velocity
v = l L / N = -L + i h_v, h_v = 2L/n.

Transforms follow the paper's index sets exactly (no FFT):
    DFT[x](k)  = sum_{l=-N}^{N-1} x(l) exp(-i pi k.l / N),   k = -N..N-1
    iDFT[X](l) = n^-3 sum_{k=-N}^{N-1} X(k) exp(+i pi k.l / N)
applied as dense per-axis matrices (O(n^4) per 3-D transform).  Frequencies
are stored like velocities: storage index K = k + N.
"""
import numpy as np


def signed_index(n):
    """Signed indices -N..N-1 in storage order."""
    return np.arange(n) - n // 2


def velocities(n, L):
    """1-D velocity nodes v_l = l L / N, l = -N..N-1."""
    return signed_index(n) * (2.0 * L / n)


def kabs2(n):
    """|k|^2 on the 3-D frequency grid (k_d in -N..N-1; the Nyquist index
    -N contributes N^2)."""
    k = signed_index(n).astype(np.float64)
    return k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2


def dft_matrix(n):
    """1-D forward DFT matrix F[k, l] = exp(-2 pi i k l / n) over signed
    indices."""
    l = signed_index(n)
    return np.exp(-2j * np.pi * np.outer(l, l) / n)


def _apply_axes(A, x):
    y = np.tensordot(A, x, axes=([1], [0]))          # axis 0
    y = np.tensordot(A, y, axes=([1], [1])).transpose(1, 0, 2)   # axis 1
    y = np.tensordot(A, y, axes=([1], [2])).transpose(1, 2, 0)   # axis 2
    return y


def dft3(x):
    """3-D DFT by dense per-axis matrices (paper's sign and index set)."""
    n = x.shape[0]
    return _apply_axes(dft_matrix(n), x.astype(np.complex128))


def idft3(X):
    """3-D inverse DFT with the 1/n^3 factor."""
    n = X.shape[0]
    return _apply_axes(np.conj(dft_matrix(n)), X.astype(np.complex128)) / n ** 3


def sinc(x):
    """Unnormalised sinc, sin(x)/x with sinc(0) = 1 (the paper's sinc;
    eq. (16) fixes the normalisation)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0.0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out
