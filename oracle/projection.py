"""Projection onto the complement of the collision invariants (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Fourier method does not conserve momentum or energy (Sec. 2.3) and the
paper only tries the mass fix Q^_0 = 0 (Sec. 4.2).  The library offers a
post-processing projection instead: with phi_a in {1, v1, v2, v3, |v|^2},
    A_ab  = sum_l M phi_a phi_b,      m_a[x] = sum_l x phi_a,
    P x   = x - M sum_a phi_a (A^-1 m[x])_a,
the orthogonal projector, in the inner product <a, b> = sum a b / M, onto
the complement of span{phi_a M}.  Then m[P x] = 0 and P(phi_a M) = 0, so
P L P conserves mass, momentum and energy exactly and annihilates the
collision invariants exactly.
"""
import numpy as np

from . import grid


def invariants(n, L):
    """[5, n, n, n]: 1, v1, v2, v3, |v|^2 on the grid."""
    v = grid.velocities(n, L)
    VX, VY, VZ = np.meshgrid(v, v, v, indexing="ij")
    return np.stack([np.ones_like(VX), VX, VY, VZ, VX ** 2 + VY ** 2 + VZ ** 2])


def moments(x, phis):
    return np.tensordot(phis, x, axes=([1, 2, 3], [0, 1, 2]))


def gram(M, phis):
    return np.einsum("aijk,bijk,ijk->ab", phis, phis, M)


def project(x, M, phis):
    A = gram(M, phis)
    c = np.linalg.solve(A, moments(x, phis))
    return x - M * np.tensordot(c, phis, axes=1)
