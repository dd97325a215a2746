"""Q1 reference element on [-1,1]^d with the 2-point Gauss rule per axis.

Section 3 of the paper discretises with bilinear / trilinear Q1^c elements on quads and
hexahedra.  The quadrature rule is not stated; the 2-point Gauss-Legendre rule per axis
(exact for Q1 x Q1 mass integrands on affine cells) is the reading used throughout.

Vertex numbering: vertex a has bit k of a set when it sits at +1 along axis k
(lexicographic, x fastest).  Gauss point q uses the same bit pattern for the sign of
+-1/sqrt(3).

Pinned by tests/test_oracle_basics.py (test_partition_of_unity_and_linear_reproduction,
test_textbook_mass_and_laplacian_2d / _3d: textbook mass and Laplacian element matrices).
"""
import numpy as np


def signs(dim):
    """s[a, k] = +-1: the side of vertex a along axis k."""
    n = 1 << dim
    return np.array([[2 * ((a >> k) & 1) - 1 for k in range(dim)] for a in range(n)], dtype=np.float64)


def gauss_points(dim):
    """Reference coordinates of the 2^d Gauss points, weights are all 1."""
    return signs(dim) / np.sqrt(3.0)


def shape(dim, xi):
    """N[p, a] at reference points xi[p, dim]."""
    s = signs(dim)
    xi = np.atleast_2d(xi)
    out = np.ones((xi.shape[0], s.shape[0]))
    for k in range(dim):
        out *= 0.5 * (1.0 + xi[:, k:k + 1] * s[None, :, k])
    return out


def shape_grad(dim, xi):
    """dN[p, a, k] = d N_a / d xi_k at reference points xi[p, dim]."""
    s = signs(dim)
    xi = np.atleast_2d(xi)
    nv = s.shape[0]
    out = np.ones((xi.shape[0], nv, dim))
    for k in range(dim):
        for m in range(dim):
            if m == k:
                out[:, :, k] *= 0.5 * s[None, :, m]
            else:
                out[:, :, k] *= 0.5 * (1.0 + xi[:, m:m + 1] * s[None, :, m])
    return out


def reference(dim):
    """(N[q,a], dN[q,a,k], w[q]) at the Gauss points of the reference cell."""
    xq = gauss_points(dim)
    return shape(dim, xq), shape_grad(dim, xq), np.ones(xq.shape[0])
