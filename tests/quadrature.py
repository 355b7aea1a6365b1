"""Collapsed-coordinate (Stroud conical product) Gauss-Jacobi rules on the
reference triangle and tetrahedron, generated from scipy's Jacobi roots.

Test helper: gives integrals that do not go through the oracle's exact
monomial formula, so the two can pin each other.
"""
import numpy as np
from scipy.special import roots_jacobi


def _gj01(n, alpha):
    """Nodes/weights on [0,1] for weight (1-u)^alpha."""
    t, w = roots_jacobi(n, alpha, 0.0)
    return (1 + t) / 2, w / 2 ** (alpha + 1)


def tet_rule(n):
    """Points as barycentric coordinates (npts, 4) and weights summing to 1/6."""
    u, wu = _gj01(n, 2.0)
    v, wv = _gj01(n, 1.0)
    s, ws = _gj01(n, 0.0)
    U, V, S = np.meshgrid(u, v, s, indexing="ij")
    W = (wu[:, None, None] * wv[None, :, None] * ws[None, None, :]).ravel()
    x = U.ravel()
    y = (V * (1 - U)).ravel()
    z = (S * (1 - U) * (1 - V)).ravel()
    lam = np.stack([1 - x - y - z, x, y, z], axis=1)
    return lam, W


def tri_rule(n):
    """Barycentric points (npts, 3) and weights summing to 1/2."""
    u, wu = _gj01(n, 1.0)
    v, wv = _gj01(n, 0.0)
    U, V = np.meshgrid(u, v, indexing="ij")
    W = (wu[:, None] * wv[None, :]).ravel()
    x = U.ravel()
    y = (V * (1 - U)).ravel()
    return np.stack([1 - x - y, x, y], axis=1), W
