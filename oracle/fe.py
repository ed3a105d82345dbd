"""Q1/Q2 Lagrange elements on squares and Gauss quadrature (oracle).

Test infrastructure only.

Sec. 3 discretises both displacement and phase field with H^1-conforming
tensor-product Lagrange elements (bilinear in the paper; biquadratic is the
same construction with p = 2). Quadrature: Gauss-Legendre with p + 1 points
per direction. On an axis-aligned square of edge H, gradients are the
reference gradients divided by H and JxW = H^2 * w_ref.
"""
from __future__ import annotations

import numpy as np


def gauss_01(n: int):
    """Gauss-Legendre points and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def basis_1d(p: int, s):
    """Equispaced Lagrange basis of degree p and its derivative at points s.

    Returns (val, der), each of shape (len(s), p + 1)."""
    s = np.atleast_1d(np.asarray(s, dtype=float))
    nodes = np.arange(p + 1) / p
    val = np.ones((s.size, p + 1))
    der = np.zeros((s.size, p + 1))
    for k in range(p + 1):
        others = [m for m in range(p + 1) if m != k]
        denom = np.prod([nodes[k] - nodes[m] for m in others])
        for m in others:
            val[:, k] *= (s - nodes[m])
        val[:, k] /= denom
        # product rule
        for r in others:
            term = np.ones(s.size)
            for m in others:
                if m != r:
                    term *= (s - nodes[m])
            der[:, k] += term
        der[:, k] /= denom
    return val, der


class Element:
    """Reference Q_p square: values and gradients of the (p+1)^2 shape
    functions at the (p+1)^2 Gauss points.

    Point q = qx + (p+1) qy, shape function k = a + (p+1) b,
    N_k(x, y) = l_a(x) l_b(y)."""

    def __init__(self, p: int):
        self.p = p
        n1 = p + 1
        self.nloc = n1 * n1
        g, w = gauss_01(n1)
        v, d = basis_1d(p, g)
        self.nq = n1 * n1
        self.N = np.zeros((self.nq, self.nloc))
        self.dNx = np.zeros((self.nq, self.nloc))
        self.dNy = np.zeros((self.nq, self.nloc))
        self.w = np.zeros(self.nq)
        self.qpts = np.zeros((self.nq, 2))
        for qy in range(n1):
            for qx in range(n1):
                q = qx + n1 * qy
                self.w[q] = w[qx] * w[qy]
                self.qpts[q] = (g[qx], g[qy])
                for b in range(n1):
                    for a in range(n1):
                        k = a + n1 * b
                        self.N[q, k] = v[qx, a] * v[qy, b]
                        self.dNx[q, k] = d[qx, a] * v[qy, b]
                        self.dNy[q, k] = v[qx, a] * d[qy, b]
