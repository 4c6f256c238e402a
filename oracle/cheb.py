"""Chebyshev-Gauss-Lobatto nodes and spectral differentiation (paper Sec. 2.1).

Each leaf box carries a tensor grid of p Chebyshev nodes per axis, shared with
neighbours on faces, and the PDE is imposed by spectral collocation.  The nodes
must include the interval end points because faces are shared, so these are the
Gauss-Lobatto points.  The differentiation matrix is the barycentric one for
those points (the formula in Trefethen, Spectral Methods in MATLAB, ch. 6),
with the diagonal set so that every row sums to zero.
"""
from __future__ import annotations

import numpy as np


def nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto points on [-1, 1] in ascending order: t_j = -cos(pi j/(p-1))."""
    if p < 2:
        raise ValueError("p must be >= 2")
    j = np.arange(p, dtype=np.float64)
    return -np.cos(np.pi * j / (p - 1))


def diffmat(p: int) -> np.ndarray:
    """Differentiation matrix D on the p Gauss-Lobatto points of [-1, 1].

    Off-diagonal: D_ij = (c_i / c_j) (-1)^(i+j) / (t_i - t_j) with c = 2 at the
    two end points and 1 elsewhere; diagonal: D_ii = -sum_{j != i} D_ij.
    (D u)_i is the derivative at t_i of the degree p-1 interpolant of u.
    """
    t = nodes(p)
    c = np.ones(p)
    c[0] = c[-1] = 2.0
    D = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1.0) ** (i + j) / (t[i] - t[j])
    for i in range(p):
        D[i, i] = -np.sum(D[i, :])  # D[i, i] is still 0 here
    return D


def box_axis_coords(lo: float, h: float, p: int) -> np.ndarray:
    """Physical node coordinates along one axis of the box [lo, lo+h]."""
    return lo + 0.5 * h * (nodes(p) + 1.0)
