"""Local collocation blocks of one leaf box and the per-box reduction.

Node numbering of one box (p nodes per axis, m = p - 2 interior per axis):
  full grid   (i, j, k) -> i + p*j + p*p*k, i along x fastest.
  interior    (i, j, k) in [1, p-2]^3 -> (i-1) + m*(j-1) + m*m*(k-1).
  faces       x-, x+, y-, y+, z-, z+ (face a = 2*axis + side); each face has m*m
              nodes indexed by its two tangential axes in increasing axis order,
              the lower axis fastest; face node index = a*m*m + local.
  Edge and corner nodes are not unknowns (paper Remark 1: without cross
  derivative terms no equation touches them).

Rows of the box operator (paper eq. Aentries):
  interior node x_i:  (A u)(x_i) = -Lap u - kappa^2 b u, by collocation with the
                      tensor Chebyshev differentiation matrices.
  face node:          the outward normal derivative of u computed from this box
                      (the interface equation sums it over the two boxes).
The partition into [A_ii A_ib; A_bi A_bb] is paper Sec. 2.2, eq. blocksys1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import cheb


def interior_full_index(p: int) -> np.ndarray:
    m = p - 2
    r = np.arange(1, p - 1)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return (i + p * j + p * p * k).ravel()


def face_full_index(p: int) -> np.ndarray:
    """Full-grid index of the 6*m*m face nodes in face order x-, x+, y-, y+, z-, z+."""
    r = np.arange(1, p - 1)
    out = []
    for axis in range(3):
        for side in range(2):
            e = 0 if side == 0 else p - 1
            s, f = np.meshgrid(r, r, indexing="ij")  # f fastest after ravel
            # tangential axes in increasing order; the lower one runs fastest
            tang = [a for a in range(3) if a != axis]
            ijk = [None, None, None]
            ijk[axis] = np.full(f.size, e)
            ijk[tang[0]] = f.ravel()
            ijk[tang[1]] = s.ravel()
            out.append(ijk[0] + p * ijk[1] + p * p * ijk[2])
    return np.concatenate(out)


def edge_corner_full_index(p: int) -> np.ndarray:
    everything = np.arange(p ** 3)
    keep = np.concatenate([interior_full_index(p), face_full_index(p)])
    return np.setdiff1d(everything, keep)


def box_node_coords(origin, h, p: int):
    """Coordinates of the interior nodes [n_i, 3] and face nodes [n_b, 3] of a box."""
    ax = [cheb.box_axis_coords(origin[a], h[a], p) for a in range(3)]
    full = np.zeros((p ** 3, 3))
    K, J, I = np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij")
    full[:, 0] = ax[0][I.ravel()]
    full[:, 1] = ax[1][J.ravel()]
    full[:, 2] = ax[2][K.ravel()]
    return full[interior_full_index(p)], full[face_full_index(p)]


def full_operator_rows(p: int, h, kappa: float, b_full: np.ndarray) -> np.ndarray:
    """Collocated -Lap - kappa^2 b on the full p^3 grid of a box (dense, p^3 x p^3).

    d/dx on [lo, lo+h] is (2/h) d/dt on [-1,1]; the second derivative along each
    axis is (2/h)^2 D D applied along that axis.
    """
    D = cheb.diffmat(p)
    D2 = D @ D
    I = np.eye(p)
    dxx = (2.0 / h[0]) ** 2 * D2
    dyy = (2.0 / h[1]) ** 2 * D2
    dzz = (2.0 / h[2]) ** 2 * D2
    # index i + p j + p^2 k: kron(slow, fast)
    lap = (np.kron(I, np.kron(I, dxx)) + np.kron(I, np.kron(dyy, I)) + np.kron(dzz, np.kron(I, I)))
    return -lap - kappa ** 2 * np.diag(b_full)


def neumann_rows(p: int, h) -> np.ndarray:
    """Outward normal derivative at every face node, as rows over the full grid.

    Face x- (i = 0) has outward normal -e_x, so its row is -(2/h_x) D[0, :] along
    the x-line through the node; face x+ uses +(2/h_x) D[p-1, :]; same for y, z.
    """
    D = cheb.diffmat(p)
    fidx = face_full_index(p)
    m = p - 2
    N = np.zeros((6 * m * m, p ** 3))
    for a in range(6):
        axis, side = divmod(a, 2)
        e = 0 if side == 0 else p - 1
        sign = -1.0 if side == 0 else 1.0
        stride = p ** axis
        for q in range(m * m):
            row = a * m * m + q
            node = fidx[row]
            base = node - e * stride  # same line, coordinate 0 along `axis`
            for l in range(p):
                N[row, base + l * stride] += sign * (2.0 / h[axis]) * D[e, l]
    return N


@dataclass
class LeafBlocks:
    A_ii: np.ndarray
    A_ib: np.ndarray
    A_bi: np.ndarray
    A_bb: np.ndarray


def local_blocks(p: int, h, kappa: float, b_int: np.ndarray) -> LeafBlocks:
    """The four blocks of eq. blocksys1 for one box; b_int is b at the interior nodes.

    b only enters interior rows, on the diagonal of A_ii, so its values at face,
    edge and corner nodes never matter (they are set to 0 here).
    """
    ii = interior_full_index(p)
    fb = face_full_index(p)
    b_full = np.zeros(p ** 3)
    b_full[ii] = b_int
    L = full_operator_rows(p, h, kappa, b_full)[ii]
    N = neumann_rows(p, h)
    return LeafBlocks(A_ii=L[:, ii], A_ib=L[:, fb], A_bi=N[:, ii], A_bb=N[:, fb])


@dataclass
class LeafReduction:
    X: np.ndarray       # A_ii^{-1} [A_ib | f_i], n_i x (n_b + 1)
    S: np.ndarray       # solution operator -A_ii^{-1} A_ib
    T: np.ndarray       # DtN map A_bb + A_bi S
    v: np.ndarray       # A_ii^{-1} f_i
    g: np.ndarray       # equivalent load f_b - A_bi v with f_b = 0
    lu: tuple           # scipy LU factors of A_ii (for transposed solves)


def leaf_reduce(blk: LeafBlocks, f_int: np.ndarray) -> LeafReduction:
    """Per-box reduction of Alg. 1 (build) and the load step of Alg. 2.

    S = -A_ii^{-1} A_ib and T = A_bb + A_bi S (Sec. 2.2; eq. t-block keeps the
    A_bb term), v = A_ii^{-1} f_i and g = f_b - A_bi v (Alg. 2), with f_b = 0
    because the interface equations of eq. Aentries have zero right-hand side.
    """
    lu = scipy.linalg.lu_factor(blk.A_ii)
    B = np.concatenate([blk.A_ib, f_int[:, None]], axis=1)
    X = scipy.linalg.lu_solve(lu, B)
    S = -X[:, :-1]
    v = X[:, -1]
    T = blk.A_bb + blk.A_bi @ S
    g = -blk.A_bi @ v
    return LeafReduction(X=X, S=S, T=T, v=v, g=g, lu=lu)


def interior_solve(blk: LeafBlocks, f_int: np.ndarray, u_b: np.ndarray) -> np.ndarray:
    """u_i = A_ii^{-1} (f_i - A_ib u_b): the interior solution given face values."""
    return np.linalg.solve(blk.A_ii, f_int - blk.A_ib @ u_b)
