"""Gradient of a data misfit with respect to the coefficient b (adjoint method).

J(b) = 1/2 sum_k (u(x_k) - d_k)^2 over box-interior collocation nodes x_k, where
u solves the global collocation system A(b) u = rhs of eq. Aentries.  b enters A
only as -kappa^2 b on the diagonal of the interior collocation rows, so
    dJ/db_n = kappa^2 * lambda_n * u_n,   A^T lambda = P^T (P u - d),
at interior nodes and 0 elsewhere.

Two routes:
  two_level_gradient   transposes the factorization of eq. factor1/factor2:
                       A^{-T} = Atil^{-T} L^{-T} D^{-T} U^{-T}, i.e. per box
                       z = A_ii^{-T} w_i, y_b = w_b - A_ib^T z (summed over the two
                       boxes of each face), lambda_b = T^{-T} y_b, and
                       lambda_i = A_ii^{-T} (w_i - A_bi^T lambda_b).
  brute_gradient       solves A^T lambda = P^T r with the dense global matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import brute, interface


def obs_local_index(obs_nodes: np.ndarray, p: int) -> np.ndarray:
    """(t, i, j, k) grid indices -> (t, interior local index)."""
    m = p - 2
    t, i, j, k = obs_nodes.T
    return np.stack([t, (i - 1) + m * (j - 1) + m * m * (k - 1)], axis=1)


def misfit(u_i: np.ndarray, obs_nodes: np.ndarray, data: np.ndarray, p: int) -> float:
    tl = obs_local_index(obs_nodes, p)
    r = u_i[tl[:, 0], tl[:, 1]] - data
    return 0.5 * float(r @ r)


def observe(u_i: np.ndarray, obs_nodes: np.ndarray, p: int) -> np.ndarray:
    tl = obs_local_index(obs_nodes, p)
    return u_i[tl[:, 0], tl[:, 1]].copy()


def two_level_gradient(prob, obs_nodes, data, b_field=None):
    """Return (J, grad [nbox, n_i], forward result) through the two-level factorization."""
    res = interface.solve(prob, b_field)
    p = prob.p
    m = p - 2
    mm = m * m
    tl = obs_local_index(obs_nodes, p)
    r = res.u_i[tl[:, 0], tl[:, 1]] - data
    J = 0.5 * float(r @ r)
    w = np.zeros_like(res.u_i)
    w[tl[:, 0], tl[:, 1]] = r
    nF = res.face_boxes.shape[0]
    y_face = np.zeros(nF * mm)
    z = []
    for t, bd in enumerate(res.boxes):
        zt = scipy.linalg.lu_solve(bd.red.lu, w[t], trans=1)
        z.append(zt)
        yb = -bd.blocks.A_ib.T @ zt
        for a in range(6):
            F = res.box_faces[t, a]
            if F >= 0:
                y_face[F * mm:(F + 1) * mm] += yb[a * mm:(a + 1) * mm]
    lam_face = res.lu.solve(y_face, trans="T") if nF > 0 else np.zeros(0)
    grad = np.zeros_like(res.u_i)
    for t, bd in enumerate(res.boxes):
        lam_b = np.zeros(6 * mm)
        for a in range(6):
            F = res.box_faces[t, a]
            if F >= 0:
                lam_b[a * mm:(a + 1) * mm] = lam_face[F * mm:(F + 1) * mm]
        lam_i = scipy.linalg.lu_solve(bd.red.lu, w[t] - bd.blocks.A_bi.T @ lam_b, trans=1)
        grad[t] = prob.kappa ** 2 * lam_i * res.u_i[t]
    return J, grad, res


def brute_gradient(prob, obs_nodes, data, b_field=None):
    """Return (J, grad [nbox, n_i]) from the dense global system."""
    u_int, u_face, sysm = brute.solve_global(prob, b_field)
    p = prob.p
    tl = obs_local_index(obs_nodes, p)
    r = u_int[tl[:, 0], tl[:, 1]] - data
    rhs = np.zeros(sysm.A.shape[0])
    ni = (p - 2) ** 3
    rhs[tl[:, 0] * ni + tl[:, 1]] = r
    lam = np.linalg.solve(sysm.A.T, rhs)
    grad = prob.kappa ** 2 * lam[:sysm.n_int].reshape(prob.nbox, ni) * u_int
    return 0.5 * float(r @ r), grad
