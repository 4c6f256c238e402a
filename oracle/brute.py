"""The global collocation system of paper eq. Aentries, formed densely and solved directly.

Unknowns: the interior nodes of every box (box-major, the box's interior order),
then the nodes of every internal face (face-major, see interface.face_numbering).
Equations:
  * one collocation row -Lap u - kappa^2 b u = f at every box-interior node;
  * one row per internal-face node: the sum of the outward normal derivatives
    computed from the two boxes sharing the face equals 0.
Dirichlet face values are known and moved to the right-hand side.  Edge and
corner nodes appear in no row (Remark 1) and are not unknowns.

No static condensation is involved, so agreement with the two-level result pins
the Schur complement, the assembly and all index maps at once.  Feasible only
for small grids (2x2x2 boxes with p <= 10 is 4864 unknowns).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import leaf
from .interface import face_numbering


@dataclass
class GlobalSystem:
    A: np.ndarray
    rhs: np.ndarray
    n_int: int          # number of interior unknowns (nbox * n_i)
    n_face: int         # number of face unknowns
    b_int: np.ndarray   # [nbox, n_i]


def assemble_global(prob, b_field=None) -> GlobalSystem:
    p = prob.p
    m = p - 2
    mm = m * m
    ni = m ** 3
    nbox = prob.nbox
    box_faces, face_boxes = face_numbering(prob.nboxes)
    nF = face_boxes.shape[0]
    n_int = nbox * ni
    n = n_int + nF * mm
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    ii = leaf.interior_full_index(p)
    fb = leaf.face_full_index(p)
    N = leaf.neumann_rows(p, prob.h)
    bf = prob.b if b_field is None else b_field
    origins = prob.box_origins()
    b_all = np.zeros((nbox, ni))

    for t in range(nbox):
        xi, xb = leaf.box_node_coords(origins[t], prob.h, p)
        b_int = bf(xi)
        b_all[t] = b_int
        b_full = np.zeros(p ** 3)
        b_full[ii] = b_int
        L = leaf.full_operator_rows(p, prob.h, prob.kappa, b_full)
        g_b = prob.g(xb)
        # map full-grid column -> global unknown (or Dirichlet value)
        col_unknown = -np.ones(p ** 3, dtype=np.int64)
        col_known = np.zeros(p ** 3)
        col_unknown[ii] = t * ni + np.arange(ni)
        for a in range(6):
            F = box_faces[t, a]
            idx = fb[a * mm:(a + 1) * mm]
            if F >= 0:
                col_unknown[idx] = n_int + F * mm + np.arange(mm)
            else:
                col_known[idx] = g_b[a * mm:(a + 1) * mm]
        # interior collocation rows
        rows = t * ni + np.arange(ni)
        Lr = L[ii]
        unk = col_unknown >= 0
        A[np.ix_(rows, col_unknown[unk])] += Lr[:, unk]
        rhs[rows] = prob.f(xi) - Lr[:, ~unk] @ col_known[~unk]
        # this box's share of the interface rows of its internal faces
        for a in range(6):
            F = box_faces[t, a]
            if F < 0:
                continue
            Nr = N[a * mm:(a + 1) * mm]
            frows = n_int + F * mm + np.arange(mm)
            A[np.ix_(frows, col_unknown[unk])] += Nr[:, unk]
            rhs[frows] -= Nr[:, ~unk] @ col_known[~unk]
    return GlobalSystem(A=A, rhs=rhs, n_int=n_int, n_face=nF * mm, b_int=b_all)


def solve_global(prob, b_field=None):
    """Return (u_int [nbox, n_i], u_face [nF*m*m], system) from a dense direct solve."""
    sysm = assemble_global(prob, b_field)
    u = np.linalg.solve(sysm.A, sysm.rhs)
    ni = (prob.p - 2) ** 3
    return u[:sysm.n_int].reshape(prob.nbox, ni), u[sysm.n_int:], sysm
