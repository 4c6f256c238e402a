"""Interface system of the two-level solver: numbering, assembly, solve, reconstruction.

Build stage (paper Alg. 1): every box contributes its DtN map T^t to the slots
of the sparse matrix T that belong to its faces; T is then factorized by a
sparse direct solver.  Solve stage (Alg. 2): per-box loads g^t are summed into
the interface right-hand side, the sparse system is solved for the face values
u_b, and each interior is filled in by u_i = v + S u_b.

Numbering.  Box t = bx + n1*(by + n2*bz).  Internal faces are enumerated axis by
axis (x-normal, then y-normal, then z-normal); within one axis, by the lower
box's (bx, by, bz) with bx fastest.  Both boxes index a shared face's nodes the
same way (tangential axes in increasing order), so no reorientation is needed.
Faces on the domain boundary carry Dirichlet data and are not unknowns.
Unknown index of node q on internal face F: F*m*m + q.

Dirichlet columns.  For a box face on the boundary, the columns of T^t that
multiply it are moved to the right-hand side with the known values g.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import leaf


def face_numbering(nboxes):
    """Return (box_faces [nbox, 6] with -1 on the boundary, face_boxes [nF, 2])."""
    n1, n2, n3 = nboxes
    nbox = n1 * n2 * n3
    box_faces = -np.ones((nbox, 6), dtype=np.int64)
    face_boxes = []
    dims = (n1, n2, n3)
    fid = 0
    for axis in range(3):
        for bz in range(n3):
            for by in range(n2):
                for bx in range(n1):
                    lo = [bx, by, bz]
                    if lo[axis] == dims[axis] - 1:
                        continue
                    hi = list(lo)
                    hi[axis] += 1
                    t_lo = lo[0] + n1 * (lo[1] + n2 * lo[2])
                    t_hi = hi[0] + n1 * (hi[1] + n2 * hi[2])
                    box_faces[t_lo, 2 * axis + 1] = fid  # + side of the lower box
                    box_faces[t_hi, 2 * axis + 0] = fid  # - side of the upper box
                    face_boxes.append((t_lo, t_hi))
                    fid += 1
    return box_faces, np.array(face_boxes, dtype=np.int64).reshape(-1, 2)


@dataclass
class BoxData:
    xi: np.ndarray          # interior node coordinates [n_i, 3]
    xb: np.ndarray          # face node coordinates [n_b, 3]
    b_int: np.ndarray
    f_int: np.ndarray
    blocks: leaf.LeafBlocks
    red: leaf.LeafReduction


@dataclass
class TwoLevelResult:
    boxes: List[BoxData]
    box_faces: np.ndarray
    face_boxes: np.ndarray
    T_ff: scipy.sparse.csr_matrix
    rhs: np.ndarray
    u_face: np.ndarray          # interface unknowns [nF * m * m]
    u_b: np.ndarray             # per-box face values [nbox, n_b] (Dirichlet data on the boundary)
    u_i: np.ndarray             # per-box interior values [nbox, n_i]
    lu: object                  # scipy SuperLU of T_ff


def box_setup(prob, t: int, b_field=None) -> BoxData:
    p = prob.p
    org = prob.box_origins()[t]
    xi, xb = leaf.box_node_coords(org, prob.h, p)
    bf = prob.b if b_field is None else b_field
    b_int = bf(xi)
    f_int = prob.f(xi)
    blk = leaf.local_blocks(p, prob.h, prob.kappa, b_int)
    red = leaf.leaf_reduce(blk, f_int)
    return BoxData(xi=xi, xb=xb, b_int=b_int, f_int=f_int, blocks=blk, red=red)


def assemble(prob, boxes: List[BoxData]):
    """T_FF and its right-hand side from the per-box DtN maps and loads (Alg. 1, Alg. 2)."""
    m = prob.p - 2
    mm = m * m
    box_faces, face_boxes = face_numbering(prob.nboxes)
    nF = face_boxes.shape[0]
    rows, cols, vals = [], [], []
    rhs = np.zeros(nF * mm)
    for t, bd in enumerate(boxes):
        T = bd.red.T
        g_dir = prob.g(bd.xb)
        for a in range(6):
            Fa = box_faces[t, a]
            if Fa < 0:
                continue
            ra = slice(a * mm, (a + 1) * mm)
            rhs[Fa * mm:(Fa + 1) * mm] += bd.red.g[ra]
            for b in range(6):
                Fb = box_faces[t, b]
                cb = slice(b * mm, (b + 1) * mm)
                blk = T[ra, cb]
                if Fb < 0:
                    rhs[Fa * mm:(Fa + 1) * mm] -= blk @ g_dir[cb]
                else:
                    R, C = np.meshgrid(np.arange(mm) + Fa * mm, np.arange(mm) + Fb * mm, indexing="ij")
                    rows.append(R.ravel())
                    cols.append(C.ravel())
                    vals.append(blk.ravel())
    if rows:
        T_ff = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                       shape=(nF * mm, nF * mm)).tocsr()
    else:
        T_ff = scipy.sparse.csr_matrix((0, 0))
    return T_ff, rhs, box_faces, face_boxes


def face_values(prob, boxes, box_faces, u_face):
    """Per-box face values: interface solution on internal faces, g on the boundary."""
    m = prob.p - 2
    mm = m * m
    u_b = np.zeros((len(boxes), 6 * mm))
    for t, bd in enumerate(boxes):
        g_dir = prob.g(bd.xb)
        for a in range(6):
            sl = slice(a * mm, (a + 1) * mm)
            F = box_faces[t, a]
            u_b[t, sl] = g_dir[sl] if F < 0 else u_face[F * mm:(F + 1) * mm]
    return u_b


def _lean(bd: BoxData) -> BoxData:
    """Keep only what assembly and reconstruction read (S, v, T, g); drops the dense
    blocks, X and the LU factors, which dominate memory at large p."""
    red = leaf.LeafReduction(X=None, S=bd.red.S, T=bd.red.T, v=bd.red.v, g=bd.red.g, lu=None)
    return BoxData(xi=bd.xi, xb=bd.xb, b_int=bd.b_int, f_int=bd.f_int, blocks=None, red=red)


def solve(prob, b_field=None, keep_boxes: bool = True, progress=None, dense: bool = False) -> TwoLevelResult:
    """Two-level solve: all leaf reductions, sparse interface solve, reconstruction.

    keep_boxes=False keeps per box only S, v, T and g (same arithmetic, less memory);
    dense=True solves the interface system with dense LAPACK LU instead of SuperLU
    (the same system; SuperLU's fill makes it far slower once the faces carry
    hundreds of nodes each); progress(msg) is called after each box and phase.
    """
    boxes = []
    for t in range(prob.nbox):
        bd = box_setup(prob, t, b_field)
        boxes.append(bd if keep_boxes else _lean(bd))
        if progress:
            progress(f"box {t + 1}/{prob.nbox}")
    T_ff, rhs, box_faces, face_boxes = assemble(prob, boxes)
    if progress:
        progress(f"interface matrix {T_ff.shape[0]} unknowns, {T_ff.nnz} nonzeros")
    if T_ff.shape[0] > 0 and dense:
        lu = None
        u_face = np.linalg.solve(T_ff.toarray(), rhs)
    elif T_ff.shape[0] > 0:
        lu = scipy.sparse.linalg.splu(T_ff.tocsc())
        u_face = lu.solve(rhs)
    else:
        lu, u_face = None, np.zeros(0)
    if progress:
        progress("interface solve done")
    u_b = face_values(prob, boxes, box_faces, u_face)
    u_i = np.stack([bd.red.v + bd.red.S @ u_b[t] for t, bd in enumerate(boxes)])
    return TwoLevelResult(boxes=boxes, box_faces=box_faces, face_boxes=face_boxes, T_ff=T_ff, rhs=rhs,
                          u_face=u_face, u_b=u_b, u_i=u_i, lu=lu)


def rel_l2(a, b) -> float:
    """Relative l2 error ||a - b|| / ||b|| (the paper's error measure, Sec. 4)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
