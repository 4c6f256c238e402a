"""Host-side structure of the block-sparse interface system (Alg. 1 step 3, Alg. 2 step 3).

The interface unknowns are the nodes of internal faces.  Face numbering: all
x-normal faces, then y-normal, then z-normal; within one orientation the
faces are ordered by their lower box (bx fastest, then by, then bz).  Box
t = bx + n1*(by + n2*bz).  A face's m^2 nodes use the tangential order of the
box numbering (lower axis fastest), identical on both sides of the face.

T is kept in block-sparse row (BSR) form with m^2 x m^2 blocks.  Block row F has
one block per distinct internal face of the two boxes that share F (at most
11, paper Fig. sparsity5 / Sec. 3.3).  The diagonal block gets a contribution
from each of the two boxes: each writes an extra slot of its own (the lower box
nslot + nface + F, the upper box nslot + F) and hps_interface_reduce sets the BSR
slot to lower + upper (fixed order, no atomics; it can run again after any box
was recomputed).  This module only builds index arrays and calls the sparse LU;
the factorization of T is p-independent and is not part of the GPU hot path.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


@dataclass
class InterfaceLayout:
    nboxes: tuple
    m: int
    nface: int
    box_faces: np.ndarray       # [nbox, 6] internal face id or -1
    slot_map: np.ndarray        # [nbox, 36] int32 BSR slot per (row face, col face) of the box
    nslot: int                  # BSR blocks (unique)
    nslot_total: int            # plus the two extra diagonal slots per face
    reduce_triples: np.ndarray  # [nface, 3] int64 (dst, lower box slot, upper box slot)
    indptr: np.ndarray
    indices: np.ndarray

    @property
    def nunknown(self) -> int:
        return self.nface * self.m * self.m


def build_layout(nboxes, m: int) -> InterfaceLayout:
    n1, n2, n3 = (int(v) for v in nboxes)
    nbox = n1 * n2 * n3

    def tid(x, y, z):
        return x + n1 * (y + n2 * z)

    box_faces = np.full((nbox, 6), -1, dtype=np.int64)
    nface = 0
    dims = (n1, n2, n3)
    for axis in range(3):
        # lower boxes of faces normal to `axis`, ordered bx fastest, then by, then bz
        cz, cy, cx = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
        coords = [cx.ravel(), cy.ravel(), cz.ravel()]
        keep = coords[axis] < dims[axis] - 1
        lo = [c[keep] for c in coords]
        hi = [c.copy() for c in lo]
        hi[axis] = hi[axis] + 1
        ids = nface + np.arange(lo[0].size)
        box_faces[tid(*lo), 2 * axis + 1] = ids
        box_faces[tid(*hi), 2 * axis] = ids
        nface += lo[0].size
    # BSR pattern: (row face, col face) pairs from every box
    rows, cols = [], []
    for a in range(6):
        for b in range(6):
            ok = (box_faces[:, a] >= 0) & (box_faces[:, b] >= 0)
            rows.append(box_faces[ok, a])
            cols.append(box_faces[ok, b])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    key = np.unique(rows * max(nface, 1) + cols)
    r_u, c_u = np.divmod(key, max(nface, 1))
    nslot = key.size
    indptr = np.zeros(nface + 1, dtype=np.int64)
    np.add.at(indptr, r_u + 1, 1)
    indptr = np.cumsum(indptr)
    slot_map = np.full((nbox, 36), -1, dtype=np.int32)
    for a in range(6):
        for b in range(6):
            Fa, Fb = box_faces[:, a], box_faces[:, b]
            ok = (Fa >= 0) & (Fb >= 0)
            s = np.searchsorted(key, Fa[ok] * max(nface, 1) + Fb[ok])
            if a == b:
                # the shared diagonal block: the upper neighbour of face Fa (a on the - side)
                # and the lower one (+ side) each write an extra slot of their own
                s = nslot + Fa[ok] if a % 2 == 0 else nslot + nface + Fa[ok]
            slot_map[ok, 6 * a + b] = s
    diag_slots = np.searchsorted(key, np.arange(nface) * max(nface, 1) + np.arange(nface))
    triples = np.stack([diag_slots, nslot + nface + np.arange(nface), nslot + np.arange(nface)],
                       axis=1).astype(np.int64)
    return InterfaceLayout(nboxes=(n1, n2, n3), m=m, nface=nface, box_faces=box_faces, slot_map=slot_map,
                           nslot=nslot, nslot_total=nslot + 2 * nface, reduce_triples=triples, indptr=indptr,
                           indices=c_u.astype(np.int64))


def bsr_matrix(layout: InterfaceLayout, T_vals: np.ndarray) -> scipy.sparse.bsr_matrix:
    mm = layout.m * layout.m
    data = np.asarray(T_vals[:layout.nslot * mm * mm]).reshape(layout.nslot, mm, mm)
    n = layout.nface * mm
    return scipy.sparse.bsr_matrix((data, layout.indices, layout.indptr), shape=(n, n))


def interface_rhs(layout: InterfaceLayout, g_loads: np.ndarray) -> np.ndarray:
    """Sum of the (Dirichlet-lifted) box loads over the two boxes of each face."""
    mm = layout.m * layout.m
    rhs = np.zeros(layout.nface * mm)
    g = g_loads.reshape(-1, 6, mm)
    for a in range(6):
        F = layout.box_faces[:, a]
        ok = F >= 0
        idx = (F[ok][:, None] * mm + np.arange(mm)[None, :]).ravel()
        np.add.at(rhs, idx, g[ok, a, :].ravel())
    return rhs


def box_face_values(layout: InterfaceLayout, u_face: np.ndarray, g_dir: np.ndarray) -> np.ndarray:
    """u_b per box: interface solution on internal faces, Dirichlet data elsewhere."""
    mm = layout.m * layout.m
    nbox = layout.box_faces.shape[0]
    ub = np.array(g_dir, dtype=np.float64).reshape(nbox, 6, mm).copy()
    for a in range(6):
        F = layout.box_faces[:, a]
        ok = F >= 0
        ub[ok, a, :] = u_face.reshape(-1, mm)[F[ok]]
    return ub.reshape(nbox, 6 * mm)


def boundary_mask(layout: InterfaceLayout) -> np.ndarray:
    """[nbox, n_b] bool: True at nodes of faces on the domain boundary."""
    mm = layout.m * layout.m
    return np.repeat(layout.box_faces < 0, mm, axis=1)


class InterfaceSolver:
    """LU of T_FF on the host, reusable for many right-hand sides (and transposed solves).

    method "auto": dense LAPACK LU (multithreaded) up to DENSE_MAX unknowns, where the
    interface of a few boxes per axis at large p is small but its m^2 x m^2 blocks make
    SuperLU's supernodes slow; SciPy SuperLU with the minimum-degree ordering of
    A^T + A above that.  "dense" and "sparse" force one of the two.
    """

    DENSE_MAX = 48000

    def __init__(self, layout: InterfaceLayout, T_vals: np.ndarray, method: str = "auto"):
        self.layout = layout
        A = bsr_matrix(layout, T_vals)
        n = A.shape[0]
        if method not in ("auto", "dense", "sparse"):
            raise ValueError("method must be 'auto', 'dense' or 'sparse'")
        self.method = ("dense" if n <= self.DENSE_MAX else "sparse") if method == "auto" else method
        self.lu = None
        if n == 0:
            return
        if self.method == "dense":
            self.lu = scipy.linalg.lu_factor(A.toarray(), check_finite=False)
        else:
            self.lu = scipy.sparse.linalg.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")

    def solve(self, rhs: np.ndarray, trans: str = "N") -> np.ndarray:
        if self.lu is None:
            return np.zeros(0)
        if self.method == "dense":
            return scipy.linalg.lu_solve(self.lu, rhs, trans=0 if trans == "N" else 1, check_finite=False)
        return self.lu.solve(rhs, trans=trans)
