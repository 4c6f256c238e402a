"""Interface system T u_F = rhs factored and solved on the GPU by nested dissection.

The paper factors the block-sparse interface matrix T with a multifrontal CPU solver
(Sec. 3.1, Alg. 1 step 3) and notes that this factorization dominates the build
stage (Sec. 3.3, Sec. 4.2).  Here the same elimination runs on the GPU with dense
fronts (fronts.hip through the C ABI):

* the box grid is bisected recursively along its longest axis (ties: the lowest
  axis) down to single boxes; a node's separator P is the set of faces between its
  two halves, its boundary B the faces on its outer boundary that are internal to
  the domain;
* a single box passes up its DtN map T^tau on its internal faces (the blocks the
  build wrote to its own slots of T_vals, before the diagonal blocks are summed);
* a node's front [[A_PP, A_PB], [A_BP, A_BB]] is the extend-add of its two halves'
  Schur complements (first half, then second: a fixed order of every sum), and its
  partial LU (pivots inside P) leaves the Schur complement on B for its parent;
* the solve runs the forward substitution up the tree (each front's load is the
  extend-add of its halves' reduced loads; a box contributes its lifted load) and the
  backward one down (each front reads its boundary values from the solution of the
  faces above it).

Nodes of equal height and front shape are factored and solved in one batched call.
This module only builds index lists and calls the library; every arithmetic step
runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import check
from .interface import InterfaceLayout
from .leaf import _ptr, _stream


def _ru(x: int, a: int) -> int:
    return (x + a - 1) // a * a


@dataclass
class _Node:
    lo: Tuple[int, int, int]
    hi: Tuple[int, int, int]
    box: int = -1                  # leaf: the box id
    kids: List["_Node"] = field(default_factory=list)
    P: List[int] = field(default_factory=list)   # separator faces (sorted)
    B: List[int] = field(default_factory=list)   # boundary faces internal to the domain (sorted)
    height: int = 0
    n_piv: int = 0
    n: int = 0
    group: Optional["_Group"] = None
    slot: int = 0                  # index inside its group

    def pos(self, face: int, mm: int) -> int:
        """Offset of a face's first unknown inside this node's front."""
        if face in self._pidx:
            return self._pidx[face] * mm
        return self.n_piv + self._bidx[face] * mm


@dataclass
class _Group:
    height: int
    n: int
    n_piv: int
    nP: int
    nB: int
    nodes: List[_Node] = field(default_factory=list)
    f_base: int = 0     # element offset of the first front in the front buffer
    v_base: int = 0     # element offset of the first vector in the vector buffer
    i_base: int = 0     # front index of the first front (perm / dinv / info rows)


class _FrontPlan:
    def __init__(self, lib, n: int, n_piv: int):
        self.lib = lib
        h = C.c_void_p()
        check(lib.hps_front_plan_create(C.byref(h), int(n), int(n_piv)), "hps_front_plan_create")
        self.handle = h
        self.dinv_elems = int(lib.hps_front_dinv_elems(h))

    def __del__(self):
        try:
            if self.handle:
                self.lib.hps_front_plan_destroy(self.handle)
        except Exception:
            pass


class DissectionLayout:
    """The dissection tree, front shapes and extend-add task lists (host only, no GPU).

    Task arrays are int64 element offsets: block tasks (dst, src, dst row stride, src row
    stride) into the front buffer (src: T_vals for box halves, the front buffer for
    internal halves); segment tasks (dst, src) for the vectors."""

    def __init__(self, layout: InterfaceLayout):
        self.layout = layout
        self.mm = layout.m * layout.m
        n1, n2, n3 = layout.nboxes
        self.dims = (n1, n2, n3)
        self.root = self._build((0, 0, 0), (n1, n2, n3))
        self.groups: List[_Group] = []
        self._plan_groups()

    # ---- tree ----------------------------------------------------------------------
    def _box(self, x, y, z) -> int:
        n1, n2, _ = self.dims
        return x + n1 * (y + n2 * z)

    def _range_faces(self, lo, hi):
        """Internal faces on the outer boundary of box range [lo, hi)."""
        bf = self.layout.box_faces
        out = []
        for a in range(3):
            for side in (0, 1):
                c = lo[a] if side == 0 else hi[a] - 1
                rng = [range(lo[k], hi[k]) if k != a else range(c, c + 1) for k in range(3)]
                for z in rng[2]:
                    for y in rng[1]:
                        for x in rng[0]:
                            f = bf[self._box(x, y, z), 2 * a + side]
                            if f >= 0:
                                out.append(int(f))
        return sorted(out)

    def _build(self, lo, hi) -> _Node:
        ext = [hi[a] - lo[a] for a in range(3)]
        node = _Node(lo=tuple(lo), hi=tuple(hi))
        node.B = self._range_faces(lo, hi)
        if max(ext) == 1:
            node.box = self._box(*lo)
            node._pidx, node._bidx = {}, {f: i for i, f in enumerate(node.B)}
            return node
        a = int(np.argmax(ext))  # longest axis, lowest on ties
        mid = lo[a] + ext[a] // 2
        hi1 = list(hi)
        hi1[a] = mid
        lo2 = list(lo)
        lo2[a] = mid
        node.kids = [self._build(lo, tuple(hi1)), self._build(tuple(lo2), hi)]
        bf = self.layout.box_faces
        P = []
        rng = [range(lo[k], hi[k]) if k != a else range(mid - 1, mid) for k in range(3)]
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    P.append(int(bf[self._box(x, y, z), 2 * a + 1]))
        node.P = sorted(P)
        node.height = 1 + max(k.height for k in node.kids)
        node.n_piv = _ru(len(node.P) * self.mm, 64)
        node.n = node.n_piv + _ru(len(node.B) * self.mm, 32)
        node._pidx = {f: i for i, f in enumerate(node.P)}
        node._bidx = {f: i for i, f in enumerate(node.B)}
        return node

    def _internal_nodes(self) -> List[_Node]:
        out, stack = [], [self.root]
        while stack:
            nd = stack.pop()
            if nd.box < 0:
                out.append(nd)
                stack.extend(nd.kids)
        return out

    # ---- groups, buffers, task lists -----------------------------------------------------
    def _plan_groups(self):
        mm = self.mm
        nodes = sorted(self._internal_nodes(), key=lambda nd: (nd.height, nd.lo[2], nd.lo[1], nd.lo[0]))
        keyed: Dict[tuple, _Group] = {}
        for nd in nodes:
            key = (nd.height, nd.n, nd.n_piv, len(nd.P), len(nd.B))
            if key not in keyed:
                keyed[key] = _Group(height=nd.height, n=nd.n, n_piv=nd.n_piv, nP=len(nd.P), nB=len(nd.B))
                self.groups.append(keyed[key])
            g = keyed[key]
            nd.group, nd.slot = g, len(g.nodes)
            g.nodes.append(nd)
        f_tot = v_tot = i_tot = 0
        for g in self.groups:
            g.f_base, g.v_base, g.i_base = f_tot, v_tot, i_tot
            f_tot += len(g.nodes) * g.n * g.n
            v_tot += len(g.nodes) * g.n
            i_tot += len(g.nodes)
        self.front_elems, self.vec_elems, self.nfront = f_tot, v_tot, i_tot
        self.max_n = max([g.n for g in self.groups] + [0])
        self.perm_base = []
        acc = 0
        for g in self.groups:
            self.perm_base.append(acc)
            acc += len(g.nodes) * g.n
        self.perm_elems = acc
        slot_map = self.layout.slot_map
        bf = self.layout.box_faces
        nb = 6 * mm
        # factor phase: per group and half, extend-add tasks from T_vals (box halves) and
        # from the fronts buffer (internal halves)
        self.f_tasks = []
        self.up_tasks = []
        self.down_tasks = []
        for g in self.groups:
            per_side = []
            up_side = []
            for side in (0, 1):
                t_leaf, t_int, u_leaf, u_int = [], [], [], []
                for nd in g.nodes:
                    kid = nd.kids[side]
                    base = g.f_base + nd.slot * g.n * g.n
                    vbase = g.v_base + nd.slot * g.n
                    if kid.box >= 0:
                        t = kid.box
                        faces = [(a, int(bf[t, a])) for a in range(6) if bf[t, a] >= 0]
                        for a, fa in faces:
                            ra = nd.pos(fa, mm)
                            u_leaf.append((vbase + ra, t * nb + a * mm))
                            for b, fb in faces:
                                s = int(slot_map[t, 6 * a + b])
                                t_leaf.append((base + ra * g.n + nd.pos(fb, mm), s * mm * mm, g.n, mm))
                    else:
                        kg = kid.group
                        kb = kg.f_base + kid.slot * kg.n * kg.n
                        kv = kg.v_base + kid.slot * kg.n
                        for i, fi in enumerate(kid.B):
                            ri = nd.pos(fi, mm)
                            ki = kid.n_piv + i * mm
                            u_int.append((vbase + ri, kv + ki))
                            for j, fj in enumerate(kid.B):
                                t_int.append((base + ri * g.n + nd.pos(fj, mm), kb + ki * kg.n + kid.n_piv + j * mm,
                                              g.n, kg.n))
                per_side.append((self._arr(t_leaf, 4), self._arr(t_int, 4)))
                up_side.append((self._arr(u_leaf, 2), self._arr(u_int, 2)))
            self.f_tasks.append(per_side)
            self.up_tasks.append(up_side)
            gather, scatter = [], []
            for nd in g.nodes:
                vbase = g.v_base + nd.slot * g.n
                for i, f in enumerate(nd.B):
                    gather.append((vbase + nd.n_piv + i * mm, f * mm))
                for i, f in enumerate(nd.P):
                    scatter.append((f * mm, vbase + i * mm))
            self.down_tasks.append((self._arr(gather, 2), self._arr(scatter, 2)))

    @staticmethod
    def _arr(rows, width) -> np.ndarray:
        return np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1, width))

    def front_bytes(self) -> int:
        """Bytes of the fronts (FP64), the dominant storage of the factorization."""
        return 8 * self.front_elems


class NestedDissection:
    """GPU factorization of T_FF (FP64) reusable for many right-hand sides."""

    def __init__(self, layout: InterfaceLayout, device="cuda"):
        self.lib = _lib.load()
        self.layout = layout
        self.device = torch.device(device)
        self.d = DissectionLayout(layout)
        self.mm = self.d.mm
        self.groups = self.d.groups
        self.nfront = self.d.nfront
        self.plans = [_FrontPlan(self.lib, g.n, g.n_piv) for g in self.groups]
        self.dinv_base = []
        acc = 0
        for g, pl in zip(self.groups, self.plans):
            self.dinv_base.append(acc)
            acc += len(g.nodes) * pl.dinv_elems
        self.dinv_elems = acc
        dev = self.device
        cv = lambda a: torch.tensor(a, device=dev).contiguous()  # noqa: E731
        self.f_tasks = [[(cv(a), cv(b)) for a, b in sides] for sides in self.d.f_tasks]
        self.up_tasks = [[(cv(a), cv(b)) for a, b in sides] for sides in self.d.up_tasks]
        self.down_tasks = [(cv(a), cv(b)) for a, b in self.d.down_tasks]
        self.factored = False
        # face values per box: internal faces from u_F, boundary faces from the Dirichlet data
        bf = layout.box_faces
        nb, mm = 6 * self.mm, self.mm
        rows = [(t * nb + a * mm, int(bf[t, a]) * mm) for t in range(bf.shape[0]) for a in range(6) if bf[t, a] >= 0]
        self.face_tasks = cv(DissectionLayout._arr(rows, 2))
        self.all_faces = cv(DissectionLayout._arr([(f * mm, f * mm) for f in range(layout.nface)], 2))

    def memory_bytes(self) -> int:
        return (8 * (self.d.front_elems + self.dinv_elems + self.d.vec_elems) +
                4 * (self.d.perm_elems + self.d.nfront))

    @staticmethod
    def estimate_bytes(layout: InterfaceLayout) -> int:
        """Device bytes of the factorization of a layout (fronts, inverses, vectors, indices)."""
        d = DissectionLayout(layout)
        return int(8 * (d.front_elems * 1.05 + d.vec_elems) + 4 * d.perm_elems)

    @staticmethod
    def supported(layout: InterfaceLayout) -> bool:
        """Whether every front fits the kernels (at most 12288 rows)."""
        return DissectionLayout(layout).max_n <= 12288

    def face_values(self, u: torch.Tensor, g_dir: torch.Tensor) -> torch.Tensor:
        """u_b [nbox, n_b]: the interface solution on internal faces, g_dir elsewhere."""
        nbox = self.layout.box_faces.shape[0]
        _ptr(g_dir, torch.float64, nbox * 6 * self.mm, "g_dir")
        ub = g_dir.clone()
        if self.face_tasks.shape[0]:
            check(self.lib.hps_front_segments(self.face_tasks.shape[0], self.face_tasks.data_ptr(), self.mm,
                                              ub.data_ptr(), _ptr(u, torch.float64, 1, "u"), 0, _stream()),
                  "hps_front_segments")
        return ub

    def axpy(self, u: torch.Tensor, du: torch.Tensor, sign: int) -> None:
        """u += sign * du over the interface unknowns (sign +1 or -1)."""
        if self.all_faces.shape[0]:
            check(self.lib.hps_front_segments(self.all_faces.shape[0], self.all_faces.data_ptr(), self.mm,
                                              _ptr(u, torch.float64, 1, "u"), _ptr(du, torch.float64, 1, "du"),
                                              int(sign), _stream()), "hps_front_segments")


    # ---- factorization -----------------------------------------------------------------
    def factor(self, T_vals: torch.Tensor) -> None:
        """Factor T from the per-box DtN blocks in T_vals (layout slots; the per-box diagonal
        slots must hold each box's own contribution, as hps_leaf_dtn writes them)."""
        lib, st, mm = self.lib, _stream(), self.mm
        dev = self.device
        d = self.d
        self.F = torch.empty(max(d.front_elems, 1), dtype=torch.float64, device=dev)
        self.perm = torch.empty(max(d.perm_elems, 1), dtype=torch.int32, device=dev)
        self.dinv = torch.empty(max(self.dinv_elems, 1), dtype=torch.float64, device=dev)
        self.info = torch.empty(max(d.nfront, 1), dtype=torch.int32, device=dev)
        self.vec = torch.empty(max(d.vec_elems, 1), dtype=torch.float64, device=dev)
        Fp = self.F.data_ptr()
        Tp = _ptr(T_vals, torch.float64, 1, "T_vals")
        for gi, g in enumerate(self.groups):
            nf = len(g.nodes)
            fb = Fp + 8 * g.f_base
            check(lib.hps_front_init(nf, g.n, g.nP * mm, g.n_piv, g.n_piv + g.nB * mm, g.n, fb, st),
                  "hps_front_init")
            for side in (0, 1):
                t_leaf, t_int = self.f_tasks[gi][side]
                if t_leaf.shape[0]:
                    check(lib.hps_front_block_add(t_leaf.shape[0], t_leaf.data_ptr(), mm, Fp, Tp, st),
                          "hps_front_block_add")
                if t_int.shape[0]:
                    check(lib.hps_front_block_add(t_int.shape[0], t_int.data_ptr(), mm, Fp, Fp, st),
                          "hps_front_block_add")
            check(lib.hps_front_factor(self.plans[gi].handle, nf, fb, self.perm.data_ptr() + 4 * d.perm_base[gi],
                                       self.dinv.data_ptr() + 8 * self.dinv_base[gi],
                                       self.info.data_ptr() + 4 * g.i_base, st), "hps_front_factor")
        bad = torch.nonzero(self.info[:self.nfront]).flatten().cpu().tolist()
        if bad:
            raise RuntimeError(f"interface fronts {bad[:8]} have a zero or non-finite pivot")
        self.factored = True

    # ---- solve -------------------------------------------------------------------------
    def solve(self, box_vectors: torch.Tensor, sign: int = 1, trans: bool = False) -> torch.Tensor:
        """u_F with T_FF u_F = sign * (sum over the two boxes of each face of box_vectors
        [nbox, n_b]) (the lifted loads, or any per-box face vectors; sign +1 or -1), or with
        T_FF^T when trans (the adjoint's solve).  Returns u_F [nface * m^2] (device)."""
        if sign not in (1, -1):
            raise ValueError("sign must be +1 or -1")
        if not self.factored:
            raise RuntimeError("factor() first")
        lib, st, mm = self.lib, _stream(), self.mm
        nbox = self.layout.box_faces.shape[0]
        _ptr(box_vectors, torch.float64, nbox * 6 * mm, "box_vectors")
        u = torch.zeros(max(self.layout.nface * mm, 1), dtype=torch.float64, device=self.device)
        if self.nfront == 0:
            return u[:self.layout.nface * mm]
        self.vec.zero_()
        Vp, Fp, Bp, Up = self.vec.data_ptr(), self.F.data_ptr(), box_vectors.data_ptr(), u.data_ptr()
        for gi, g in enumerate(self.groups):  # upward
            for side in (0, 1):
                u_leaf, u_int = self.up_tasks[gi][side]
                if u_leaf.shape[0]:
                    check(lib.hps_front_segments(u_leaf.shape[0], u_leaf.data_ptr(), mm, Vp, Bp, sign, st),
                          "hps_front_segments")
                if u_int.shape[0]:
                    check(lib.hps_front_segments(u_int.shape[0], u_int.data_ptr(), mm, Vp, Vp, 1, st),
                          "hps_front_segments")
            self._front_solve(gi, g, 2 if trans else 0)
        for gi in range(len(self.groups) - 1, -1, -1):  # downward
            g = self.groups[gi]
            gather, scatter = self.down_tasks[gi]
            if gather.shape[0]:
                check(lib.hps_front_segments(gather.shape[0], gather.data_ptr(), mm, Vp, Up, 0, st),
                      "hps_front_segments")
            self._front_solve(gi, g, 3 if trans else 1)
            check(lib.hps_front_segments(scatter.shape[0], scatter.data_ptr(), mm, Up, Vp, 0, st),
                  "hps_front_segments")
        return u[:self.layout.nface * mm]

    def _front_solve(self, gi, g, mode):
        check(self.lib.hps_front_solve(self.plans[gi].handle, len(g.nodes), self.F.data_ptr() + 8 * g.f_base,
                                       self.perm.data_ptr() + 4 * self.d.perm_base[gi],
                                       self.dinv.data_ptr() + 8 * self.dinv_base[gi],
                                       self.vec.data_ptr() + 8 * g.v_base, mode, _stream()), "hps_front_solve")
