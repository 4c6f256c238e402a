"""Host checks of the nested-dissection interface solver's index structure.

The dissection tree, front shapes and extend-add task lists of
paper_2503_04033_amd.nested.DissectionLayout drive the GPU kernels.  Here the four
kernel steps are emulated in NumPy on exactly those task lists (front init, block
extend-add, partial LU with pivots inside the separator, the upward and downward
vector solves) and the result must equal a dense solve of the assembled interface
matrix: a wrong offset, face order or tree traversal fails it.  The numerics of the
GPU kernels themselves are tested on the GPU.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_2503_04033_amd import interface as itf
from paper_2503_04033_amd.nested import DissectionLayout


def _random_box_blocks(layout, rng):
    """Per-box DtN-like blocks in the layout's slots (diagonally dominant), then the
    diagonal reduction (dst = lower + upper), as the GPU build leaves T_vals."""
    mm = layout.m * layout.m
    T = np.zeros((layout.nslot_total + 1) * mm * mm)
    nbox = layout.box_faces.shape[0]
    for t in range(nbox):
        for a in range(6):
            for b in range(6):
                s = layout.slot_map[t, 6 * a + b]
                if s < 0:
                    continue
                blk = rng.standard_normal((mm, mm)) * 0.1
                if a == b:
                    blk += 3.0 * np.eye(mm)
                T[s * mm * mm:(s + 1) * mm * mm] = blk.ravel()
    for dst, lo, hi in layout.reduce_triples:
        T[dst * mm * mm:(dst + 1) * mm * mm] = (T[lo * mm * mm:(lo + 1) * mm * mm] +
                                                T[hi * mm * mm:(hi + 1) * mm * mm])
    return T


def _emulate(d: DissectionLayout, T_vals, box_vectors):
    mm = d.mm
    F = np.zeros(max(d.front_elems, 1))
    fac = {}
    for gi, g in enumerate(d.groups):
        for k in range(len(g.nodes)):  # front init
            base = g.f_base + k * g.n * g.n
            A = np.zeros((g.n, g.n))
            for i in list(range(g.nP * mm, g.n_piv)) + list(range(g.n_piv + g.nB * mm, g.n)):
                A[i, i] = 1.0
            F[base:base + g.n * g.n] = A.ravel()
        for side in (0, 1):
            for tasks, src in zip(d.f_tasks[gi][side], (T_vals, F)):
                dsts = set()
                for dst, s, ldd, lds in tasks:
                    assert dst not in dsts  # one writer per block and call
                    dsts.add(dst)
                    for i in range(mm):
                        F[dst + i * ldd:dst + i * ldd + mm] += src[s + i * lds:s + i * lds + mm]
        for k in range(len(g.nodes)):  # partial LU, pivots inside P
            base = g.f_base + k * g.n * g.n
            A = F[base:base + g.n * g.n].reshape(g.n, g.n)
            p = g.n_piv
            lu = scipy.linalg.lu_factor(A[:p, :p])
            L = np.tril(lu[0], -1) + np.eye(p)
            U = np.triu(lu[0])
            perm = np.arange(p)
            for i, j in enumerate(lu[1]):
                perm[[i, j]] = perm[[j, i]]
            U12 = scipy.linalg.solve_triangular(L, A[perm, p:], lower=True, unit_diagonal=True)
            L21 = scipy.linalg.solve_triangular(U.T, A[p:, :p].T, lower=True).T
            A[p:, p:] -= L21 @ U12
            fac[(gi, k)] = (L, U, perm, L21, U12)
    V = np.zeros(max(d.vec_elems, 1))
    for gi, g in enumerate(d.groups):  # upward
        for side in (0, 1):
            for tasks, src in zip(d.up_tasks[gi][side], (box_vectors.ravel(), V)):
                for dst, s in tasks:
                    V[dst:dst + mm] += src[s:s + mm]
        for k in range(len(g.nodes)):
            L, U, perm, L21, U12 = fac[(gi, k)]
            v = V[g.v_base + k * g.n:g.v_base + (k + 1) * g.n]
            p = g.n_piv
            y = scipy.linalg.solve_triangular(L, v[:p][perm], lower=True, unit_diagonal=True)
            v[p:] -= L21 @ y
            v[:p] = y
    u = np.zeros(d.layout.nface * mm)
    for gi in range(len(d.groups) - 1, -1, -1):  # downward
        g = d.groups[gi]
        gather, scatter = d.down_tasks[gi]
        for dst, s in gather:
            V[dst:dst + mm] = u[s:s + mm]
        for k in range(len(g.nodes)):
            L, U, perm, L21, U12 = fac[(gi, k)]
            v = V[g.v_base + k * g.n:g.v_base + (k + 1) * g.n]
            p = g.n_piv
            v[:p] = scipy.linalg.solve_triangular(U, v[:p] - U12 @ v[p:], lower=False)
        for dst, s in scatter:
            u[dst:dst + mm] = V[s:s + mm]
    return u


@pytest.mark.parametrize("nboxes,m", [((2, 1, 1), 3), ((2, 2, 2), 3), ((3, 2, 2), 2), ((4, 4, 4), 2),
                                      ((5, 3, 2), 2), ((1, 1, 3), 3)])
def test_emulated_dissection_equals_dense_solve(nboxes, m):
    layout = itf.build_layout(nboxes, m)
    rng = np.random.default_rng(sum(nboxes) * 10 + m)
    T_vals = _random_box_blocks(layout, rng)
    nbox = layout.box_faces.shape[0]
    mm = m * m
    g = rng.standard_normal((nbox, 6 * mm)) * np.repeat(layout.box_faces >= 0, mm, axis=1)
    d = DissectionLayout(layout)
    u = _emulate(d, T_vals, g)
    T = itf.bsr_matrix(layout, T_vals).toarray()
    ref = np.linalg.solve(T, itf.interface_rhs(layout, g))
    assert np.abs(u - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


def test_tree_shapes_and_separators():
    # every internal face is eliminated exactly once, at the node whose halves it separates
    layout = itf.build_layout((4, 4, 4), 3)
    d = DissectionLayout(layout)
    seen = []
    for g in d.groups:
        for nd in g.nodes:
            seen += nd.P
            assert set(nd.P).isdisjoint(nd.B)
    assert sorted(seen) == list(range(layout.nface))
    assert d.root.B == [] and d.groups[-1].nodes[0] is d.root
    # power-of-two grid: one front shape per height and boundary-face count
    heights = sorted({g.height for g in d.groups})
    assert heights == list(range(1, 7))
