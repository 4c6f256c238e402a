"""CPU tests: the C ABI library loads and exports every declared symbol, and the
host-side interface bookkeeping (BSR layout, slot maps, load summation) is
consistent with the oracle's face numbering.  No GPU computation here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import interface as oi
from paper_2503_04033_amd import _lib
from paper_2503_04033_amd import interface as itf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "hps_leaf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hps_status|const char\*|size_t)\s+(hps_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert set(_declared_symbols()) == set(_lib.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhps_leaf.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def test_status_strings():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhps_leaf.so not built")
    lib = _lib.load()
    assert lib.hps_status_string(0) == b"ok"
    assert b"invalid" in lib.hps_status_string(-1)


def test_plan_rejects_bad_sizes():
    # argument validation happens before any device call
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhps_leaf.so not built")
    lib = _lib.load()
    d = _lib.LeafDesc()
    d.p, d.kappa, d.precision, d.ir_max_iter, d.ir_tol = 3, 1.0, 0, 1, 1e-12
    for a in range(3):
        d.h[a] = 0.5
    h = ctypes.c_void_p()
    assert lib.hps_plan_create(ctypes.byref(h), ctypes.byref(d)) == _lib.HPS_EUNSUPPORTED
    d.p = 8
    d.h[1] = -1.0
    assert lib.hps_plan_create(ctypes.byref(h), ctypes.byref(d)) == _lib.HPS_EINVAL
    d.h[1] = 0.5
    d.precision = 7
    assert lib.hps_plan_create(ctypes.byref(h), ctypes.byref(d)) == _lib.HPS_EINVAL
    assert lib.hps_interface_reduce(-1, None, 10, None, None) == _lib.HPS_EINVAL
    assert lib.hps_leaf_reconstruct(None, 1, None, None, None, None) == _lib.HPS_EINVAL


@pytest.mark.parametrize("nboxes", [(2, 2, 2), (3, 2, 4), (1, 1, 1), (4, 1, 1)])
def test_face_numbering_matches_oracle(nboxes):
    lay = itf.build_layout(nboxes, 3)
    bf, fb = oi.face_numbering(nboxes)
    np.testing.assert_array_equal(lay.box_faces, bf)
    assert lay.nface == fb.shape[0]


@pytest.mark.parametrize("nboxes", [(2, 2, 2), (3, 3, 3), (5, 5, 5), (3, 2, 4)])
def test_bsr_layout(nboxes):
    m = 2
    lay = itf.build_layout(nboxes, m)
    nbox = int(np.prod(nboxes))
    # every block row has at most 11 blocks (paper Sec. 3.3, Fig. sparsity5)
    per_row = np.diff(lay.indptr)
    assert per_row.max() <= 11 and per_row.min() >= 1
    if nboxes == (5, 5, 5):
        assert per_row.max() == 11
    # slots: each unique off-diagonal block and each extra diagonal slot written by exactly
    # one box; the BSR diagonal slots only by the reduction (dst = lower + upper)
    used = lay.slot_map[lay.slot_map >= 0]
    counts = np.bincount(used, minlength=lay.nslot_total)
    dst, lo, hi = lay.reduce_triples.T
    assert np.all(counts[dst] == 0) and np.all(counts[lo] == 1) and np.all(counts[hi] == 1)
    assert counts.sum() == counts.size - lay.nface
    assert lay.nslot_total == lay.nslot + 2 * lay.nface
    # the lower box of face F writes lo, the upper box hi
    for F in range(lay.nface):
        t_lo = np.nonzero(lay.box_faces[:, 1::2] == F)[0][0]
        a = 2 * int(np.nonzero(lay.box_faces[t_lo, 1::2] == F)[0][0]) + 1
        assert lay.slot_map[t_lo, 6 * a + a] == lo[F]
    # slot map is -1 exactly where a row or column face is on the boundary
    ok = (lay.box_faces[:, :, None] >= 0) & (lay.box_faces[:, None, :] >= 0)
    np.testing.assert_array_equal(lay.slot_map.reshape(nbox, 6, 6) >= 0, ok)
    # BSR indices within each row are sorted and unique
    for r in range(lay.nface):
        cols = lay.indices[lay.indptr[r]:lay.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
        assert r in cols


def test_bsr_assembly_equals_coo_sum():
    # fill each box's 36 blocks with random values, reduce duplicates like the GPU, compare with COO sum
    nboxes, m = (3, 2, 2), 2
    mm = m * m
    lay = itf.build_layout(nboxes, m)
    nbox = int(np.prod(nboxes))
    rng = np.random.default_rng(0)
    Tbox = rng.normal(size=(nbox, 6, 6, mm, mm))
    vals = np.zeros((lay.nslot_total, mm, mm))
    for t in range(nbox):
        for a in range(6):
            for b in range(6):
                s = lay.slot_map[t, 6 * a + b]
                if s >= 0:
                    vals[s] = Tbox[t, a, b]
    for dst, lo, hi in lay.reduce_triples:
        vals[dst] = vals[lo] + vals[hi]
    A = itf.bsr_matrix(lay, vals.ravel()).toarray()
    ref = np.zeros((lay.nface * mm, lay.nface * mm))
    for t in range(nbox):
        for a in range(6):
            for b in range(6):
                Fa, Fb = lay.box_faces[t, a], lay.box_faces[t, b]
                if Fa >= 0 and Fb >= 0:
                    ref[Fa * mm:(Fa + 1) * mm, Fb * mm:(Fb + 1) * mm] += Tbox[t, a, b]
    np.testing.assert_allclose(A, ref, atol=1e-14)


def test_interface_rhs_and_face_values():
    nboxes, m = (2, 2, 1), 3
    mm = m * m
    lay = itf.build_layout(nboxes, m)
    nbox = 4
    g = np.arange(nbox * 6 * mm, dtype=float).reshape(nbox, 6 * mm)
    rhs = itf.interface_rhs(lay, g)
    for F in range(lay.nface):
        tot = np.zeros(mm)
        for t in range(nbox):
            for a in range(6):
                if lay.box_faces[t, a] == F:
                    tot += g[t, a * mm:(a + 1) * mm]
        np.testing.assert_allclose(rhs[F * mm:(F + 1) * mm], tot)
    uf = np.arange(lay.nface * mm, dtype=float) + 1000
    gd = -np.ones((nbox, 6 * mm))
    ub = itf.box_face_values(lay, uf, gd)
    mask = itf.boundary_mask(lay)
    assert np.all(ub[mask] == -1)
    assert np.all(ub[~mask] >= 1000)


def test_interface_solver_dense_and_sparse_agree():
    # the host interface LU: dense LAPACK and SuperLU give the same solution and transposed
    # solution of the same block-sparse system
    from paper_2503_04033_amd import interface as itf
    layout = itf.build_layout((3, 2, 2), 4)
    mm = 16
    rng = np.random.default_rng(3)
    T = rng.standard_normal(layout.nslot_total * mm * mm + 1) * 0.1
    T_primary = T[:layout.nslot * mm * mm].reshape(layout.nslot, mm, mm)
    for r in range(len(layout.indptr) - 1):
        for s in range(layout.indptr[r], layout.indptr[r + 1]):
            if layout.indices[s] == r:
                T_primary[s] += 4.0 * np.eye(mm)
    rhs = rng.standard_normal((len(layout.indptr) - 1) * mm)
    dense = itf.InterfaceSolver(layout, T, method="dense")
    sparse = itf.InterfaceSolver(layout, T, method="sparse")
    assert dense.method == "dense" and sparse.method == "sparse"
    A = itf.bsr_matrix(layout, T).toarray()
    for trans, M in (("N", A), ("T", A.T)):
        xd, xs = dense.solve(rhs, trans=trans), sparse.solve(rhs, trans=trans)
        assert np.allclose(M @ xd, rhs, atol=1e-10)
        assert np.allclose(xd, xs, atol=1e-10)


def test_pivot_rule_reference():
    # the host elimination that the GPU pivot-rule test compares against: on a matrix without
    # ties it chooses LAPACK's partial-pivoting rows, and its factors reproduce the matrix
    import scipy.linalg as sl
    from tests.test_gpu_parity import _lu_rule, _tie_matrix
    n = 40
    A = np.random.default_rng(3).standard_normal((n, n))
    order, B, ties = _lu_rule(A)
    assert ties == 0
    P, L, U = sl.lu(A)  # A = P L U: position i holds row argmax(P[:, i])
    assert np.array_equal(order, np.argmax(P, axis=0))
    assert np.allclose(np.tril(B, -1), np.tril(L, -1), atol=1e-12) and np.allclose(np.triu(B), U, atol=1e-12)
    # and the tie matrix (as at p = 8): ties at nearly every step, exact integer factors, and
    # the first maximum is taken (the lowest current position)
    A, (order, B, ties) = _tie_matrix(224, 7)
    assert ties > 0.9 * 224
    assert np.array_equal((np.tril(B, -1) + np.eye(224)) @ np.triu(B), A[order])
    first = np.abs(A[:, 0]) == np.abs(A[:, 0]).max()
    assert order[0] == np.flatnonzero(first)[0]
