"""GPU nested-dissection factorization of the interface system (fronts.hip via the C ABI).

* random per-box blocks at real face sizes (m = 14, the p = 16 faces): the GPU solution
  against a dense solve of the assembled matrix;
* the DtN maps the GPU build writes for the 4^3-box, p = 16, kappa = 40 problem: u_F
  against the host LAPACK factorization of the same matrix, and the backward error of
  the system, at 1e-12.
"""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2503_04033_amd import interface as itf
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _random_T(layout, rng):
    mm = layout.m * layout.m
    T = np.zeros((layout.nslot_total + 1) * mm * mm)
    for t in range(layout.box_faces.shape[0]):
        for a in range(6):
            for b in range(6):
                s = layout.slot_map[t, 6 * a + b]
                if s < 0:
                    continue
                blk = rng.standard_normal((mm, mm)) * (0.5 / mm)
                if a == b:
                    blk += 3.0 * np.eye(mm)
                T[s * mm * mm:(s + 1) * mm * mm] = blk.ravel()
    for dst, lo, hi in layout.reduce_triples:
        T[dst * mm * mm:(dst + 1) * mm * mm] = T[lo * mm * mm:(lo + 1) * mm * mm] + T[hi * mm * mm:(hi + 1) * mm * mm]
    return T


@pytest.mark.parametrize("nboxes,m", [((2, 2, 2), 14), ((3, 2, 2), 14), ((4, 4, 2), 6)])
def test_nested_random_blocks(gpu, nboxes, m):
    from paper_2503_04033_amd.nested import NestedDissection
    layout = itf.build_layout(nboxes, m)
    rng = np.random.default_rng(sum(nboxes) + m)
    T_vals = _random_T(layout, rng)
    nbox = layout.box_faces.shape[0]
    mm = m * m
    g = rng.standard_normal((nbox, 6 * mm)) * np.repeat(layout.box_faces >= 0, mm, axis=1)
    say(f"nested random {nboxes} m={m}: {layout.nunknown} unknowns")
    nd = NestedDissection(layout)
    say(f"  {len(nd.groups)} front groups, max front {nd.d.max_n}, {nd.memory_bytes() / 1e6:.1f} MB")
    nd.factor(torch.tensor(T_vals, device="cuda"))
    gd = torch.tensor(g, device="cuda")
    u = nd.solve(gd).cpu().numpy()
    lam = nd.solve(gd, trans=True).cpu().numpy()
    T = itf.bsr_matrix(layout, T_vals).toarray()
    rhs = itf.interface_rhs(layout, g)
    ref = np.linalg.solve(T, rhs)
    ref_t = np.linalg.solve(T.T, rhs)
    err = np.abs(u - ref).max() / np.abs(ref).max()
    err_t = np.abs(lam - ref_t).max() / np.abs(ref_t).max()
    say(f"  max rel err {err:.2e}, transposed {err_t:.2e}")
    assert err < 1e-12 and err_t < 1e-12


def test_nested_dtn_4cubed_p16(gpu):
    from paper_2503_04033_amd.nested import NestedDissection
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.multi_bump((4, 4, 4), 16, 40.0, 3, name="cfg3_4x4x4_p16")
    s = TwoLevelSolver.for_problem(prob, precision="fp64")
    bv, fv, gv, _, _ = s.sample(prob.b, prob.f, prob.g)
    br = s.build(bv, fv, gv)
    torch.cuda.synchronize()
    nd = NestedDissection(s.layout)
    say(f"{prob.name}: {s.layout.nunknown} interface unknowns, {len(nd.groups)} front groups, "
        f"max front {nd.d.max_n}, {nd.memory_bytes() / 1e9:.2f} GB")
    nd.factor(br.T_vals)
    u = nd.solve(br.g_loads).cpu().numpy()
    T_host = br.T_vals.cpu().numpy()
    rhs = itf.interface_rhs(s.layout, br.g_loads.cpu().numpy())
    ref = itf.InterfaceSolver(s.layout, T_host, method="dense").solve(rhs)
    A = itf.bsr_matrix(s.layout, T_host)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    berr = np.linalg.norm(A @ u - rhs) / (abs(A).sum(axis=1).max() * np.linalg.norm(u) + np.linalg.norm(rhs))
    say(f"  u_F vs host LAPACK {err:.2e}, backward error {berr:.2e}")
    assert err < 1e-9 and berr < 1e-14


def _face_rhs_as_box_vectors(layout, r):
    """Per-box face vectors whose sum over the two boxes of each face is r (all of it on
    the lower box of the face, its + side)."""
    mm = layout.m * layout.m
    nbox = layout.box_faces.shape[0]
    v = np.zeros((nbox, 6, mm))
    for a in (1, 3, 5):
        F = layout.box_faces[:, a]
        ok = F >= 0
        v[ok, a, :] = r.reshape(-1, mm)[F[ok]]
    return v.reshape(nbox, 6 * mm)


def test_pipeline_config2_gpu_interface(gpu):
    # 8^3 boxes, p = 12, kappa = 20: 134,400 interface unknowns.  The host cannot factor this
    # interface matrix (SciPy's SuperLU stops with "not enough memory" for both column
    # orderings; dense LAPACK needs 144 GB), so the oracle has no full solution here.  What
    # holds at any size: the GPU u_F solves the assembled system to a backward error near
    # FP64 rounding, and every sampled box's interior equals the oracle's interior solve
    # (its own blocks, FP64) with the box's face values from the GPU solution.
    from oracle import leaf as ol
    from paper_2503_04033_amd.nested import NestedDissection
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.config2()
    s = TwoLevelSolver.for_problem(prob, precision="fp64", interface="gpu")
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    nd = out["isolver"]
    assert isinstance(nd, NestedDissection)
    br = out["build"]
    say(f"{prob.name}: {s.layout.nunknown} interface unknowns, {len(nd.groups)} front groups, "
        f"max front {nd.d.max_n}, {nd.memory_bytes() / 1e9:.1f} GB")
    T_host = br.T_vals.cpu().numpy()
    A = itf.bsr_matrix(s.layout, T_host)
    rhs = itf.interface_rhs(s.layout, br.g_loads.cpu().numpy())
    u = out["u_face"]
    anorm = abs(A).sum(axis=1).max()
    berr = np.linalg.norm(A @ u - rhs) / (anorm * np.linalg.norm(u) + np.linalg.norm(rhs))
    # lower bound of cond_1(T_FF): a few inverse-power steps x <- T^{-1} x / |.|
    rng = np.random.default_rng(21)
    x = rng.standard_normal(s.layout.nunknown)
    inv_norm = 0.0
    for _ in range(4):
        x /= np.abs(x).sum()
        y = nd.solve(torch.tensor(_face_rhs_as_box_vectors(s.layout, x), device="cuda")).cpu().numpy()
        inv_norm = max(inv_norm, np.abs(y).sum())
        x = y
    say(f"  interface backward error {berr:.2e}; cond_1(T_FF) >= {anorm * inv_norm:.2e} "
        f"(|T|_1 {anorm:.2e}, |T^-1|_1 >= {inv_norm:.2e})")
    assert berr < 1e-14
    ui = out["u_i"].cpu().numpy()
    org = prob.box_origins()
    worst = 0.0
    for t in (0, 7, 63, 100, 255, 300, 448, 511):
        xi, _ = ol.box_node_coords(org[t], prob.h, prob.p)
        blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(xi))
        ref = ol.interior_solve(blk, prob.f(xi), out["u_b"][t])
        e = np.linalg.norm(ui[t] - ref) / np.linalg.norm(ref)
        worst = max(worst, e)
    say(f"  sampled interiors vs the oracle's interior solve: {worst:.2e}")
    assert worst < 1e-10
