"""GPU parity: the HIP leaf path (through the C ABI) against the FP64 oracle.

Tolerances.  FP64 path: the kernels and the oracle evaluate the same exact
algebra in different orders; with kappa(A_ii) <= ~1e4 the forward error is
bounded by kappa * O(n u64) ~ 1e-11, so 1e-10 relative (Frobenius, per box)
is used for X and T.  FP32 + FP64 refinement: the metric's bar, 1e-9 relative.
Solutions: relative l2 over all nodes, same bars.  Boxes of the headline grids
(h = 1/16 at p = 16, h = 1/8 at p = 12) also meet a regression guard of 1e-11, the
level this path measures there (1e-13 to 1e-12); large boxes (h = 1/2 to 1) are worse
conditioned and land at up to ~5e-11 in FP32 + refinement.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import interface as oi
from tests.gpu_helpers import gpu_leaf_boxes, oracle_leaf_boxes, rel, rel_fro_max, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
IR_TOL = 1e-9
GUARD = 1e-11


def _check_leaf(prob, box_ids, precision, tol, f_on=True, tuning=None, guard=None):
    say(f"case {prob.name} p={prob.p} boxes={list(box_ids)} {precision} tuning={tuning}")
    gout = gpu_leaf_boxes(prob, box_ids, precision, f_on=f_on, tuning=tuning)
    ored = oracle_leaf_boxes(prob, box_ids, f_on=f_on)
    assert np.all(gout["info"] == 0)
    Xo = [np.concatenate([-r.S, r.v[:, None]], axis=1) for _, r in ored]
    To = [r.T for _, r in ored]
    go = [r.g for _, r in ored]
    eX = rel_fro_max(gout["X"], Xo)
    eT = rel_fro_max(gout["T"], To)
    eg = rel_fro_max(gout["g"], go) if f_on else 0.0
    say(f"  errors X {eX:.2e} T {eT:.2e} g {eg:.2e} iters {gout['iters'].tolist()[:8]} "
        f"berr max {gout['berr'].max():.2e}")
    assert eX < tol and eT < tol and eg < tol
    if guard is not None:  # regression guard at the level measured for this case
        assert max(eX, eT, eg) < guard, f"X {eX:.2e} T {eT:.2e} g {eg:.2e} above {guard}"
    return gout


@pytest.mark.parametrize("p", [4, 5, 6, 7, 8, 9])
def test_leaf_fp64_small(gpu, p):
    prob = W.multi_bump((2, 2, 2), p, 6.0, 11, gaussian_source=True, name=f"bump_p{p}")
    _check_leaf(prob, range(8), "fp64", FP64_TOL)


@pytest.mark.parametrize("p", [4, 5, 6, 8, 9])
def test_leaf_fp32_ir_small(gpu, p):
    prob = W.multi_bump((2, 2, 2), p, 6.0, 12, gaussian_source=True, name=f"bump_p{p}")
    out = _check_leaf(prob, range(8), "fp32_ir", IR_TOL)
    assert np.all(out["iters"] >= 0)


@pytest.mark.parametrize("precision,case", [("fp64", "p9"), ("fp32_ir", "p9"), ("fp32_ir", "p14"),
                                            ("fp32_ir", "p20")])
def test_trsm_schedules(gpu, precision, case):
    # every schedule and occupancy of the interior solves and every column blocking of the
    # refinement residual: parity with the oracle, and bitwise the same results (same
    # tiles, same order of every sum); p = 14 (1728 rows, 64 mod 128) takes the forward
    # sweep whose 64-row block comes first; p = 20 takes the segmented FP32 sums
    if case == "p9":
        prob, boxes = W.multi_bump((2, 2, 2), 9, 6.0, 14, gaussian_source=True, name="sched_p9"), range(8)
    elif case == "p14":
        prob, boxes = W.multi_bump((2, 2, 2), 14, 6.0, 16, gaussian_source=True, name="sched_p14"), [0, 7]
    else:
        prob, boxes = W.config3_p20(), [5]
    tol = FP64_TOL if precision == "fp64" else IR_TOL
    sweep = _check_leaf(prob, boxes, precision, tol, tuning={"trsm_schedule": 1})
    for waves, cols in ((4, 8), (6, 4), (8, 2)):
        rows = gpu_leaf_boxes(prob, boxes, precision,
                              tuning={"trsm_schedule": 0, "trsm_waves": waves, "residual_cols": cols})
        for k in ("X", "T", "g", "iters"):
            assert np.array_equal(sweep[k], rows[k]), (waves, cols, k)
    plan = rows["plan"]
    from paper_2503_04033_amd._lib import HpsError
    with pytest.raises(HpsError):
        plan.hps_plan_set_tuning("trsm_schedule", 2)
    with pytest.raises(HpsError):
        plan.hps_plan_set_tuning("trsm_waves", 5)
    assert plan.hps_plan_get_tuning("trsm_schedule") == 0 and plan.hps_plan_get_tuning("trsm_waves") == 8
    with pytest.raises(HpsError):
        plan.hps_plan_set_tuning("residual_cols", 16)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_first_nonzero_rows_of_rhs(gpu, precision):
    # The forward sweep of the first solve skips, per 64-column tile of B = [A_ib | f],
    # the leading rows of P B that are zero.  The tile starts the library computed
    # (white box: they sit in the workspace after the per-box scalars) must equal the
    # structure of the oracle's A_ib under the factor's row permutation (the f column
    # counts as dense), rounded down to 64.  Tiles hold the columns in the solves'
    # internal order: FP64 natural; FP32 + refinement 16-column groups stably sorted by
    # the first row their (unpermuted) A_ib columns touch, the f column's group first.
    prob = W.multi_bump((1, 1, 2), 12, 8.0, 13, gaussian_source=True, name="skip_p12")
    out = _check_leaf(prob, [0, 1], precision, FP64_TOL if precision == "fp64" else IR_TOL)
    i = out["plan"].info
    nb, ntn = 2, i.ldx // 64
    off = 8 * i.n_pad * i.ldx * nb + 64 * nb
    ks = out["ws"].view(torch.uint8)[off:off + 4 * ntn * nb].view(torch.int32).view(nb, ntn).cpu().numpy()
    for k, (blk, _) in enumerate(oracle_leaf_boxes(prob, [0, 1])):
        B = np.zeros((i.n_pad, i.ldx))
        B[:i.n_i, :i.n_b] = blk.A_ib
        PB = B[out["perm"][k]] != 0
        first = np.where(PB.any(axis=0), PB.argmax(axis=0), i.n_pad)
        first[i.n_b] = 0
        order = np.arange(i.ldx // 16)
        if precision == "fp32_ir":
            nz = blk.A_ib != 0
            f0 = np.full(i.ldx, i.n_pad)
            f0[:i.n_b] = nz.argmax(axis=0)
            f0[i.n_b] = 0
            order = np.argsort(f0.reshape(-1, 16).min(axis=1), kind="stable")
        first = first.reshape(-1, 16)[order].reshape(-1)
        want = first.reshape(ntn, 64).min(axis=1) // 64 * 64
        say(f"  box {k}: tile starts {ks[k].tolist()}")
        assert np.array_equal(ks[k], want)
        assert ks[k].max() > 0  # at p = 12 some tiles start below the top


def test_factorization_property(gpu):
    # P A = L U for the stored factors (any valid pivot sequence), FP64, ragged last panel
    prob = W.multi_bump((1, 1, 2), 9, 8.0, 13, name="lu_p9")
    out = gpu_leaf_boxes(prob, [0, 1], "fp64")
    n = out["plan"].info.n_pad
    for k in range(2):
        A, LU, perm = out["A0"][k], out["LU"][k], out["perm"][k]
        assert sorted(perm.tolist()) == list(range(n))
        PLU = LU[perm]
        L = np.tril(PLU, -1) + np.eye(n)
        U = np.triu(PLU)
        err = np.abs(L @ U - A[perm]).max() / np.abs(A).max()
        say(f"  |PA-LU|/|A| = {err:.2e}, max|L| = {np.abs(L).max():.3f}")
        assert err < 1e-13
        assert np.abs(L).max() <= 1.0 + 1e-12  # partial pivoting bound


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_ir", IR_TOL)])
def test_leaf_p12_sampled(gpu, precision, tol):
    # configuration-2 boxes (p = 12, kappa = 20, single bump); oracle on 4 boxes
    prob = W.config2()
    _check_leaf(prob, [0, 63, 300, 511], precision, tol, f_on=False, guard=GUARD)


def test_leaf_p16_sampled_fp32_ir(gpu):
    prob = W.config3()
    _check_leaf(prob, [0, 2047], "fp32_ir", IR_TOL, f_on=False, guard=GUARD)


def _pipeline(prob, precision, tol, interface="auto"):
    from paper_2503_04033_amd.solver import TwoLevelSolver
    say(f"pipeline {prob.name} p={prob.p} {precision} interface={interface}")
    s = TwoLevelSolver.for_problem(prob, precision=precision, interface=interface)
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    ref = oi.solve(prob)
    eu = rel(out["u_i"].cpu().numpy(), ref.u_i)
    ef = rel(out["u_face"], ref.u_face) if ref.u_face.size else 0.0
    say(f"  u_i err {eu:.2e}  u_face err {ef:.2e}")
    assert eu < tol and ef < tol
    return out, ref


@pytest.mark.parametrize("interface", ["gpu", "host"])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_ir", IR_TOL)])
def test_pipeline_config1(gpu, precision, tol, interface):
    prob = W.config1()
    out, ref = _pipeline(prob, precision, tol, interface)
    exact = prob.u_exact(out["xi"]).reshape(out["u_i"].shape)
    err = rel(out["u_i"].cpu().numpy(), exact)
    say(f"  vs exact {err:.2e}")
    assert err < 2e-6  # p = 6 discretisation error of the manufactured plane wave


@pytest.mark.parametrize("interface", ["gpu", "host"])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_ir", IR_TOL)])
def test_pipeline_ragged_grid(gpu, precision, tol, interface):
    prob = W.multi_bump((3, 2, 2), 8, 9.0, 21, gaussian_source=True, name="grid3x2x2_p8")
    _pipeline(prob, precision, tol, interface)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_ir", IR_TOL)])
def test_pipeline_recompute_chunked(gpu, precision, tol):
    # chunks of 5 boxes (ragged last chunk) and X recomputed in the solve stage
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.multi_bump((3, 2, 2), 7, 8.0, 23, gaussian_source=True, name="recompute_p7")
    say(f"pipeline recompute {prob.name} {precision}")
    s = TwoLevelSolver.for_problem(prob, precision=precision, chunk=5, keep=False)
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    ref = oi.solve(prob)
    eu = rel(out["u_i"].cpu().numpy(), ref.u_i)
    ef = rel(out["u_face"], ref.u_face)
    say(f"  u_i err {eu:.2e}  u_face err {ef:.2e}")
    assert eu < tol and ef < tol


@pytest.mark.parametrize("p", [17, 18, 19])
def test_leaf_large_p_fp32_ir(gpu, p):
    # p = 17, 18: the largest MFMA residuals (m = 15, 16); p = 19: the first size with
    # segmented FP32 sums in the solves and the fallback residual
    # boxes of a 4^3 grid (h = 1/4) at kappa = 40, as in configuration 3's p = 20 case
    prob = W.multi_bump((4, 4, 4), p, 40.0, 17, gaussian_source=True, name=f"large_p{p}")
    _check_leaf(prob, [21], "fp32_ir", IR_TOL)


def test_leaf_p20_sampled_fp32_ir(gpu):
    # the 4^3, p = 20 case of configuration 3 (5832 interior nodes, ragged last panel)
    prob = W.config3_p20()
    _check_leaf(prob, [21], "fp32_ir", IR_TOL, f_on=False)


def test_pipeline_single_box(gpu):
    prob = W.multi_bump((1, 1, 1), 7, 5.0, 22, gaussian_source=True, name="one_box")
    _pipeline(prob, "fp64", FP64_TOL)


@pytest.mark.parametrize("keep", [True, False])
def test_fp64_fallback_for_unconverged_boxes(gpu, keep):
    # no correction step and an unreachable tolerance: every box ends above ir_tol, is
    # flagged (ir_iters = -1) and is factored and solved again in FP64
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.multi_bump((2, 2, 2), 8, 6.0, 31, gaussian_source=True, name="fallback_p8")
    say(f"fallback {prob.name} keep={keep}")
    s = TwoLevelSolver.for_problem(prob, precision="fp32_ir", ir_max_iter=0, ir_tol=1e-30, chunk=3, keep=keep)
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    br = out["build"]
    assert br.extra["fp64_fallback"] == list(range(prob.nbox))
    assert br.extra["interior_fp64"] == list(range(prob.nbox))
    assert np.all(br.ir_iters.cpu().numpy() == -1)
    ref = oi.solve(prob)
    eu = rel(out["u_i"].cpu().numpy(), ref.u_i)
    ef = rel(out["u_face"], ref.u_face)
    say(f"  u_i err {eu:.2e}  u_face err {ef:.2e}")
    assert eu < FP64_TOL and ef < FP64_TOL


def _near_resonant(p=8, delta=1e-7):
    """2x2x2 boxes, b = 1 in box 0 and 1.2 elsewhere (b only enters at interior nodes, so a
    jump on box faces is fine), kappa^2 = (an eigenvalue of box 0's -Lap_ii) * (1 + delta):
    box 0's A_ii has a condition number ~1/delta, beyond FP32 refinement, while the other
    boxes are well conditioned.  The eigenvalue comes from the oracle's D2."""
    from oracle import cheb
    h = 0.5
    D = cheb.diffmat(p)
    d2 = (D @ D)[1:-1, 1:-1] * (2.0 / h) ** 2
    mu = np.sort(-np.linalg.eigvals(d2).real)
    lam = 3.0 * mu[0]  # the lowest mode, (i, j, k) = (0, 0, 0)
    kappa = float(np.sqrt(lam * (1.0 + delta)))
    base = W.multi_bump((2, 2, 2), p, kappa, 41, gaussian_source=True, name="near_resonant")

    def b(x):
        x = np.asarray(x)
        inside = (x[..., 0] < 0.5) & (x[..., 1] < 0.5) & (x[..., 2] < 0.5)
        return np.where(inside, 1.0, 1.2)

    import dataclasses
    return dataclasses.replace(base, b=b)


def test_fp64_fallback_near_singular_box(gpu):
    # A box whose FP32 refinement really diverges: the build flags it and redoes its DtN in
    # FP64 (bitwise the FP64 plan's blocks), the solve stage takes its interior from FP64
    # factors (the FP32 ones leave a backward error far above tolerance), the other boxes
    # stay on the FP32 path.  Against the oracle the tolerance is cond(A_ii) u64 ~ 1e-10
    # scaled by the interface amplification; without the FP64 interiors the error is O(1).
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = _near_resonant()
    say(f"near-singular box: kappa={prob.kappa:.10f}")
    s = TwoLevelSolver.for_problem(prob, precision="fp32_ir", chunk=8)
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    br = out["build"]
    it = br.ir_iters.cpu().numpy()
    say(f"  ir_iters {it.tolist()}  fallback {br.extra['fp64_fallback']}  interior fp64 "
        f"{br.extra['interior_fp64']}  interior berr max {br.extra['interior_berr_max']:.2e}")
    assert br.extra["fp64_fallback"] == [0] and it[0] < 0 and np.all(it[1:] >= 0)
    assert 0 in br.extra["interior_fp64"] and br.extra["interior_berr_max"] <= 1e-12
    # box 0's blocks and load equal the FP64 plan's, bitwise
    g64 = gpu_leaf_boxes(prob, [0], "fp64")
    g32 = gpu_leaf_boxes(prob, [0], "fp32_ir")
    assert g32["iters"][0] < 0
    blocks = _box_blocks(s, br, 0)
    assert len(blocks) == 9
    for (a, b), blk in blocks.items():
        assert np.array_equal(blk, g64["T6"][0, a, b]), (a, b)
    ref = oi.solve(prob)
    eu = rel(out["u_i"].cpu().numpy(), ref.u_i)
    ef = rel(out["u_face"], ref.u_face)
    say(f"  u_i err {eu:.2e}  u_face err {ef:.2e}")
    assert eu < 1e-6 and ef < 1e-6


def _box_blocks(s, br, t):
    """{(a, b): block} of the DtN blocks box t wrote into its own slots of the interface
    matrix (both faces internal; the shared diagonal blocks in the box's own extra slot)."""
    i = s.info
    mm = i.m * i.m
    T = br.T_vals[:-1].view(-1, mm, mm).cpu().numpy()
    out = {}
    for a in range(6):
        for b in range(6):
            sl = int(s.layout.slot_map[t, 6 * a + b])
            if sl >= 0:
                out[(a, b)] = T[sl]
    return out


_ORACLE = {}


def _oracle_solution(prob):
    # lean boxes and a dense interface LU: same arithmetic, within the memory and time
    # of a test; progress lines keep the run visibly alive
    def progress(msg):
        if not msg.startswith("box") or msg.split()[1].split("/")[0] in ("1", "16", "32", "48", "64"):
            say(f"  oracle: {msg}")
    if prob.name not in _ORACLE:
        _ORACLE[prob.name] = oi.solve(prob, keep_boxes=False, dense=True, progress=progress)
    return _ORACLE[prob.name]


def _backward_error(T_ff, rhs, u):
    r = T_ff @ u - rhs
    return float(np.abs(r).max() / (abs(T_ff).sum(axis=1).max() * np.abs(u).max() + np.abs(rhs).max()))


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_pipeline_4cubed_p16(gpu, precision):
    # interface and interior solution parity of the configuration-3 family at 4^3 boxes,
    # p = 16, kappa = 40 (the 16^3 interface system is beyond the host solvers).  This
    # interface system amplifies the rounding of the DtN maps ~5e5-fold (FP64 maps give
    # 2e-10 here; FP32+IR maps, ~1e-13 from FP64, gave 4e-7 before the solve stage's
    # outer refinement), so solutions are held to the metric's 1e-9 for both paths, and
    # the GPU interface solution must solve the oracle's interface system to backward
    # error 1e-11.
    tol = IR_TOL
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.multi_bump((4, 4, 4), 16, 40.0, 3, name="grid4_p16")
    say(f"pipeline {prob.name} {precision}")
    s = TwoLevelSolver.for_problem(prob, precision=precision, chunk=32, interface="gpu")
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    ref = _oracle_solution(prob)
    eu = rel(out["u_i"].cpu().numpy(), ref.u_i)
    ef = rel(out["u_face"], ref.u_face)
    be = _backward_error(ref.T_ff, ref.rhs, np.asarray(out["u_face"]))
    say(f"  u_i err {eu:.2e}  u_face err {ef:.2e}  backward error in the oracle's system {be:.2e}  "
        f"refinement steps {out['refine_history']}")
    assert eu < tol and ef < tol and be < 1e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_pipeline_config3_p20_samples(gpu, precision):
    tol = IR_TOL  # solutions: the metric's bar (see test_pipeline_4cubed_p16)
    # 4^3 boxes at p = 20 (5832 interior nodes per box): the oracle's solution at seeded
    # interior and interface nodes and its norms (tests/golden/config3_p20_samples.json)
    import json
    import os
    from paper_2503_04033_amd.solver import TwoLevelSolver
    with open(os.path.join(os.path.dirname(__file__), "golden", "config3_p20_samples.json")) as fh:
        gold = json.load(fh)
    prob = W.config3_p20()
    say(f"pipeline {prob.name} {precision} (sampled oracle)")
    s = TwoLevelSolver.for_problem(prob, precision=precision, chunk=16)
    out = s.solve_problem(prob)
    torch.cuda.synchronize()
    ui = out["u_i"].cpu().numpy()
    got_i = ui[gold["interior_box"], gold["interior_node"]]
    got_f = np.asarray(out["u_face"])[gold["face_index"]]
    ei = rel(got_i, np.asarray(gold["interior_value"]))
    ef = rel(got_f, np.asarray(gold["face_value"]))
    en_i = abs(np.linalg.norm(ui) - gold["norm_u_i"]) / gold["norm_u_i"]
    en_f = abs(np.linalg.norm(out["u_face"]) - gold["norm_u_face"]) / gold["norm_u_face"]
    say(f"  sampled u_i err {ei:.2e}  u_face err {ef:.2e}  norms {en_i:.2e} {en_f:.2e}")
    assert ei < tol and ef < tol and en_i < tol and en_f < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_interior_solve_and_flux(gpu, precision):
    # hps_leaf_interior_solve: u_i = A_ii^{-1} (f_i - A_ib u_b) from the factors with FP64
    # refinement; hps_leaf_flux: A_bi u_i + A_bb u_b; both against the oracle's dense blocks
    prob = W.multi_bump((2, 2, 1), 9, 7.0, 33, gaussian_source=True, name="interior_p9")
    say(f"interior solve and flux {prob.name} {precision}")
    dev = torch.device("cuda")
    ids = list(range(prob.nbox))
    from paper_2503_04033_amd.leaf import LeafPlan
    from oracle import leaf as ol
    plan = LeafPlan(prob.p, prob.h, prob.kappa, precision)
    i = plan.info
    nb = len(ids)
    org = prob.box_origins()
    xi = np.stack([ol.box_node_coords(org[t], prob.h, prob.p)[0] for t in ids])
    rng = np.random.default_rng(8)
    ub = rng.standard_normal((nb, i.n_b))
    bv = torch.tensor(prob.b(xi), device=dev).contiguous()
    fv = torch.tensor(prob.f(xi), device=dev).contiguous()
    ubd = torch.tensor(ub, device=dev).contiguous()
    bufs = plan.alloc(nb, dev)
    plan.hps_leaf_operators(nb, bv, bufs["A"], bufs["anorm"])
    plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
    ui = torch.empty(nb, i.n_i, dtype=torch.float64, device=dev)
    flux = torch.empty(nb, i.n_b, dtype=torch.float64, device=dev)
    berr = torch.empty(nb, dtype=torch.float64, device=dev)
    plan.hps_leaf_interior_solve(nb, bufs["A"], bufs["perm"], bufs["dinv"], bv, bufs["anorm"], fv, ubd, ui, 2, berr,
                                 bufs["ws"])
    plan.hps_leaf_flux(nb, ui, ubd, flux)
    torch.cuda.synchronize()
    say(f"  interior backward errors {berr.cpu().numpy().tolist()}")
    assert float(berr.max()) < 1e-14
    ui_h, fl_h = ui.cpu().numpy(), flux.cpu().numpy()
    for k, t in enumerate(ids):
        blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(xi[k]))
        u_ref = ol.interior_solve(blk, prob.f(xi[k]), ub[k])
        fl_ref = blk.A_bi @ u_ref + blk.A_bb @ ub[k]
        eu, ef = rel(ui_h[k], u_ref), rel(fl_h[k], fl_ref)
        say(f"  box {t}: u_i err {eu:.2e}  flux err {ef:.2e}")
        assert eu < FP64_TOL and ef < FP64_TOL


def test_pipeline_tuned_matches_default(gpu):
    # the solver with every non-default scheduling knob gives bitwise the default solution
    from paper_2503_04033_amd.solver import TwoLevelSolver
    prob = W.multi_bump((2, 2, 2), 8, 6.0, 15, gaussian_source=True, name="tuned_p8")
    outs = []
    for tuning in (None, {"trsm_schedule": 1, "trsm_waves": 8, "residual_cols": 4}):
        s = TwoLevelSolver.for_problem(prob, precision="fp32_ir", tuning=tuning)
        outs.append(s.solve_problem(prob))
        torch.cuda.synchronize()
    assert torch.equal(outs[0]["u_i"], outs[1]["u_i"])
    assert np.array_equal(outs[0]["u_face"], outs[1]["u_face"])


def test_mixed_refinement_steps(gpu):
    # Boxes of one launch that stop after 0 corrections keep the FP32 first solution as X;
    # the others take the correction path.  ir_tol is set between the boxes' backward
    # errors after the first solve so both kinds occur; each box must equal, bitwise, the
    # run that takes the same number of steps.
    prob = W.multi_bump((2, 2, 2), 9, 6.0, 16, gaussian_source=True, name="mixed_p9")
    zero = gpu_leaf_boxes(prob, range(8), "fp32_ir", ir_max_iter=0, ir_tol=1e-30)
    tol = float(np.median(zero["berr"]))
    mixed = gpu_leaf_boxes(prob, range(8), "fp32_ir", ir_max_iter=3, ir_tol=tol)
    full = gpu_leaf_boxes(prob, range(8), "fp32_ir", ir_max_iter=3, ir_tol=1e-12)
    it = mixed["iters"]
    say(f"  berr after the first solve {zero['berr'].tolist()}; steps at tol {tol:.2e}: {it.tolist()}")
    assert (it == 0).any() and (it > 0).any()
    for k in range(8):
        ref = zero if it[k] == 0 else full
        if it[k] > 0:
            assert full["iters"][k] == it[k]
        for key in ("X", "T", "g"):
            assert np.array_equal(mixed[key][k], ref[key][k]), (k, key)


def test_panel_threads_1024_bitwise(gpu):
    # the 1024-thread panel factorization (three rows per thread) at p = 16 chooses the same
    # pivots and computes every row with the same operations as the 512-thread one: LU
    # factors, pivot order and the whole reduction agree bitwise
    prob = W.multi_bump((2, 2, 2), 16, 6.0, 30, gaussian_source=True, name="panel1024_p16")
    runs = [gpu_leaf_boxes(prob, range(3), "fp32_ir", tuning={"panel_threads": nt}) for nt in (512, 1024)]
    assert runs[0]["plan"].info.n_pad > 2048
    for key in ("LU", "perm", "X", "T", "g", "info", "iters"):
        assert np.array_equal(runs[0][key], runs[1][key]), key


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_workspace_bytes(gpu, precision):
    # hps_leaf_workspace_bytes states each call's workspace: the DtN's per-box figure of
    # hps_plan_get_info, one FP64 vector and three scalars per box for the interior solve,
    # two padded FP64 vectors per box for the adjoint solve; bad arguments are rejected
    from paper_2503_04033_amd._lib import HpsError, check
    from paper_2503_04033_amd.leaf import LeafPlan
    plan = LeafPlan(12, (0.5, 0.5, 0.5), 10.0, precision)
    i = plan.info
    for nb in (0, 1, 37):
        assert plan.hps_leaf_workspace_bytes("dtn", nb) == nb * i.ws_bytes
        assert plan.hps_leaf_workspace_bytes("interior_solve", nb) == 8 * nb * (i.n_i + 3)
        assert plan.hps_leaf_workspace_bytes("adjoint_solve", nb) == 16 * nb * i.n_pad
    assert plan.hps_leaf_workspace_bytes("interior_solve", 1) <= i.ws_bytes
    import ctypes as C
    v = C.c_size_t(7)
    with pytest.raises(HpsError):
        check(plan.lib.hps_leaf_workspace_bytes(plan.handle, 3, 1, C.byref(v)), "bad call")
    assert v.value == 7
    with pytest.raises(HpsError):
        plan.hps_leaf_workspace_bytes("dtn", -1)


def test_zero_load_passed_converges(gpu):
    # a load that is passed but exactly zero: its column's backward error is 0 / 0, which
    # counts as converged (every box stops after its usual correction, bitwise the run
    # without a load)
    prob = W.multi_bump((2, 2, 2), 8, 6.0, 12, name="zero_load_p8")
    assert not np.any(prob.f(np.random.default_rng(0).random((5, 3))))
    withf = gpu_leaf_boxes(prob, range(8), "fp32_ir", f_on=True)
    nof = gpu_leaf_boxes(prob, range(8), "fp32_ir", f_on=False)
    assert np.all(withf["iters"] >= 0)
    for key in ("X", "T", "g", "iters"):
        assert np.array_equal(withf[key], nof[key]), key


@pytest.mark.parametrize("ir_max_iter,ir_tol", [(0, 1e-30), (3, None)])
def test_berr_includes_load_column(gpu, ir_max_iter, ir_tol):
    # berr is the larger of the backward error over all columns of [A_ib | f] and that of
    # the load column alone (whose entries are far smaller than A_ib's).  Both are formed
    # here from the GPU's own X with the oracle's dense A_ii and compared with berr: after
    # the first FP32 solve (no correction; both figures near 1e-7, far above rounding) and
    # after refinement (below the tolerance)
    from oracle import leaf as ol
    prob = W.multi_bump((2, 2, 2), 8, 6.0, 12, gaussian_source=True, name="berr_p8")
    out = gpu_leaf_boxes(prob, range(4), "fp32_ir", ir_max_iter=ir_max_iter, ir_tol=ir_tol, f_on=True)
    for k in range(4):
        blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(out["xi"][k]))
        A = blk.A_ii
        B = np.concatenate([blk.A_ib, prob.f(out["xi"][k])[:, None]], axis=1)
        X = out["X"][k]
        R = B - A @ X
        anorm = np.abs(A).sum(axis=1).max()
        be_all = np.abs(R).max() / (anorm * np.abs(X).max() + np.abs(B).max())
        be_f = np.abs(R[:, -1]).max() / (anorm * np.abs(X[:, -1]).max() + np.abs(B[:, -1]).max())
        ref = max(be_all, be_f)
        say(f"  box {k}: berr {out['berr'][k]:.3e}, host all-columns {be_all:.3e}, load column {be_f:.3e}")
        if ir_max_iter == 0:
            assert 0.5 * ref <= out["berr"][k] <= 2.0 * ref
        else:
            from paper_2503_04033_amd.leaf import default_ir_tol
            assert out["berr"][k] <= default_ir_tol(prob.p)
            assert be_f <= 1e-11


def _lu_rule(A):
    """Partial pivoting as hps_leaf_factor documents it: in column k the row of largest
    modulus among the rows not yet pivoted, the lowest current position on ties; the
    chosen row takes position k and the rows it passes keep their order.  Returns
    (order, B, ties): order[i] = the row at position i, B[i] = row i of L (below the
    diagonal) and U, ties = the steps where more than one row had the largest modulus."""
    B = A.copy()
    n = len(B)
    order = np.arange(n)
    ties = 0
    for k in range(n):
        col = np.abs(B[k:, k])
        j = k + int(np.argmax(col))  # (the first maximum: lowest position)
        ties += int(np.count_nonzero(col == col[j - k]) > 1)
        if j != k:
            B[k:j + 1] = np.roll(B[k:j + 1], 1, axis=0)
            order[k:j + 1] = np.roll(order[k:j + 1], 1)
        lk = B[k + 1:, k] / B[k, k]
        B[k + 1:, k] = lk
        B[k + 1:, k + 1:] -= np.outer(lk, B[k, k + 1:])
    return order, B, ties


_TIE_REF = {}


def _tie_matrix(n, seed):
    # rows of diag(H_64 (x) I_q, H_32) (H_64 and H_32 the Sylvester-Hadamard matrices, H_32
    # only where n = 64 q + 32), in a seeded order
    H = [np.ones((1, 1))]
    for _ in range(6):
        H.append(np.block([[H[-1], H[-1]], [H[-1], -H[-1]]]))
    q, rem = divmod(n, 64)
    assert rem in (0, 32)
    A = np.zeros((n, n))
    A[:64 * q, :64 * q] = np.kron(H[6], np.eye(q))
    if rem:
        A[64 * q:, 64 * q:] = H[5]
    A = A[np.random.default_rng(seed).permutation(n)]
    if (n, seed) not in _TIE_REF:
        _TIE_REF[(n, seed)] = _lu_rule(A)
    return A, _TIE_REF[(n, seed)]


@pytest.mark.parametrize("precision,p,threads", [("fp32_ir", 8, None), ("fp64", 8, None), ("fp32_ir", 15, 1024),
                                                 ("fp32_ir", 15, 512), ("fp64", 15, None)])
def test_pivot_ties_exact(gpu, precision, p, threads):
    # A matrix with a tie in modulus at nearly every elimination step whose factors are exact
    # in any summation order (every entry of L is 0 or +-1, of U an integer up to 64, every
    # partial sum of products below 2^9 in modulus): the pivot order and the factors must be the rule's
    # exactly (p = 15: n_pad 2240, the 1024- and 512-thread FP32 panels)
    from paper_2503_04033_amd.leaf import LeafPlan
    plan = LeafPlan(p, (0.5, 0.5, 0.5), 5.0, precision)
    if threads:
        plan.hps_plan_set_tuning("panel_threads", threads)
    i = plan.info
    n, nb = i.n_pad, 2 if p == 8 else 1
    say(f"case pivot ties p={p} n_pad={n} {precision} panel_threads={threads}")
    dev = torch.device("cuda")
    bufs = plan.alloc(nb, dev)
    mats = [_tie_matrix(n, 7 + k) for k in range(nb)]
    A = bufs["A"].view(nb, n, n)
    for k, (Ak, _) in enumerate(mats):
        A[k].copy_(torch.tensor(Ak, dtype=A.dtype))
    plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
    torch.cuda.synchronize()
    perm = bufs["perm"].view(nb, n).cpu().numpy()
    LU = A.cpu().numpy().astype(np.float64)
    assert np.all(bufs["info"].cpu().numpy() == 0)
    for k, (Ak, (order, B, ties)) in enumerate(mats):
        say(f"  box {k}: ties at {ties} of {n} steps; pivots equal {np.array_equal(perm[k], order)}, "
            f"factors equal {np.array_equal(LU[k][perm[k]], B)}")
        assert ties > 0.9 * n
        assert np.abs(B).max() <= 64 and np.array_equal(B, np.round(B))  # integer factors
        assert np.array_equal((np.tril(B, -1) + np.eye(n)) @ np.triu(B), Ak[order])  # exact
        assert np.array_equal(perm[k], order)
        assert np.array_equal(LU[k][perm[k]], B)
