"""GPU: several independent problems batched in one stream (configuration 4).

* Oracle parity on sampled boxes of every size group: every DtN block a box
  writes (both faces internal; a shared diagonal block in the box's own slot,
  before the reduction sums the two boxes) and the Dirichlet-lifted loads
  g = -A_bi v - sum_{boundary faces b} T[:, b] g_b, FP32+IR bar 1e-9.
* The batched run equals per-problem runs bitwise (same kernels, same chunks).
* A HIP graph of the whole build stage, replayed three times with eager work
  and synchronizations in between, reproduces the eager result bitwise.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import leaf as ol
from tests.gpu_helpers import rel, say

pytestmark = pytest.mark.gpu


def _oracle_box(prob, t):
    org = prob.box_origins()[t]
    xi, xb = ol.box_node_coords(org, prob.h, prob.p)
    blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(xi))
    return ol.leaf_reduce(blk, prob.f(xi)), xb


def _check_group(br, q, prob, boxes):
    gr = br.groups[q]
    m = gr.plan.info.m
    mm = m * m
    T = gr.T_vals[:-1].view(-1, mm, mm)
    gl = gr.g_loads.cpu().numpy()
    for t in boxes:
        red, xb = _oracle_box(prob, t)
        faces = gr.layout.box_faces[t]
        gdir = np.where(np.repeat(faces < 0, mm), prob.g(xb), 0.0)
        worst = 0.0
        for a in range(6):
            for bb in range(6):
                s = gr.layout.slot_map[t, 6 * a + bb]
                if s >= 0:
                    got = T[s].cpu().numpy()
                    ref = red.T[a * mm:(a + 1) * mm, bb * mm:(bb + 1) * mm]
                    worst = max(worst, rel(got, ref))
        g_ref = red.g - red.T @ gdir
        rows = np.repeat(faces >= 0, mm)
        eg = rel(gl[t][rows], g_ref[rows])
        say(f"  group p={prob.p} box {t}: T blocks err {worst:.2e}, lifted load err {eg:.2e}")
        assert worst < 1e-9 and eg < 1e-9


def test_three_problem_batch(gpu):
    from paper_2503_04033_amd.batch import BatchedLeafReduction
    probs = W.config4()
    say("batch: " + ", ".join(f"{p.name} ({p.nbox} boxes, p={p.p})" for p in probs))
    br = BatchedLeafReduction(probs, "fp32_ir", hbm_budget=24e9)
    for q, pr in enumerate(probs):
        br.sample_inputs(q, pr)
    br.allocate()
    br.run()
    torch.cuda.synchronize()
    for q, pr in enumerate(probs):
        n1 = pr.nboxes[0]
        interior = n1 // 2 + n1 * (n1 // 2 + n1 * (n1 // 2))
        _check_group(br, q, pr, [0, interior])
        assert int((br.groups[q].info != 0).sum()) == 0
        assert int(br.groups[q].iters.min()) >= 0
    eager = [(g.T_vals.clone(), g.g_loads.clone()) for g in br.groups]
    # each problem alone gives the same bits
    for q, pr in enumerate(probs):
        one = BatchedLeafReduction([pr], "fp32_ir", chunks=[br.groups[q].chunk])
        one.set_inputs(0, br.groups[q].b, br.groups[q].f, br.groups[q].g_dir)
        one.allocate()
        one.run()
        torch.cuda.synchronize()
        assert torch.equal(one.groups[0].T_vals, eager[q][0])
        assert torch.equal(one.groups[0].g_loads, eager[q][1])
        del one
    # graph capture and replays
    br.capture()
    for rep in range(3):
        for g in br.groups:
            g.T_vals[:-1].fill_(-1.0)  # the last element is a spare, never written by kernels
            g.g_loads.fill_(-1.0)
        torch.cuda.synchronize()
        br.run()
        torch.cuda.synchronize()
        for q, g in enumerate(br.groups):
            assert torch.equal(g.T_vals, eager[q][0]), f"replay {rep} group {q}: T differs"
            assert torch.equal(g.g_loads, eager[q][1]), f"replay {rep} group {q}: g differs"
        say(f"  graph replay {rep}: bitwise equal to the eager run")
    # the three groups on concurrent streams: eagerly, then as a captured graph whose branches
    # overlap, each replay bitwise the sequential results
    for g in br.groups:
        g.T_vals[:-1].fill_(-1.0)
        g.g_loads.fill_(-1.0)
    br.graph = None
    br.run(concurrent=True)
    torch.cuda.synchronize()
    for q, g in enumerate(br.groups):
        assert torch.equal(g.T_vals, eager[q][0]) and torch.equal(g.g_loads, eager[q][1])
    br.capture(concurrent=True)
    for rep in range(3):
        for g in br.groups:
            g.T_vals[:-1].fill_(-1.0)
            g.g_loads.fill_(-1.0)
        torch.cuda.synchronize()
        br.run()
        torch.cuda.synchronize()
        for q, g in enumerate(br.groups):
            assert torch.equal(g.T_vals, eager[q][0]), f"concurrent replay {rep} group {q}: T differs"
            assert torch.equal(g.g_loads, eager[q][1]), f"concurrent replay {rep} group {q}: g differs"
        say(f"  concurrent-branch graph replay {rep}: bitwise equal to the eager run")


def test_autotune_config4(gpu, tmp_path):
    # the autotuner's choices (chunk, solve schedule, occupancy, residual blocking, panel threads) per size group: valid,
    # cached, and bitwise the same results as the untuned run
    from paper_2503_04033_amd.batch import PANEL_KNOBS, RESIDUAL_KNOBS, TRSM_KNOBS, BatchedLeafReduction, autotune
    probs = W.config4()
    cache = str(tmp_path / "tune.json")
    tuned = autotune(probs, "fp32_ir", candidates=(256, 4096), hbm_budget=24e9, cache=cache)
    for pr, t in zip(probs, tuned):
        say(f"  autotune p={pr.p} nbox={pr.nbox}: chunk {t['chunk']}, {t['tuning']}")
        assert t["chunk"] in (256, min(4096, pr.nbox))
        # the panel's thread count is tuned only for the p = 16 group (2744 rows)
        assert set(t["tuning"]) == {"trsm_schedule", "trsm_waves", "residual_cols"} | (
            {"panel_threads"} if pr.p == 16 else set())
        if pr.p == 16:
            assert {"panel_threads": t["tuning"]["panel_threads"]} in PANEL_KNOBS
        assert {k: t["tuning"][k] for k in ("trsm_schedule", "trsm_waves")} in TRSM_KNOBS
        assert {"residual_cols": t["tuning"]["residual_cols"]} in RESIDUAL_KNOBS
    assert autotune(probs, "fp32_ir", candidates=(256, 4096), hbm_budget=24e9, cache=cache) == tuned
    runs = []
    for kw in ({}, {"chunks": [t["chunk"] for t in tuned], "tuning": [t["tuning"] for t in tuned]}):
        br = BatchedLeafReduction(probs, "fp32_ir", hbm_budget=24e9, **kw)
        for q, pr in enumerate(probs):
            br.sample_inputs(q, pr)
        br.allocate()
        br.run()
        torch.cuda.synchronize()
        runs.append([(g.T_vals.clone(), g.g_loads.clone(), g.iters.clone()) for g in br.groups])
        del br
    for q in range(len(probs)):
        for a, b in zip(runs[0][q], runs[1][q]):
            assert torch.equal(a, b), f"group {q}: tuned run differs"


def test_full_size_config3_sampled(gpu):
    # The headline workload at full size in the launch configuration the benchmark times
    # (16^3 boxes, p = 16, FP32 + refinement, chunks of 2048 boxes, f = 0 passed as null):
    # every box factors and converges; sampled boxes (corner, edge, interior, last)
    # against the oracle: off-diagonal DtN blocks and lifted loads, bar 1e-9.  (About
    # 213 GB of HBM: memory cached by earlier tests is released first.)
    from paper_2503_04033_amd.batch import BatchedLeafReduction
    torch.cuda.empty_cache()
    prob = W.config3()
    br = BatchedLeafReduction([prob], "fp32_ir", chunks=[2048])
    br.sample_inputs(0, prob)
    gr = br.groups[0]
    br.set_inputs(0, gr.b, None, gr.g_dir)
    br.allocate()
    say(f"full size: {prob.nbox} boxes, chunk {gr.chunk}")
    br.run()
    torch.cuda.synchronize()
    assert int((gr.info != 0).sum()) == 0
    it = gr.iters.cpu().numpy()
    say(f"  refinement steps: {np.bincount(it[it >= 0]).tolist()}, unconverged {(it < 0).sum()}")
    assert it.min() >= 0
    n1 = prob.nboxes[0]
    _check_group(br, 0, prob, [0, n1 - 1, 8 + n1 * (8 + n1 * 8), prob.nbox - 1])
    del br, gr
    torch.cuda.empty_cache()


def test_batch_fp64_fallback_after_replay(gpu):
    # ir_max_iter = 0 and an unreachable tolerance: every box of the FP32 + refinement run is
    # flagged; fallback() redoes them with FP64 factors after the (captured) run and
    # reduces the diagonal blocks again, giving bitwise the FP64 run's interface matrix
    from paper_2503_04033_amd.batch import BatchedLeafReduction
    prob = W.multi_bump((2, 2, 3), 8, 6.0, 51, gaussian_source=True, name="batch_fallback")
    f64 = BatchedLeafReduction([prob], "fp64", chunks=[5])
    f64.sample_inputs(0, prob)
    f64.allocate()
    f64.run()
    bad = BatchedLeafReduction([prob], "fp32_ir", ir_max_iter=0, ir_tol=1e-30, chunks=[4])
    gr = bad.groups[0]
    bad.set_inputs(0, f64.groups[0].b, f64.groups[0].f, f64.groups[0].g_dir)
    bad.allocate()
    bad.capture()
    for rep in range(2):
        gr.T_vals[:-1].fill_(-1.0)
        gr.g_loads.fill_(-1.0)
        bad.run()
        torch.cuda.synchronize()
        assert int((gr.iters >= 0).sum()) == 0
        done = bad.fallback()
        torch.cuda.synchronize()
        assert done == {0: list(range(prob.nbox))}
        assert torch.equal(gr.T_vals, f64.groups[0].T_vals), f"replay {rep}: T differs"
        assert torch.equal(gr.g_loads, f64.groups[0].g_loads), f"replay {rep}: g differs"
        say(f"  replay {rep}: fallback gives bitwise the FP64 interface matrix")
