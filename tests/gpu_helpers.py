"""Helpers for the GPU parity tests: run the HIP path and the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import interface as oi
from oracle import leaf as ol
from paper_2503_04033_amd.leaf import LeafPlan


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_leaf_boxes(prob, box_ids, precision="fp64", ir_max_iter=3, ir_tol=1e-12, f_on=True, tuning=None):
    """Run a1..a4 on the listed boxes with a slot map that keeps every DtN block.

    tuning: optional {knob: value} set on the plan (hps_plan_set_tuning) first.

    Returns dict with X [nb, n_i, nrhs], T [nb, n_b, n_b], g [nb, n_b], info, iters, berr.
    """
    dev = torch.device("cuda")
    plan = LeafPlan(prob.p, prob.h, prob.kappa, precision, ir_max_iter, ir_tol)
    for k, v in (tuning or {}).items():
        plan.hps_plan_set_tuning(k, v)
        assert plan.hps_plan_get_tuning(k) == v
    i = plan.info
    nb = len(box_ids)
    org = prob.box_origins()[box_ids]
    xi = np.zeros((nb, i.n_i, 3))
    for k, t in enumerate(box_ids):
        xi[k], _ = ol.box_node_coords(org[k], prob.h, prob.p)
    b = torch.tensor(prob.b(xi), dtype=torch.float64, device=dev).contiguous()
    f = torch.tensor(prob.f(xi), dtype=torch.float64, device=dev).contiguous() if f_on else None
    bufs = plan.alloc(nb, dev)
    mm = i.m * i.m
    slot = torch.arange(nb * 36, dtype=torch.int32, device=dev)
    T_vals = torch.zeros(nb * 36 * mm * mm, dtype=torch.float64, device=dev)
    g = torch.zeros(nb, i.n_b, dtype=torch.float64, device=dev)
    say(f"  gpu leaf: p={prob.p} nbox={nb} prec={precision} n_pad={i.n_pad} ldx={i.ldx}")
    plan.hps_leaf_operators(nb, b, bufs["A"], bufs["anorm"])
    A0 = bufs["A"].clone()
    plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
    plan.hps_leaf_dtn(nb, bufs["A"], bufs["perm"], bufs["dinv"], b, bufs["anorm"], f, None, slot, T_vals, g,
                      bufs["X"], bufs["ir_iters"], bufs["berr"], bufs["ws"])
    torch.cuda.synchronize()
    X = bufs["X"].view(nb, i.n_pad, i.ldx)[:, :i.n_i, :i.nrhs].cpu().numpy()
    T6 = T_vals.view(nb, 6, 6, mm, mm).cpu().numpy()
    T = T6.transpose(0, 1, 3, 2, 4).reshape(nb, i.n_b, i.n_b)
    return {"X": X, "T": T, "T6": T6, "g": g.cpu().numpy(), "info": bufs["info"].cpu().numpy(),
            "iters": bufs["ir_iters"].cpu().numpy(), "berr": bufs["berr"].cpu().numpy(),
            "A0": A0.view(nb, i.n_pad, i.n_pad).cpu().numpy(),
            "LU": bufs["A"].view(nb, i.n_pad, i.n_pad).cpu().numpy(),
            "perm": bufs["perm"].view(nb, i.n_pad).cpu().numpy(), "plan": plan, "xi": xi, "ws": bufs["ws"]}


def oracle_leaf_boxes(prob, box_ids, f_on=True):
    org = prob.box_origins()
    out = []
    for t in box_ids:
        xi, xb = ol.box_node_coords(org[t], prob.h, prob.p)
        blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(xi))
        f = prob.f(xi) if f_on else np.zeros(xi.shape[0])
        out.append((blk, ol.leaf_reduce(blk, f)))
    return out


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def rel_fro_max(A, B):
    """max over boxes of ||A_t - B_t||_F / ||B_t||_F."""
    return max(rel(a, b) for a, b in zip(A, B))


def oracle_solution(prob):
    return oi.solve(prob)
