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


def box_boundary_faces(prob, t):
    """Faces (0..5 = x-, x+, y-, y+, z-, z+) of box t that lie on the domain boundary."""
    n1, n2, n3 = prob.nboxes
    c = (t % n1, (t // n1) % n2, t // (n1 * n2))
    dims = (n1, n2, n3)
    return [2 * a + s for a in range(3) for s in range(2) if c[a] == (0 if s == 0 else dims[a] - 1)]


def gpu_leaf_boxes(prob, box_ids, precision="fp64", ir_max_iter=3, ir_tol=None, f_on=True, tuning=None,
                   plan_nodes=False, lift=False, copy_factors=True):
    """Run a1..a4 on the listed boxes with a slot map that keeps every DtN block.

    tuning: optional {knob: value} set on the plan (hps_plan_set_tuning) first.
    plan_nodes: evaluate b and f at the node coordinates of hps_leaf_nodes (else at the
    oracle's coordinates).  lift: pass the Dirichlet data of the boxes' boundary faces
    (g_dir), so that g is the lifted load.  copy_factors: also return A0, LU and perm.

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
    xb = np.zeros((nb, i.n_b, 3))
    if plan_nodes:
        xid = torch.empty(nb * i.n_i * 3, dtype=torch.float64, device=dev)
        xbd = torch.empty(nb * i.n_b * 3, dtype=torch.float64, device=dev)
        plan.hps_leaf_nodes(nb, torch.tensor(org, device=dev).contiguous(), xid, xbd)
        xi, xb = xid.view(nb, i.n_i, 3).cpu().numpy(), xbd.view(nb, i.n_b, 3).cpu().numpy()
    else:
        for k, t in enumerate(box_ids):
            xi[k], xb[k] = ol.box_node_coords(org[k], prob.h, prob.p)
    gd = None
    if lift:
        mm_ = i.m * i.m
        gd_h = np.zeros((nb, i.n_b))
        for k, t in enumerate(box_ids):
            for a in box_boundary_faces(prob, t):
                gd_h[k, a * mm_:(a + 1) * mm_] = prob.g(xb[k, a * mm_:(a + 1) * mm_])
        gd = torch.tensor(gd_h, device=dev).contiguous()
    b = torch.tensor(prob.b(xi), dtype=torch.float64, device=dev).contiguous()
    f = torch.tensor(prob.f(xi), dtype=torch.float64, device=dev).contiguous() if f_on else None
    bufs = plan.alloc(nb, dev)
    mm = i.m * i.m
    slot_h = np.arange(nb * 36, dtype=np.int32).reshape(nb, 6, 6)
    if lift:  # the library lifts by the columns whose slot is -1 (boundary faces); their rows drop too
        for k, t in enumerate(box_ids):
            for a in box_boundary_faces(prob, t):
                slot_h[k, a, :] = -1
                slot_h[k, :, a] = -1
    slot = torch.tensor(slot_h.reshape(-1), device=dev)
    T_vals = torch.zeros(nb * 36 * mm * mm, dtype=torch.float64, device=dev)
    g = torch.zeros(nb, i.n_b, dtype=torch.float64, device=dev)
    say(f"  gpu leaf: p={prob.p} nbox={nb} prec={precision} n_pad={i.n_pad} ldx={i.ldx}")
    plan.hps_leaf_operators(nb, b, bufs["A"], bufs["anorm"])
    A0 = bufs["A"].clone() if copy_factors else None
    plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
    plan.hps_leaf_dtn(nb, bufs["A"], bufs["perm"], bufs["dinv"], b, bufs["anorm"], f, gd, slot, T_vals, g,
                      bufs["X"], bufs["ir_iters"], bufs["berr"], bufs["ws"])
    torch.cuda.synchronize()
    X = bufs["X"].view(nb, i.n_pad, i.ldx)[:, :i.n_i, :i.nrhs].cpu().numpy()
    T6 = T_vals.view(nb, 6, 6, mm, mm).cpu().numpy()
    T = T6.transpose(0, 1, 3, 2, 4).reshape(nb, i.n_b, i.n_b)
    out = {"X": X, "T": T, "T6": T6, "g": g.cpu().numpy(), "info": bufs["info"].cpu().numpy(),
           "iters": bufs["ir_iters"].cpu().numpy(), "berr": bufs["berr"].cpu().numpy(), "plan": plan, "xi": xi,
           "xb": xb, "ws": bufs["ws"], "g_dir": gd.cpu().numpy() if gd is not None else None}
    if copy_factors:
        out.update(A0=A0.view(nb, i.n_pad, i.n_pad).cpu().numpy(),
                   LU=bufs["A"].view(nb, i.n_pad, i.n_pad).cpu().numpy(),
                   perm=bufs["perm"].view(nb, i.n_pad).cpu().numpy())
    return out


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
