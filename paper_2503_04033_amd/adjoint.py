"""Gradient of a data misfit with respect to the coefficient b (spec a6).

u = A(b)^{-1} rhs is the two-level solution (eq. factor2).  b enters A only as
-kappa^2 b on the diagonal of interior collocation rows, so for any scalar
J(u_i):  dJ/db_n = kappa^2 lambda_n u_n  with  A^T lambda = dJ/du  (interior nodes).
The transpose of eq. factor2, A^{-T} = Atil^{-T} L^{-T} D^{-T} U^{-T}, gives per box
    z = A_ii^{-T} w_i,  y_b = -A_ib^T z     (GPU, hps_leaf_adjoint_solve)
    lambda_F = T_FF^{-T} sum_boxes y_b      (host sparse LU, transposed)
    lambda_i = A_ii^{-T} (w_i - A_bi^T lambda_b)   (GPU)
    grad = kappa^2 lambda_i * u_i           (GPU, hps_leaf_adjoint_grad)
The LU factors of every box stay on the GPU between the forward and backward
passes (FP64 plans).
"""
from __future__ import annotations

import numpy as np
import torch

from . import interface as itf
from .leaf import hps_interface_reduce
from .solver import TwoLevelSolver


class ResidentForward:
    """Forward two-level solve that keeps every box's factors for the adjoint."""

    def __init__(self, solver: TwoLevelSolver):
        if solver.plan.precision != "fp64":
            raise ValueError("the adjoint path runs on FP64 plans")
        self.s = solver
        i = solver.info
        nbox = solver.nbox
        self.bufs = solver.plan.alloc(nbox, solver.device)
        mm = i.m * i.m
        self.T_vals = torch.zeros(solver.layout.nslot_total * mm * mm + 1, dtype=torch.float64,
                                  device=solver.device)
        self.g_loads = torch.empty(nbox, i.n_b, dtype=torch.float64, device=solver.device)

    def forward(self, b: torch.Tensor, f, g_dir: torch.Tensor):
        s, B, plan, nbox, i = self.s, self.bufs, self.s.plan, self.s.nbox, self.s.info
        b = b.contiguous()
        plan.hps_leaf_operators(nbox, b, B["A"], B["anorm"])
        plan.hps_leaf_factor(nbox, B["A"], B["perm"], B["dinv"], B["info"])
        self.T_vals.zero_()
        plan.hps_leaf_dtn(nbox, B["A"], B["perm"], B["dinv"], b, B["anorm"], f, g_dir, s.slot_map, self.T_vals,
                          self.g_loads, B["X"], B["ir_iters"], B["berr"], B["ws"])
        pairs = torch.tensor(s.layout.reduce_pairs, device=s.device)
        if pairs.shape[0]:
            hps_interface_reduce(pairs, (i.m * i.m) ** 2, self.T_vals)
        self.isolver = itf.InterfaceSolver(s.layout, self.T_vals.cpu().numpy())
        rhs = itf.interface_rhs(s.layout, self.g_loads.cpu().numpy())
        u_face = self.isolver.solve(rhs)
        ub = torch.tensor(itf.box_face_values(s.layout, u_face, g_dir.cpu().numpy()), device=s.device)
        ui = torch.empty(nbox, i.n_i, dtype=torch.float64, device=s.device)
        plan.hps_leaf_reconstruct(nbox, B["X"], ub, ui)
        self.b = b
        self.u_i = ui
        return ui, u_face

    def gradient(self, w_i: torch.Tensor) -> torch.Tensor:
        """dJ/db at interior nodes for dJ/du_i = w_i (both [nbox, n_i])."""
        s, B, plan, nbox, i = self.s, self.bufs, self.s.plan, self.s.nbox, self.s.info
        w_i = w_i.contiguous().to(torch.float64)
        z = torch.empty(nbox, i.n_i, dtype=torch.float64, device=s.device)
        yb = torch.empty(nbox, i.n_b, dtype=torch.float64, device=s.device)
        plan.hps_leaf_adjoint_solve(nbox, B["A"], B["perm"], B["dinv"], self.b, w_i, None, z, yb, B["ws"])
        y_face = itf.interface_rhs(s.layout, yb.cpu().numpy())
        lam_face = self.isolver.solve(y_face, trans="T")
        lam_b = itf.box_face_values(s.layout, lam_face, np.zeros((nbox, i.n_b)))
        lam_b_d = torch.tensor(lam_b, device=s.device)
        lam_i = torch.empty(nbox, i.n_i, dtype=torch.float64, device=s.device)
        plan.hps_leaf_adjoint_solve(nbox, B["A"], B["perm"], B["dinv"], self.b, w_i, lam_b_d, lam_i, None, B["ws"])
        grad = torch.empty(nbox, i.n_i, dtype=torch.float64, device=s.device)
        plan.hps_leaf_adjoint_grad(nbox, lam_i, self.u_i, grad)
        return grad


class HPSSolve(torch.autograd.Function):
    """u_i = two-level solution for coefficient b (interior nodes); differentiable in b."""

    @staticmethod
    def forward(ctx, b, solver, f, g_dir):
        fwd = ResidentForward(solver)
        ui, _ = fwd.forward(b, f, g_dir)
        ctx.fwd = fwd
        return ui.clone()

    @staticmethod
    def backward(ctx, grad_u):
        return ctx.fwd.gradient(grad_u), None, None, None
