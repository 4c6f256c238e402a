"""Gradient of a data misfit with respect to the coefficient b (spec a6).

u = A(b)^{-1} rhs is the two-level solution (eq. factor2).  b enters A only as
-kappa^2 b on the diagonal of interior collocation rows, so for any scalar
J(u_i):  dJ/db_n = kappa^2 lambda_n u_n  with  A^T lambda = dJ/du  (interior nodes).
The transpose of eq. factor2, A^{-T} = Atil^{-T} L^{-T} D^{-T} U^{-T}, gives per box
    z = A_ii^{-T} w_i,  y_b = -A_ib^T z     (GPU, hps_leaf_adjoint_solve)
    lambda_F = T_FF^{-T} sum_boxes y_b      (transposed interface solve: GPU nested
                                             dissection, or the host LU)
    lambda_i = A_ii^{-T} (w_i - A_bi^T lambda_b)   (GPU)
    grad = kappa^2 lambda_i * u_i           (GPU, hps_leaf_adjoint_grad)

The transposed solves use every box's FP64 LU factors.  When they fit the HBM
budget next to the interface matrix they stay resident from the forward pass;
otherwise each chunk's operators and factors are computed again in each backward
pass (the paper's recompute-instead-of-store, Sec. 3.2).  The factorization of a
box does not depend on the chunk it is in, so both modes give bitwise the same
gradient.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import interface as itf
from .leaf import hps_interface_reduce
from .nested import NestedDissection
from .solver import TwoLevelSolver, chunk_bytes_per_box, factor_bytes_per_box


class AdjointSolve:
    """Forward two-level solve (FP64 plans) and the gradient of a misfit in b."""

    INTERIOR_STEPS = 1

    def __init__(self, solver: TwoLevelSolver, hbm_budget: Optional[float] = None, resident: Optional[bool] = None,
                 chunk: Optional[int] = None):
        if solver.plan.precision != "fp64":
            raise ValueError("the adjoint path runs on FP64 plans")
        self.s = solver
        i = solver.info
        nbox = solver.nbox
        budget = solver.hbm_budget if hbm_budget is None else float(hbm_budget)
        mm = i.m * i.m
        t_bytes = 8 * (solver.layout.nslot_total * mm * mm + 1) + 8 * nbox * (3 * i.n_i + 3 * i.n_b + 4)
        keep_bytes = nbox * factor_bytes_per_box(i)
        per_chunk_box = chunk_bytes_per_box(i)
        fits = t_bytes + keep_bytes + per_chunk_box <= budget
        if resident is None:
            resident = fits
        elif resident and not fits:
            raise ValueError(f"resident factors need {(t_bytes + keep_bytes) / 1e9:.1f} GB plus a chunk; the "
                             f"HBM budget is {budget / 1e9:.1f} GB")
        self.resident = bool(resident)
        fit = int((budget - t_bytes - (keep_bytes if self.resident else 0)) // per_chunk_box)
        if fit < 1:
            raise ValueError("one box of working buffers does not fit the HBM budget")
        self.chunk = min(int(chunk) if chunk else solver.chunk, fit, nbox)
        dev = solver.device
        C = self.chunk
        self.bufs = solver.plan.alloc(C, dev)
        a_el, d_el = i.a_bytes // i.elem_bytes, i.dinv_bytes // i.elem_bytes
        self.factors = None
        if self.resident:
            self.factors = {"LU": torch.empty(nbox * a_el, dtype=torch.float64, device=dev),
                            "perm": torch.empty(nbox * i.n_pad, dtype=torch.int32, device=dev),
                            "dinv": torch.empty(nbox * d_el, dtype=torch.float64, device=dev)}
        self.T_vals = torch.zeros(solver.layout.nslot_total * mm * mm + 1, dtype=torch.float64, device=dev)
        self.g_loads = torch.empty(nbox, i.n_b, dtype=torch.float64, device=dev)
        self.anorm = torch.empty(nbox, dtype=torch.float64, device=dev)
        self.info = torch.empty(nbox, dtype=torch.int32, device=dev)
        self.refactorizations = 0

    def _chunks(self):
        for c0 in range(0, self.s.nbox, self.chunk):
            yield c0, min(self.chunk, self.s.nbox - c0)

    def _factors(self, c0: int, nb: int, b: torch.Tensor, fresh: bool = False):
        """Factors of boxes [c0, c0 + nb): resident slices, or operators and LU computed into
        the chunk buffers (always when `fresh`, i.e. the forward pass that writes them)."""
        i, plan, B = self.s.info, self.s.plan, self.bufs
        sl = slice(c0, c0 + nb)
        if self.resident:
            a_el, d_el = i.a_bytes // i.elem_bytes, i.dinv_bytes // i.elem_bytes
            A = self.factors["LU"][c0 * a_el:(c0 + nb) * a_el]
            perm = self.factors["perm"][c0 * i.n_pad:(c0 + nb) * i.n_pad]
            dinv = self.factors["dinv"][c0 * d_el:(c0 + nb) * d_el]
        else:
            A, perm, dinv = B["A"], B["perm"], B["dinv"]
        if fresh or not self.resident:
            plan.hps_leaf_operators(nb, b[sl].contiguous(), A, self.anorm[sl])
            plan.hps_leaf_factor(nb, A, perm, dinv, self.info[sl])
            self.refactorizations += 1
        return A, perm, dinv

    def forward(self, b: torch.Tensor, f, g_dir: torch.Tensor):
        s, plan, nbox, i = self.s, self.s.plan, self.s.nbox, self.s.info
        b = b.contiguous()
        self.T_vals.zero_()
        B = self.bufs
        for c0, nb in self._chunks():
            sl = slice(c0, c0 + nb)
            A, perm, dinv = self._factors(c0, nb, b, fresh=True)
            plan.hps_leaf_dtn(nb, A, perm, dinv, b[sl], self.anorm[sl], f[sl].contiguous() if f is not None else None,
                              g_dir[sl].contiguous(), s.slot_map[sl].contiguous(), self.T_vals, self.g_loads[sl],
                              B["X"], B["ir_iters"], B["berr"], B["ws"])
        triples = torch.tensor(s.layout.reduce_triples, device=s.device)
        if triples.shape[0]:
            hps_interface_reduce(triples, (i.m * i.m) ** 2, self.T_vals)
        self.isolver = s.factor_interface(self.T_vals)
        if isinstance(self.isolver, NestedDissection):
            u_d = self.isolver.solve(self.g_loads)
            ub = self.isolver.face_values(u_d, g_dir.contiguous())
            u_face = u_d.cpu().numpy()
        else:
            rhs = itf.interface_rhs(s.layout, self.g_loads.cpu().numpy())
            u_face = self.isolver.solve(rhs)
            ub = torch.tensor(itf.box_face_values(s.layout, u_face, g_dir.cpu().numpy()), device=s.device)
        ui = torch.empty(nbox, i.n_i, dtype=torch.float64, device=s.device)
        for c0, nb in self._chunks():
            sl = slice(c0, c0 + nb)
            A, perm, dinv = self._factors(c0, nb, b)
            plan.hps_leaf_interior_solve(nb, A, perm, dinv, b[sl], self.anorm[sl],
                                         f[sl].contiguous() if f is not None else None, ub[sl].contiguous(), ui[sl],
                                         self.INTERIOR_STEPS, None, B["ws"])
        self.b = b
        self.u_i = ui
        return ui, u_face

    def gradient(self, w_i: torch.Tensor) -> torch.Tensor:
        """dJ/db at interior nodes for dJ/du_i = w_i (both [nbox, n_i])."""
        s, plan, nbox, i = self.s, self.s.plan, self.s.nbox, self.s.info
        w_i = w_i.contiguous().to(torch.float64)
        dev = s.device
        yb = torch.empty(nbox, i.n_b, dtype=torch.float64, device=dev)
        z = torch.empty(self.chunk, i.n_i, dtype=torch.float64, device=dev)
        for c0, nb in self._chunks():
            sl = slice(c0, c0 + nb)
            A, perm, dinv = self._factors(c0, nb, self.b)
            plan.hps_leaf_adjoint_solve(nb, A, perm, dinv, self.b[sl], w_i[sl], None, z, yb[sl], self.bufs["ws"])
        if isinstance(self.isolver, NestedDissection):
            lam = self.isolver.solve(yb, trans=True)
            lam_b = self.isolver.face_values(lam, torch.zeros(nbox, i.n_b, dtype=torch.float64, device=dev))
        else:
            y_face = itf.interface_rhs(s.layout, yb.cpu().numpy())
            lam_face = self.isolver.solve(y_face, trans="T")
            lam_b = torch.tensor(itf.box_face_values(s.layout, lam_face, np.zeros((nbox, i.n_b))), device=dev)
        lam_i = torch.empty(nbox, i.n_i, dtype=torch.float64, device=dev)
        for c0, nb in self._chunks():
            sl = slice(c0, c0 + nb)
            A, perm, dinv = self._factors(c0, nb, self.b)
            plan.hps_leaf_adjoint_solve(nb, A, perm, dinv, self.b[sl], w_i[sl], lam_b[sl].contiguous(), lam_i[sl],
                                        None, self.bufs["ws"])
        grad = torch.empty(nbox, i.n_i, dtype=torch.float64, device=dev)
        plan.hps_leaf_adjoint_grad(nbox, lam_i, self.u_i, grad)
        return grad


class HPSSolve(torch.autograd.Function):
    """u_i = two-level solution for coefficient b (interior nodes); differentiable in b.

    forward(b, solver, f, g_dir, opts=None): opts is an optional dict of AdjointSolve
    arguments (hbm_budget, resident, chunk)."""

    @staticmethod
    def forward(ctx, b, solver, f, g_dir, opts=None):
        fwd = AdjointSolve(solver, **(opts or {}))
        ui, _ = fwd.forward(b, f, g_dir)
        ctx.fwd = fwd
        return ui.clone()

    @staticmethod
    def backward(ctx, grad_u):
        return ctx.fwd.gradient(grad_u), None, None, None, None
