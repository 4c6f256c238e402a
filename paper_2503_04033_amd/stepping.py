"""Crank-Nicolson time stepping with one build (paper Sec. 4.4).

For u_t = nu Lap u + kappa^2 b(x) u on the box grid with u = 0 on the boundary, the step
(I - dt/2 M) u^{n+1} = (I + dt/2 M) u^n, M = nu Lap + kappa^2 b, multiplied by 2/(nu dt),
is the elliptic problem

    A u^{n+1} = c u^n - A u^n,   A = -Lap - b_e (wavenumber 1),
    b_e = kappa^2 b / nu - 2/(nu dt),   c = 4/(nu dt).

The operator is the same every step, so the leaf factorizations and the interface
factorization are made once (the paper's point: the build stage is skipped after the
first step).  Each step then runs, on the GPU:
  f      = c u_i - A_ii u_i - A_ib u_b           (hps_leaf_cn_rhs)
  g      = -A_bi A_ii^{-1} f per box             (hps_leaf_interior_solve with u_b = 0,
                                                  then hps_leaf_flux)
  u_F    = T^{-1} (sum over the boxes of g)      (nested-dissection solve on the GPU)
  u_i    = A_ii^{-1} (f - A_ib u_b)              (hps_leaf_interior_solve, FP64 refinement;
                                                  FP32 factors add the solve stage's outer
                                                  refinement of u_F)
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .nested import NestedDissection
from .solver import TwoLevelSolver


class CrankNicolson:
    """States u_i [nbox, n_i] and u_b [nbox, n_b] on the device, advanced by step()."""

    def __init__(self, pp, precision: str = "fp64", device="cuda", refine: Optional[int] = None,
                 chunk: Optional[int] = None):
        self.pp = pp
        self.c = 4.0 / (pp.nu * pp.dt)
        s = TwoLevelSolver(pp.nboxes, pp.lo, pp.hi, pp.p, 1.0, precision=precision, keep=True,
                           keep_what="factors", interface="gpu", device=device, refine=refine, chunk=chunk)
        if not NestedDissection.supported(s.layout):
            raise ValueError("the interface fronts of this grid exceed the GPU factorization's size limit")
        self.s = s
        xi, xb = s.nodes()
        xi_h, xb_h = xi.cpu().numpy(), xb.cpu().numpy()
        nu, dt, k2 = pp.nu, pp.dt, pp.kappa ** 2
        self.b_e = torch.tensor(k2 * pp.b(xi_h) / nu - 2.0 / (nu * dt), device=s.device).contiguous()
        self.g_dir = torch.zeros(s.nbox, s.info.n_b, dtype=torch.float64, device=s.device)
        self.zero_b = torch.zeros_like(self.g_dir)
        self.br = s.build(self.b_e, None, self.g_dir)
        self.nd = s.interface_solver(self.br)
        self.u_i = torch.tensor(pp.u0(xi_h), device=s.device).contiguous()
        ub = np.where(s.bmask, 0.0, pp.u0(xb_h))
        self.u_b = torch.tensor(ub, device=s.device).contiguous()
        self.f = torch.empty_like(self.u_i)
        self.nsteps = 0

    def step(self) -> None:
        s = self.s
        s.plan.hps_leaf_cn_rhs(s.nbox, self.b_e, self.c, self.u_i, self.u_b, self.f)
        _, flux = s._interiors(self.br, self.zero_b, self.b_e, self.f, want_flux=True)
        _, ub, ui = s.solve_device(self.br, self.g_dir, self.nd, self.b_e, self.f, loads=flux, sign=-1)
        self.u_i, self.u_b = ui, ub
        self.nsteps += 1

    def face_solution(self) -> torch.Tensor:
        """u on the internal faces, face-major [nface * m^2] (the interface unknowns' order)."""
        lay = self.s.layout
        mm = lay.m * lay.m
        out = torch.empty(lay.nface * mm, dtype=torch.float64, device=self.s.device)
        ub = self.u_b.view(self.s.nbox, 6, mm)
        for a in range(1, 6, 2):  # each internal face once, from its lower box
            F = lay.box_faces[:, a]
            ok = np.nonzero(F >= 0)[0]
            if ok.size:
                out.view(-1, mm)[torch.tensor(F[ok], device=out.device)] = ub[torch.tensor(ok, device=out.device), a]
        return out
