"""Two-level HPS driver over the leaf-box C ABI (paper Alg. 1 build stage, Alg. 2 solve stage).

Per chunk of boxes the GPU runs: hps_leaf_operators (a1) -> hps_leaf_factor (a2)
-> hps_leaf_dtn (a3 solves + refinement, a4 DtN/load scatter into the BSR
interface matrix).  The host then reduces the duplicate diagonal blocks on the
GPU (hps_interface_reduce), copies T and the loads, and factors the sparse
interface matrix (p-independent, off the hot path).  The solve stage sums
loads, solves for the interface values and reconstructs the interiors on the
GPU (hps_leaf_reconstruct, a5).  X (the interior solution operator and load
response) is kept in HBM per box when `keep_X` is set; otherwise the chunk is
recomputed in the solve stage, as the paper does for large problems.

Outer refinement of the solve stage (`refine` rounds; default 1 for FP32_IR,
0 for FP64): the interface system amplifies the rounding left in the DtN maps
(FP32_IR maps agree with FP64 to ~1e-13, and at kappa h ~ 10 the amplification
reaches ~5e5).  Each round recomputes every interior from the box factors in FP64
(hps_leaf_interior_solve), takes the flux mismatch on the interfaces as the exact
residual of T_FF u_F = rhs (hps_leaf_flux), and corrects u_F with the existing
interface factorization; each round shrinks the error by that amplification times
the maps' relative error.  The final interiors come from the factors as well.

FP32_IR plans: a box whose refinement ends above ir_tol (ir_iters < 0) is
factored and solved again with an FP64 plan before the interface matrix is
reduced; its ir_iters stays negative and its id is listed in
BuildResult.extra["fp64_fallback"].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

from . import interface as itf
from .leaf import LeafPlan, hps_interface_reduce


def _box_origins(nboxes, lo, h) -> np.ndarray:
    n1, n2, n3 = nboxes
    t = np.arange(n1 * n2 * n3)
    bx, rem = t % n1, t // n1
    by, bz = rem % n2, rem // n2
    return np.stack([lo[0] + bx * h[0], lo[1] + by * h[1], lo[2] + bz * h[2]], axis=1).astype(np.float64)


@dataclass
class BuildResult:
    T_vals: torch.Tensor            # BSR blocks (+ extra diagonal slots), device
    g_loads: torch.Tensor           # [nbox, n_b] lifted loads, device
    info: torch.Tensor              # [nbox] LU info
    ir_iters: torch.Tensor
    berr: torch.Tensor
    X: Optional[torch.Tensor] = None  # [nbox * n_pad * ldx] when kept
    factors: Optional[dict] = None    # LU, perm, dinv of every box when kept
    extra: dict = field(default_factory=dict)


class TwoLevelSolver:
    """Solve -Lap u - kappa^2 b u = f on a box grid with Dirichlet data g."""

    def __init__(self, nboxes, lo, hi, p: int, kappa: float, precision: str = "fp64", ir_max_iter: int = 3,
                 ir_tol: float = 1e-12, chunk: Optional[int] = None, keep_X: bool = True, device="cuda",
                 refine: Optional[int] = None, refine_steps: int = 2, tuning: Optional[dict] = None):
        self.nboxes = tuple(int(v) for v in nboxes)
        self.nbox = int(np.prod(self.nboxes))
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.h = tuple((self.hi[a] - self.lo[a]) / self.nboxes[a] for a in range(3))
        self.p, self.kappa = int(p), float(kappa)
        self.device = torch.device(device)
        self.plan = LeafPlan(p, self.h, kappa, precision, ir_max_iter, ir_tol)
        for k, v in (tuning or {}).items():  # scheduling knobs (batch.autotune's choices)
            self.plan.hps_plan_set_tuning(k, v)
        self.info = self.plan.info
        self.layout = itf.build_layout(self.nboxes, self.info.m)
        self.chunk = int(chunk) if chunk else self.nbox
        self.keep_X = keep_X
        self.refine = (1 if precision == "fp32_ir" else 0) if refine is None else int(refine)
        self.refine_steps = int(refine_steps)
        self.keep_factors = keep_X and self.refine > 0
        self.precision = precision
        self._plan64 = None
        self.origins = torch.tensor(_box_origins(self.nboxes, self.lo, self.h), device=self.device)
        self.slot_map = torch.tensor(self.layout.slot_map, device=self.device)
        self.bmask = itf.boundary_mask(self.layout)

    @classmethod
    def for_problem(cls, prob, **kw) -> "TwoLevelSolver":
        return cls(prob.nboxes, prob.lo, prob.hi, prob.p, prob.kappa, **kw)

    # ---- problem data at the collocation nodes --------------------------------
    def nodes(self):
        i = self.info
        xi = torch.empty(self.nbox * i.n_i * 3, dtype=torch.float64, device=self.device)
        xb = torch.empty(self.nbox * i.n_b * 3, dtype=torch.float64, device=self.device)
        self.plan.hps_leaf_nodes(self.nbox, self.origins, xi, xb)
        return xi.view(self.nbox, i.n_i, 3), xb.view(self.nbox, i.n_b, 3)

    def sample(self, b: Callable, f: Optional[Callable], g: Callable):
        """Evaluate b, f at interior nodes and g at boundary-face nodes; device tensors."""
        xi, xb = self.nodes()
        xi_h, xb_h = xi.cpu().numpy(), xb.cpu().numpy()
        bv = torch.tensor(b(xi_h), dtype=torch.float64, device=self.device).contiguous()
        fv = torch.tensor(f(xi_h), dtype=torch.float64, device=self.device).contiguous() if f else None
        gd = np.where(self.bmask, g(xb_h), 0.0)
        gv = torch.tensor(gd, dtype=torch.float64, device=self.device).contiguous()
        return bv, fv, gv, xi_h, xb_h

    # ---- build stage (Alg. 1) ---------------------------------------------------
    def build(self, b: torch.Tensor, f: Optional[torch.Tensor], g_dir: torch.Tensor) -> BuildResult:
        i, plan, nbox = self.info, self.plan, self.nbox
        mm = i.m * i.m
        # one spare element keeps the pointer valid when the grid has no internal face
        T_vals = torch.zeros(self.layout.nslot_total * mm * mm + 1, dtype=torch.float64, device=self.device)
        g_loads = torch.empty(nbox, i.n_b, dtype=torch.float64, device=self.device)
        info = torch.empty(nbox, dtype=torch.int32, device=self.device)
        iters = torch.empty(nbox, dtype=torch.int32, device=self.device)
        berr = torch.empty(nbox, dtype=torch.float64, device=self.device)
        X_all = torch.empty(nbox * i.n_pad * i.ldx, dtype=torch.float64, device=self.device) if self.keep_X else None
        C = min(self.chunk, nbox)
        bufs = plan.alloc(C, self.device)
        xs = i.n_pad * i.ldx
        a_el, d_el = i.a_bytes // i.elem_bytes, i.dinv_bytes // i.elem_bytes
        factors = None
        if self.keep_factors:
            factors = {"LU": torch.empty(nbox * a_el, dtype=plan.elem, device=self.device),
                       "perm": torch.empty(nbox * i.n_pad, dtype=torch.int32, device=self.device),
                       "dinv": torch.empty(nbox * d_el, dtype=plan.elem, device=self.device)}
        for c0 in range(0, nbox, C):
            nb = min(C, nbox - c0)
            sl = slice(c0, c0 + nb)
            bb = b[sl].contiguous()
            ff = f[sl].contiguous() if f is not None else None
            X = X_all[c0 * xs:(c0 + nb) * xs] if X_all is not None else bufs["X"]
            A, perm, dinv = bufs["A"], bufs["perm"], bufs["dinv"]
            if factors is not None:
                A = factors["LU"][c0 * a_el:(c0 + nb) * a_el]
                perm = factors["perm"][c0 * i.n_pad:(c0 + nb) * i.n_pad]
                dinv = factors["dinv"][c0 * d_el:(c0 + nb) * d_el]
            plan.hps_leaf_operators(nb, bb, A, bufs["anorm"])
            plan.hps_leaf_factor(nb, A, perm, dinv, info[sl])
            plan.hps_leaf_dtn(nb, A, perm, dinv, bb, bufs["anorm"], ff,
                              g_dir[sl].contiguous(), self.slot_map[sl].contiguous(), T_vals, g_loads[sl], X,
                              iters[sl], berr[sl], bufs["ws"])
        redo = self._unconverged(iters)
        if redo:
            self._redo_fp64(redo, b, f, g_dir, T_vals, g_loads, berr, X_all)
        pairs = torch.tensor(self.layout.reduce_pairs, device=self.device)
        if pairs.shape[0]:
            hps_interface_reduce(pairs, mm * mm, T_vals)
        return BuildResult(T_vals=T_vals, g_loads=g_loads, info=info, ir_iters=iters, berr=berr, X=X_all,
                           factors=factors, extra={"fp64_fallback": redo})

    # ---- boxes whose FP64 refinement did not converge ----------------------------
    def _unconverged(self, iters: torch.Tensor, offset: int = 0) -> list:
        if self.precision != "fp32_ir":
            return []
        return [offset + int(t) for t in torch.nonzero(iters < 0).flatten().cpu().tolist()]

    def _redo_fp64(self, ids: list, b, f, g_dir, T_vals, g_loads, berr, X_all=None, X_chunk=None, c0: int = 0):
        """Factor and solve boxes `ids` again in FP64, overwriting their T blocks, loads,
        backward errors and X (in X_all, or in X_chunk whose first box is c0)."""
        if self._plan64 is None:
            self._plan64 = LeafPlan(self.p, self.h, self.kappa, "fp64")
        plan, i = self._plan64, self.info
        xs = i.n_pad * i.ldx
        C = min(self.chunk, len(ids))
        bufs = plan.alloc(C, self.device)
        for k0 in range(0, len(ids), C):
            part = ids[k0:k0 + C]
            nb = len(part)
            idx = torch.tensor(part, dtype=torch.long, device=self.device)
            bb = b[idx].contiguous()
            ff = f[idx].contiguous() if f is not None else None
            gl = torch.empty(nb, i.n_b, dtype=torch.float64, device=self.device)
            plan.hps_leaf_operators(nb, bb, bufs["A"], bufs["anorm"])
            plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
            plan.hps_leaf_dtn(nb, bufs["A"], bufs["perm"], bufs["dinv"], bb, bufs["anorm"], ff,
                              g_dir[idx].contiguous(), self.slot_map[idx].contiguous(), T_vals, gl, bufs["X"],
                              bufs["ir_iters"], bufs["berr"], bufs["ws"])
            g_loads[idx] = gl
            if berr is not None:
                berr[idx] = bufs["berr"][:nb]
            Xn = bufs["X"][:nb * xs].view(nb, xs)
            if X_all is not None:
                X_all.view(self.nbox, xs)[idx] = Xn
            elif X_chunk is not None:
                X_chunk.view(-1, xs)[idx - c0] = Xn

    # ---- solve stage (Alg. 2) ---------------------------------------------------
    def solve(self, br: BuildResult, g_dir: torch.Tensor, isolver: Optional[itf.InterfaceSolver] = None,
              b: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None):
        """Return (u_face, u_b [nbox, n_b], u_i [nbox, n_i], interface solver).

        With X kept from the build the interiors are one GEMV per box.  Otherwise
        (keep_X=False) every chunk's operators, factors and X are recomputed here,
        as the paper does for problems whose local operators do not fit in
        memory (Sec. 3.2); b and f must then be passed again.
        """
        if isolver is None:
            isolver = itf.InterfaceSolver(self.layout, br.T_vals.cpu().numpy())
        rhs = itf.interface_rhs(self.layout, br.g_loads.cpu().numpy())
        u_face = isolver.solve(rhs)
        gd = g_dir.cpu().numpy()
        ub = itf.box_face_values(self.layout, u_face, gd)
        ub_d = torch.tensor(ub, device=self.device)
        self.refine_history = []
        if self.refine > 0 and u_face.size:
            if b is None:
                raise ValueError("the outer refinement needs b (and f) again")
            for _ in range(self.refine):
                _, flux = self._interiors(br, ub_d, b, f, want_flux=True)
                du = isolver.solve(itf.interface_rhs(self.layout, -flux.cpu().numpy()))
                self.refine_history.append(float(np.linalg.norm(du) / max(np.linalg.norm(u_face), 1e-300)))
                u_face = u_face + du
                ub = itf.box_face_values(self.layout, u_face, gd)
                ub_d = torch.tensor(ub, device=self.device)
            ui, _ = self._interiors(br, ub_d, b, f, want_flux=False)
            return u_face, ub, ui, isolver
        ui = torch.empty(self.nbox, self.info.n_i, dtype=torch.float64, device=self.device)
        if br.X is not None:
            self.plan.hps_leaf_reconstruct(self.nbox, br.X, ub_d, ui)
            return u_face, ub, ui, isolver
        if b is None:
            raise ValueError("recompute mode needs b (and f) again")
        i, plan, nbox = self.info, self.plan, self.nbox
        mm = i.m * i.m
        C = min(self.chunk, nbox)
        bufs = plan.alloc(C, self.device)
        scratch_T = torch.zeros(self.layout.nslot_total * mm * mm + 1, dtype=torch.float64, device=self.device)
        scratch_g = torch.empty(C, i.n_b, dtype=torch.float64, device=self.device)
        for c0 in range(0, nbox, C):
            nb = min(C, nbox - c0)
            sl = slice(c0, c0 + nb)
            bb = b[sl].contiguous()
            ff = f[sl].contiguous() if f is not None else None
            plan.hps_leaf_operators(nb, bb, bufs["A"], bufs["anorm"])
            plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
            plan.hps_leaf_dtn(nb, bufs["A"], bufs["perm"], bufs["dinv"], bb, bufs["anorm"], ff,
                              g_dir[sl].contiguous(), self.slot_map[sl].contiguous(), scratch_T, scratch_g[:nb],
                              bufs["X"], bufs["ir_iters"], bufs["berr"], bufs["ws"])
            redo = self._unconverged(bufs["ir_iters"][:nb], c0)
            if redo:
                self._redo_fp64(redo, b, f, g_dir, scratch_T, torch.empty(self.nbox, i.n_b, dtype=torch.float64,
                                device=self.device), None, X_chunk=bufs["X"], c0=c0)
            plan.hps_leaf_reconstruct(nb, bufs["X"], ub_d[sl].contiguous(), ui[sl])
        return u_face, ub, ui, isolver

    def _interiors(self, br: BuildResult, ub_d: torch.Tensor, b, f, want_flux: bool):
        """u_i = A_ii^{-1} (f_i - A_ib u_b) of every box from its factors, refined in FP64
        (hps_leaf_interior_solve), and optionally the outward face fluxes (hps_leaf_flux).
        Factors come from the build when kept, else each chunk is factored again."""
        i, plan, nbox = self.info, self.plan, self.nbox
        ui = torch.empty(nbox, i.n_i, dtype=torch.float64, device=self.device)
        flux = torch.empty(nbox, i.n_b, dtype=torch.float64, device=self.device) if want_flux else None
        C = min(self.chunk, nbox)
        bufs = plan.alloc(C, self.device)
        a_el, d_el = i.a_bytes // i.elem_bytes, i.dinv_bytes // i.elem_bytes
        for c0 in range(0, nbox, C):
            nb = min(C, nbox - c0)
            sl = slice(c0, c0 + nb)
            bb = b[sl].contiguous()
            ff = f[sl].contiguous() if f is not None else None
            if br.factors is not None:
                A = br.factors["LU"][c0 * a_el:(c0 + nb) * a_el]
                perm = br.factors["perm"][c0 * i.n_pad:(c0 + nb) * i.n_pad]
                dinv = br.factors["dinv"][c0 * d_el:(c0 + nb) * d_el]
            else:
                A, perm, dinv = bufs["A"], bufs["perm"], bufs["dinv"]
                plan.hps_leaf_operators(nb, bb, A, bufs["anorm"])
                plan.hps_leaf_factor(nb, A, perm, dinv, bufs["info"])
            ubs = ub_d[sl].contiguous()
            plan.hps_leaf_interior_solve(nb, A, perm, dinv, bb, ff, ubs, ui[sl], self.refine_steps, bufs["ws"])
            if want_flux:
                plan.hps_leaf_flux(nb, ui[sl], ubs, flux[sl])
        return ui, flux

    def solve_problem(self, prob):
        bv, fv, gv, xi, xb = self.sample(prob.b, prob.f, prob.g)
        br = self.build(bv, fv, gv)
        u_face, ub, ui, isolver = self.solve(br, gv, b=bv, f=fv)
        return {"build": br, "u_face": u_face, "u_b": ub, "u_i": ui, "xi": xi, "xb": xb, "b": bv, "f": fv,
                "g_dir": gv, "isolver": isolver, "refine_history": list(self.refine_history)}
