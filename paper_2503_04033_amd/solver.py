"""Two-level HPS driver over the leaf-box C ABI (paper Alg. 1 build stage, Alg. 2 solve stage).

Per chunk of boxes the GPU runs: hps_leaf_operators (a1) -> hps_leaf_factor (a2)
-> hps_leaf_dtn (a3 solves + refinement, a4 DtN/load scatter into the BSR
interface matrix).  The host then reduces the duplicate diagonal blocks on the
GPU (hps_interface_reduce), copies T and the loads, and factors the sparse
interface matrix (p-independent, off the hot path).  The solve stage sums
loads, solves for the interface values and fills in the interiors on the GPU.

What stays in HBM between the two stages is decided by an HBM budget (default:
90 % of the free device memory when the solver is made).  Without the outer
refinement (refine = 0) the interiors are one GEMV per box with X
(hps_leaf_reconstruct), so X is the per-box data worth keeping; with it the
interiors come from the box factors (hps_leaf_interior_solve), so the factors
are.  `keep` = None keeps them when they fit next to the interface matrix and
one chunk of working buffers, True insists (error if they do not fit), False
never keeps them: every chunk's operators and factors are then computed again
in the solve stage, as the paper does for problems whose local operators do not
fit in memory (Sec. 3.2).

Outer refinement of the solve stage (`refine` rounds; default 1 for FP32_IR,
0 for FP64): the interface system amplifies the rounding left in the DtN maps
(FP32_IR maps agree with FP64 to ~1e-13, and at kappa h ~ 10 the amplification
reaches ~5e5).  Each round recomputes every interior from the box factors in FP64
(hps_leaf_interior_solve), takes the flux mismatch on the interfaces as the exact
residual of T_FF u_F = rhs (hps_leaf_flux), and corrects u_F with the existing
interface factorization; each round shrinks the error by that amplification times
the maps' relative error.  The final interiors come from the factors as well.

Boxes whose FP32 factors are not good enough.  In the build, a box whose
refinement ends above ir_tol (ir_iters < 0) is factored and solved again with an
FP64 plan before the interface matrix is reduced; its ir_iters stays negative and
its id is listed in BuildResult.extra["fp64_fallback"].  In the solve stage those
boxes, and any box whose interior solve ends with a backward error above
`interior_tol`, get their interiors from FP64 factors; a box still above
`interior_tol` then raises RuntimeError.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

from . import interface as itf
from .leaf import LeafPlan, hps_interface_reduce
from .nested import NestedDissection


def _box_origins(nboxes, lo, h) -> np.ndarray:
    n1, n2, n3 = nboxes
    t = np.arange(n1 * n2 * n3)
    bx, rem = t % n1, t // n1
    by, bz = rem % n2, rem // n2
    return np.stack([lo[0] + bx * h[0], lo[1] + by * h[1], lo[2] + bz * h[2]], axis=1).astype(np.float64)


def chunk_bytes_per_box(info) -> int:
    """Working buffers of one box in a chunk: A/LU, perm, dinv, X, workspace, scalars."""
    return info.a_bytes + info.perm_bytes + info.dinv_bytes + info.x_bytes + info.ws_bytes + 64


def factor_bytes_per_box(info) -> int:
    return info.a_bytes + info.perm_bytes + info.dinv_bytes + 8


def fp64_redo(plan64: LeafPlan, ids: list, b, f, g_dir, slot_map, T_vals, g_loads, berr, chunk: int, device,
              keep_x: Optional[Callable] = None) -> None:
    """Boxes `ids` (an FP32_IR run left them above ir_tol) factored and solved again with
    the FP64 plan plan64: their DtN blocks are written into their slots of T_vals (the
    shared diagonal blocks need hps_interface_reduce afterwards), their loads and backward
    errors into g_loads and berr; keep_x(idx, X_rows) receives their X if given."""
    i = plan64.info
    xs = i.n_pad * i.ldx
    C = min(chunk, len(ids))
    bufs = plan64.alloc(C, device)
    for k0 in range(0, len(ids), C):
        part = ids[k0:k0 + C]
        nb = len(part)
        idx = torch.tensor(part, dtype=torch.long, device=device)
        bb = b[idx].contiguous()
        ff = f[idx].contiguous() if f is not None else None
        gl = torch.empty(nb, i.n_b, dtype=torch.float64, device=device)
        plan64.hps_leaf_operators(nb, bb, bufs["A"], bufs["anorm"])
        plan64.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
        plan64.hps_leaf_dtn(nb, bufs["A"], bufs["perm"], bufs["dinv"], bb, bufs["anorm"], ff,
                            g_dir[idx].contiguous(), slot_map[idx].contiguous(), T_vals, gl, bufs["X"],
                            bufs["ir_iters"], bufs["berr"], bufs["ws"])
        g_loads[idx] = gl
        if berr is not None:
            berr[idx] = bufs["berr"][:nb]
        if keep_x is not None:
            keep_x(idx, bufs["X"][:nb * xs].view(nb, xs))


@dataclass
class BuildResult:
    T_vals: torch.Tensor            # BSR blocks (+ extra diagonal slots), device
    g_loads: torch.Tensor           # [nbox, n_b] lifted loads, device
    info: torch.Tensor              # [nbox] LU info
    ir_iters: torch.Tensor
    berr: torch.Tensor
    anorm: torch.Tensor             # [nbox] |A_ii|_inf
    X: Optional[torch.Tensor] = None  # [nbox * n_pad * ldx] when kept
    factors: Optional[dict] = None    # LU, perm, dinv of every box when kept
    extra: dict = field(default_factory=dict)


class TwoLevelSolver:
    """Solve -Lap u - kappa^2 b u = f on a box grid with Dirichlet data g."""

    MAX_CHUNK = 1024

    def __init__(self, nboxes, lo, hi, p: int, kappa: float, precision: str = "fp64", ir_max_iter: int = 3,
                 ir_tol: Optional[float] = None, chunk: Optional[int] = None, keep: Optional[bool] = None, device="cuda",
                 refine: Optional[int] = None, refine_steps: Optional[int] = None, tuning: Optional[dict] = None,
                 hbm_budget: Optional[float] = None, interior_tol: float = 1e-12, interface: str = "auto",
                 keep_what: Optional[str] = None):
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
        self.refine = (1 if precision == "fp32_ir" else 0) if refine is None else int(refine)
        # FP64 refinement steps of the interior solves: FP32 factors gain ~6 digits a step (2
        # reach FP64 rounding); FP64 factors are at FP64 rounding already
        self.refine_steps = (2 if precision == "fp32_ir" else 0) if refine_steps is None else int(refine_steps)
        self.interior_tol = float(interior_tol)
        self.precision = precision
        if interface not in ("auto", "gpu", "host"):
            raise ValueError("interface must be 'auto', 'gpu' or 'host'")
        self.interface = interface
        if keep_what not in (None, "X", "factors"):
            raise ValueError("keep_what must be None, 'X' or 'factors'")
        self.keep_what = keep_what or ("factors" if self.refine > 0 else "X")
        self._plan64 = None
        self._plan_memory(chunk, keep, hbm_budget)
        self.origins = torch.tensor(_box_origins(self.nboxes, self.lo, self.h), device=self.device)
        self.slot_map = torch.tensor(self.layout.slot_map, device=self.device)
        self.bmask = itf.boundary_mask(self.layout)

    @classmethod
    def for_problem(cls, prob, **kw) -> "TwoLevelSolver":
        return cls(prob.nboxes, prob.lo, prob.hi, prob.p, prob.kappa, **kw)

    # ---- memory plan ------------------------------------------------------------
    def _plan_memory(self, chunk, keep, hbm_budget):
        """Chunk size and what the solve stage finds resident, within hbm_budget bytes."""
        i = self.info
        if hbm_budget is None:
            free = torch.cuda.mem_get_info(self.device)[0] if self.device.type == "cuda" else 0
            hbm_budget = 0.9 * free
        self.hbm_budget = float(hbm_budget)
        mm = i.m * i.m
        # interface matrix, loads and per-box scalars, and the host-facing copies made on the device
        resident = 8 * (self.layout.nslot_total * mm * mm + 1) + 8 * self.nbox * (3 * i.n_b + 4)
        per_box_keep = factor_bytes_per_box(i) if self.keep_what == "factors" else i.x_bytes
        keep_total = per_box_keep * self.nbox
        per_chunk_box = chunk_bytes_per_box(i)
        fits_keep = resident + keep_total + per_chunk_box <= self.hbm_budget
        if keep is None:
            keep = fits_keep
        elif keep and not fits_keep:
            raise ValueError(f"keeping the per-box data needs {(resident + keep_total) / 1e9:.1f} GB plus a "
                             f"chunk; the HBM budget is {self.hbm_budget / 1e9:.1f} GB")
        self.keep = bool(keep)
        avail = self.hbm_budget - resident - (keep_total if self.keep else 0)
        fit = int(avail // per_chunk_box)
        if fit < 1:
            raise ValueError(f"one box of working buffers ({per_chunk_box / 1e6:.1f} MB) does not fit the HBM "
                             f"budget of {self.hbm_budget / 1e9:.2f} GB next to the interface matrix")
        if chunk:
            if int(chunk) > fit:
                raise ValueError(f"chunk {chunk} exceeds the {fit} boxes that fit the HBM budget")
            self.chunk = int(chunk)
        else:
            self.chunk = min(self.nbox, fit, self.MAX_CHUNK)
        self.keep_X = self.keep and self.keep_what == "X"
        self.keep_factors = self.keep and self.keep_what == "factors"

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
        anorm = torch.empty(nbox, dtype=torch.float64, device=self.device)
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
            plan.hps_leaf_operators(nb, bb, A, anorm[sl])
            plan.hps_leaf_factor(nb, A, perm, dinv, info[sl])
            plan.hps_leaf_dtn(nb, A, perm, dinv, bb, anorm[sl], ff,
                              g_dir[sl].contiguous(), self.slot_map[sl].contiguous(), T_vals, g_loads[sl], X,
                              iters[sl], berr[sl], bufs["ws"])
        del bufs
        redo = self._unconverged(iters)
        if redo:
            self._redo_fp64(redo, b, f, g_dir, T_vals, g_loads, berr, X_all)
        triples = torch.tensor(self.layout.reduce_triples, device=self.device)
        if triples.shape[0]:
            hps_interface_reduce(triples, mm * mm, T_vals)
        return BuildResult(T_vals=T_vals, g_loads=g_loads, info=info, ir_iters=iters, berr=berr, anorm=anorm,
                           X=X_all, factors=factors, extra={"fp64_fallback": redo})

    # ---- boxes whose FP64 refinement did not converge ----------------------------
    def _unconverged(self, iters: torch.Tensor, offset: int = 0) -> list:
        if self.precision != "fp32_ir":
            return []
        return [offset + int(t) for t in torch.nonzero(iters < 0).flatten().cpu().tolist()]

    def _fp64_plan(self) -> LeafPlan:
        if self._plan64 is None:
            self._plan64 = LeafPlan(self.p, self.h, self.kappa, "fp64")
        return self._plan64

    def _redo_fp64(self, ids: list, b, f, g_dir, T_vals, g_loads, berr, X_all=None, X_chunk=None, c0: int = 0):
        """Factor and solve boxes `ids` again in FP64, overwriting their T blocks, loads,
        backward errors and X (in X_all, or in X_chunk whose first box is c0)."""
        i = self.info
        xs = i.n_pad * i.ldx

        def keep_x(idx, Xn):
            if X_all is not None:
                X_all.view(self.nbox, xs)[idx] = Xn
            elif X_chunk is not None:
                X_chunk.view(-1, xs)[idx - c0] = Xn

        fp64_redo(self._fp64_plan(), ids, b, f, g_dir, self.slot_map, T_vals, g_loads, berr, self.chunk,
                  self.device, keep_x)

    # ---- interface factorization (Alg. 1 step 3) ---------------------------------
    def interface_solver(self, br: BuildResult):
        """Factor the interface matrix: on the GPU by nested dissection with dense fronts
        (NestedDissection) when interface is 'gpu', or 'auto' and its fronts fit the free
        device memory and the kernels' size limit; else on the host (InterfaceSolver)."""
        return self.factor_interface(br.T_vals)

    def factor_interface(self, T_vals: torch.Tensor):
        """interface_solver() for interface blocks T_vals (the layout's slots)."""
        use_gpu = self.interface == "gpu"
        if self.interface == "auto" and self.device.type == "cuda" and self.layout.nface > 0:
            free = torch.cuda.mem_get_info(self.device)[0]
            use_gpu = (NestedDissection.supported(self.layout) and
                       NestedDissection.estimate_bytes(self.layout) < 0.8 * free)
        if use_gpu:
            nd = NestedDissection(self.layout, self.device)
            nd.factor(T_vals)
            return nd
        return itf.InterfaceSolver(self.layout, T_vals.cpu().numpy())

    # ---- solve stage (Alg. 2) ---------------------------------------------------
    def solve(self, br: BuildResult, g_dir: torch.Tensor, isolver=None,
              b: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None):
        """Return (u_face, u_b [nbox, n_b], u_i [nbox, n_i], interface solver).

        With X kept from the build the interiors are one GEMV per box.  Otherwise
        the interiors come from the box factors (kept, or computed again per chunk),
        which needs b and f again.
        """
        if isolver is None:
            isolver = self.interface_solver(br)
        if isinstance(isolver, NestedDissection):
            return self._solve_gpu(br, g_dir, isolver, b, f)
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
        if br.X is not None:
            ui = torch.empty(self.nbox, self.info.n_i, dtype=torch.float64, device=self.device)
            self.plan.hps_leaf_reconstruct(self.nbox, br.X, ub_d, ui)
            return u_face, ub, ui, isolver
        if b is None:
            raise ValueError("recompute mode needs b (and f) again")
        ui, _ = self._interiors(br, ub_d, b, f, want_flux=False)
        return u_face, ub, ui, isolver

    def _solve_gpu(self, br: BuildResult, g_dir: torch.Tensor, nd: NestedDissection, b, f):
        u, ub_d, ui = self.solve_device(br, g_dir, nd, b, f)
        return u.cpu().numpy(), ub_d.cpu().numpy(), ui, nd

    def solve_device(self, br: BuildResult, g_dir: torch.Tensor, nd: NestedDissection, b, f,
                     loads: Optional[torch.Tensor] = None, sign: int = 1):
        """The solve stage with the interface factorization on the GPU; every step stays in
        HBM (interface solve, face values, refinement, interiors).  The interface load is
        sign * loads per box ([nbox, n_b]; default the build's lifted loads).  Returns
        (u_F, u_b [nbox, n_b], u_i [nbox, n_i]) on the device."""
        u = nd.solve(br.g_loads if loads is None else loads, sign)
        ub_d = nd.face_values(u, g_dir)
        self.refine_history = []
        if self.refine > 0 and self.layout.nface > 0:
            if b is None:
                raise ValueError("the outer refinement needs b (and f) again")
            for _ in range(self.refine):
                _, flux = self._interiors(br, ub_d, b, f, want_flux=True)
                du = nd.solve(flux)  # T du = rhs(flux); the correction is -du
                self.refine_history.append(float(torch.linalg.norm(du) / max(float(torch.linalg.norm(u)), 1e-300)))
                nd.axpy(u, du, -1)
                ub_d = nd.face_values(u, g_dir)
            ui, _ = self._interiors(br, ub_d, b, f, want_flux=False)
        elif br.X is not None:
            ui = torch.empty(self.nbox, self.info.n_i, dtype=torch.float64, device=self.device)
            self.plan.hps_leaf_reconstruct(self.nbox, br.X, ub_d, ui)
        else:
            if b is None:
                raise ValueError("recompute mode needs b (and f) again")
            ui, _ = self._interiors(br, ub_d, b, f, want_flux=False)
        return u, ub_d, ui

    def _interiors(self, br: BuildResult, ub_d: torch.Tensor, b, f, want_flux: bool):
        """u_i = A_ii^{-1} (f_i - A_ib u_b) of every box from its factors, refined in FP64
        (hps_leaf_interior_solve), and optionally the outward face fluxes (hps_leaf_flux).
        Factors come from the build when kept, else each chunk is factored again.  Boxes of
        the build's FP64 fallback, and boxes whose interior backward error ends above
        interior_tol, are solved again with FP64 factors."""
        i, plan, nbox = self.info, self.plan, self.nbox
        ui = torch.empty(nbox, i.n_i, dtype=torch.float64, device=self.device)
        berr = torch.empty(nbox, dtype=torch.float64, device=self.device)
        C = min(self.chunk, nbox)
        bufs = plan.alloc(C, self.device) if br.factors is None else None
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
                ws = self._interior_ws(nb)
            else:
                A, perm, dinv, ws = bufs["A"], bufs["perm"], bufs["dinv"], bufs["ws"]
                plan.hps_leaf_operators(nb, bb, A, bufs["anorm"])
                plan.hps_leaf_factor(nb, A, perm, dinv, bufs["info"])
            plan.hps_leaf_interior_solve(nb, A, perm, dinv, bb, br.anorm[sl], ff, ub_d[sl].contiguous(), ui[sl],
                                         self.refine_steps, berr[sl], ws)
        del bufs
        redo = set(br.extra.get("fp64_fallback", []))
        if self.precision == "fp32_ir":
            redo |= set(torch.nonzero(~(berr <= self.interior_tol)).flatten().cpu().tolist())
        redo = sorted(redo)
        if redo:
            self._interiors_fp64(redo, ub_d, b, f, ui, berr)
        worst = float(berr.max()) if nbox else 0.0
        if not worst <= self.interior_tol:
            bad = torch.nonzero(~(berr <= self.interior_tol)).flatten().cpu().tolist()
            raise RuntimeError(f"interior solves of boxes {bad[:16]} end with backward error up to {worst:.2e} "
                               f"(> {self.interior_tol:.1e}) even with FP64 factors")
        br.extra["interior_berr_max"] = worst
        br.extra["interior_fp64"] = redo
        flux = None
        if want_flux:
            flux = torch.empty(nbox, i.n_b, dtype=torch.float64, device=self.device)
            plan.hps_leaf_flux(nbox, ui, ub_d, flux)
        return ui, flux

    def _interior_ws(self, nb: int) -> torch.Tensor:
        """Workspace of an interior solve of nb boxes (one vector and three scalars per box)."""
        return torch.empty(8 * nb * (self.info.n_i + 3), dtype=torch.uint8, device=self.device)

    def _interiors_fp64(self, ids: list, ub_d, b, f, ui, berr):
        """Interiors of boxes `ids` from FP64 factors (written into ui and berr)."""
        plan, i = self._fp64_plan(), self.info
        C = min(self.chunk, len(ids))
        bufs = plan.alloc(C, self.device)
        for k0 in range(0, len(ids), C):
            idx = torch.tensor(ids[k0:k0 + C], dtype=torch.long, device=self.device)
            nb = idx.numel()
            bb = b[idx].contiguous()
            ff = f[idx].contiguous() if f is not None else None
            u = torch.empty(nb, i.n_i, dtype=torch.float64, device=self.device)
            e = torch.empty(nb, dtype=torch.float64, device=self.device)
            plan.hps_leaf_operators(nb, bb, bufs["A"], bufs["anorm"])
            plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
            plan.hps_leaf_interior_solve(nb, bufs["A"], bufs["perm"], bufs["dinv"], bb, bufs["anorm"], ff,
                                         ub_d[idx].contiguous(), u, 1, e, bufs["ws"])
            ui[idx] = u
            berr[idx] = e

    def solve_problem(self, prob):
        bv, fv, gv, xi, xb = self.sample(prob.b, prob.f, prob.g)
        br = self.build(bv, fv, gv)
        u_face, ub, ui, isolver = self.solve(br, gv, b=bv, f=fv)
        return {"build": br, "u_face": u_face, "u_b": ub, "u_i": ui, "xi": xi, "xb": xb, "b": bv, "f": fv,
                "g_dir": gv, "isolver": isolver, "refine_history": list(self.refine_history)}
