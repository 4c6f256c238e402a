"""Python binding of the leaf-box C ABI (include/hps_leaf.h), same names.

Arguments are torch tensors on the GPU; every call checks dtype, device and
size and passes raw pointers plus the current HIP stream.  All computation
happens in libhps_leaf.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import HPS_FP32_IR, HPS_FP64, check


def _ptr(t: Optional[torch.Tensor], dtype=None, numel: int = 0, name: str = "") -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Info:
    m: int
    n_i: int
    n_b: int
    n_pad: int
    nrhs: int
    ldx: int
    npanel: int
    elem_bytes: int
    a_bytes: int
    perm_bytes: int
    dinv_bytes: int
    x_bytes: int
    ws_bytes: int


def default_ir_tol(p: int) -> float:
    """Backward-error tolerance of the FP64 refinement when the caller gives none.

    The forward error of X is about cond(A_ii) times the backward error, and cond(A_ii)
    grows with p (like p^4 for the spectral second derivative) and near interior
    resonances of the box.  1e-12 leaves X within ~1e-13 of FP64 at p <= 16 (one
    correction); at p = 17-20 one correction can end just under 1e-12 with X still
    ~6e-10 away, so those take 1e-13 (two corrections, X within ~3e-13)."""
    return 1e-12 if int(p) <= 16 else 1e-13


class LeafPlan:
    """Owns one hps_plan (Chebyshev tables on the device) for a box size and wavenumber."""

    def __init__(self, p: int, h, kappa: float, precision: str = "fp64", ir_max_iter: int = 3,
                 ir_tol: Optional[float] = None):
        if ir_tol is None:
            ir_tol = default_ir_tol(p)
        self.lib = _lib.load()
        d = _lib.LeafDesc()
        d.p = int(p)
        for a in range(3):
            d.h[a] = float(h[a])
        d.kappa = float(kappa)
        if precision not in ("fp64", "fp32_ir"):
            raise ValueError("precision must be 'fp64' or 'fp32_ir'")
        d.precision = HPS_FP32_IR if precision == "fp32_ir" else HPS_FP64
        d.ir_max_iter = int(ir_max_iter)
        d.ir_tol = float(ir_tol)
        self.desc = d
        self.precision = precision
        self.p, self.h, self.kappa = int(p), tuple(float(x) for x in h), float(kappa)
        handle = C.c_void_p()
        check(self.lib.hps_plan_create(C.byref(handle), C.byref(d)), "hps_plan_create")
        self.handle = handle
        pi = _lib.PlanInfo()
        check(self.lib.hps_plan_get_info(handle, C.byref(pi)), "hps_plan_get_info")
        self.info = Info(**{f: getattr(pi, f) for f, _ in pi._fields_})
        self.elem = torch.float32 if precision == "fp32_ir" else torch.float64

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.hps_plan_destroy(h)
            self.handle = None

    # ---- run-time tuning (scheduling only; results are bitwise the same) -------
    def hps_plan_set_tuning(self, key: str, value: int) -> None:
        check(self.lib.hps_plan_set_tuning(self.handle, _lib.TUNING_KEYS[key], int(value)), "hps_plan_set_tuning")

    def hps_leaf_workspace_bytes(self, call: str, nbox: int) -> int:
        v = C.c_size_t(0)
        check(self.lib.hps_leaf_workspace_bytes(self.handle, _lib.CALLS[call], int(nbox), C.byref(v)),
              "hps_leaf_workspace_bytes")
        return int(v.value)

    def hps_plan_get_tuning(self, key: str) -> int:
        v = C.c_int32(0)
        check(self.lib.hps_plan_get_tuning(self.handle, _lib.TUNING_KEYS[key], C.byref(v)), "hps_plan_get_tuning")
        return int(v.value)

    # ---- kernel timing ---------------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        check(self.lib.hps_plan_profile_enable(self.handle, 1 if on else 0), "hps_plan_profile_enable")

    def profile_read(self) -> dict:
        pr = _lib.Profile()
        check(self.lib.hps_plan_profile_read(self.handle, C.byref(pr)), "hps_plan_profile_read")
        return {name: {"launches": int(pr.launches[k]), "ms": float(pr.ms[k]), "flops": float(pr.flops[k]),
                       "exec_flops": float(pr.exec_flops[k])}
                for k, name in enumerate(_lib.PROFILE_FAMILIES)}

    # ---- allocation helpers -------------------------------------------------
    def alloc(self, nbox: int, device="cuda") -> dict:
        """Caller-owned device buffers for `nbox` boxes."""
        i = self.info
        es = i.elem_bytes
        return {
            "A": torch.empty(nbox * i.a_bytes // es, dtype=self.elem, device=device),
            "perm": torch.empty(nbox * i.n_pad, dtype=torch.int32, device=device),
            "dinv": torch.empty(nbox * i.dinv_bytes // es, dtype=self.elem, device=device),
            "info": torch.empty(nbox, dtype=torch.int32, device=device),
            "anorm": torch.empty(nbox, dtype=torch.float64, device=device),
            "X": torch.empty(nbox * i.n_pad * i.ldx, dtype=torch.float64, device=device),
            "ws": torch.empty(nbox * i.ws_bytes, dtype=torch.uint8, device=device),
            "ir_iters": torch.empty(nbox, dtype=torch.int32, device=device),
            "berr": torch.empty(nbox, dtype=torch.float64, device=device),
        }

    # ---- ABI calls ----------------------------------------------------------
    def hps_leaf_nodes(self, nbox: int, origin, xi, xb):
        i = self.info
        check(self.lib.hps_leaf_nodes(self.handle, nbox, _ptr(origin, torch.float64, 3 * nbox, "origin"),
                                      _ptr(xi, torch.float64, nbox * i.n_i * 3, "xi"),
                                      _ptr(xb, torch.float64, nbox * i.n_b * 3, "xb"), _stream()),
              "hps_leaf_nodes")

    def hps_leaf_operators(self, nbox: int, b, A, anorm):
        i = self.info
        check(self.lib.hps_leaf_operators(self.handle, nbox, _ptr(b, torch.float64, nbox * i.n_i, "b"),
                                          _ptr(A, self.elem, nbox * i.n_pad * i.n_pad, "A"),
                                          _ptr(anorm, torch.float64, nbox, "anorm"), _stream()),
              "hps_leaf_operators")

    def hps_leaf_factor(self, nbox: int, A, perm, dinv, info):
        i = self.info
        check(self.lib.hps_leaf_factor(self.handle, nbox, _ptr(A, self.elem, nbox * i.n_pad * i.n_pad, "A"),
                                       _ptr(perm, torch.int32, nbox * i.n_pad, "perm"),
                                       _ptr(dinv, self.elem, nbox * i.dinv_bytes // i.elem_bytes, "dinv"),
                                       _ptr(info, torch.int32, nbox, "info"), _stream()),
              "hps_leaf_factor")

    def hps_leaf_dtn(self, nbox: int, LU, perm, dinv, b, anorm, f, g_dir, slot_map, T_vals, g, X, ir_iters,
                     berr, ws):
        i = self.info
        check(self.lib.hps_leaf_dtn(
            self.handle, nbox, _ptr(LU, self.elem, nbox * i.n_pad * i.n_pad, "LU"),
            _ptr(perm, torch.int32, nbox * i.n_pad, "perm"),
            _ptr(dinv, self.elem, nbox * i.dinv_bytes // i.elem_bytes, "dinv"),
            _ptr(b, torch.float64, nbox * i.n_i, "b"), _ptr(anorm, torch.float64, nbox, "anorm"),
            _ptr(f, torch.float64, nbox * i.n_i, "f"), _ptr(g_dir, torch.float64, nbox * i.n_b, "g_dir"),
            _ptr(slot_map, torch.int32, nbox * 36, "slot_map"), _ptr(T_vals, torch.float64, 1, "T_vals"),
            _ptr(g, torch.float64, nbox * i.n_b, "g"), _ptr(X, torch.float64, nbox * i.n_pad * i.ldx, "X"),
            _ptr(ir_iters, torch.int32, nbox, "ir_iters"), _ptr(berr, torch.float64, nbox, "berr"),
            _ptr(ws, torch.uint8, self.hps_leaf_workspace_bytes("dtn", nbox), "ws"), _stream()), "hps_leaf_dtn")

    def hps_leaf_reconstruct(self, nbox: int, X, u_b, u_i):
        i = self.info
        check(self.lib.hps_leaf_reconstruct(self.handle, nbox, _ptr(X, torch.float64, nbox * i.n_pad * i.ldx, "X"),
                                            _ptr(u_b, torch.float64, nbox * i.n_b, "u_b"),
                                            _ptr(u_i, torch.float64, nbox * i.n_i, "u_i"), _stream()),
              "hps_leaf_reconstruct")

    def _interior_args(self, nbox, LU, perm, dinv, b, anorm, f, u_b, u_i, berr):
        i = self.info
        return (self.handle, nbox, _ptr(LU, self.elem, nbox * i.n_pad * i.n_pad, "LU"),
                _ptr(perm, torch.int32, nbox * i.n_pad, "perm"),
                _ptr(dinv, self.elem, nbox * i.dinv_bytes // i.elem_bytes, "dinv"),
                _ptr(b, torch.float64, nbox * i.n_i, "b"), _ptr(anorm, torch.float64, nbox, "anorm"),
                _ptr(f, torch.float64, nbox * i.n_i, "f"), _ptr(u_b, torch.float64, nbox * i.n_b, "u_b"),
                _ptr(u_i, torch.float64, nbox * i.n_i, "u_i"))

    def hps_leaf_interior_solve(self, nbox: int, LU, perm, dinv, b, anorm, f, u_b, u_i, steps: int, berr, ws):
        check(self.lib.hps_leaf_interior_solve(
            *self._interior_args(nbox, LU, perm, dinv, b, anorm, f, u_b, u_i, berr), int(steps),
            _ptr(berr, torch.float64, nbox, "berr"),
            _ptr(ws, torch.uint8, self.hps_leaf_workspace_bytes("interior_solve", nbox), "ws"),
            _stream()), "hps_leaf_interior_solve")

    def hps_leaf_interior_solve_noalloc(self, nbox: int, LU, perm, dinv, b, anorm, f, u_b, u_i, steps: int,
                                        berr):
        """hps_leaf_interior_solve with the library's fixed device scratch (allocates nothing)."""
        check(self.lib.hps_leaf_interior_solve_noalloc(
            *self._interior_args(nbox, LU, perm, dinv, b, anorm, f, u_b, u_i, berr), int(steps),
            _ptr(berr, torch.float64, nbox, "berr"), _stream()), "hps_leaf_interior_solve_noalloc")

    def hps_leaf_cn_rhs(self, nbox: int, b, c: float, u_i, u_b, f):
        i = self.info
        check(self.lib.hps_leaf_cn_rhs(self.handle, nbox, _ptr(b, torch.float64, nbox * i.n_i, "b"), float(c),
                                       _ptr(u_i, torch.float64, nbox * i.n_i, "u_i"),
                                       _ptr(u_b, torch.float64, nbox * i.n_b, "u_b"),
                                       _ptr(f, torch.float64, nbox * i.n_i, "f"), _stream()), "hps_leaf_cn_rhs")

    def hps_leaf_flux(self, nbox: int, u_i, u_b, flux):
        i = self.info
        check(self.lib.hps_leaf_flux(self.handle, nbox, _ptr(u_i, torch.float64, nbox * i.n_i, "u_i"),
                                     _ptr(u_b, torch.float64, nbox * i.n_b, "u_b"),
                                     _ptr(flux, torch.float64, nbox * i.n_b, "flux"), _stream()), "hps_leaf_flux")

    def hps_leaf_adjoint_solve(self, nbox: int, LU, perm, dinv, b, w_i, lam_b, z, y_b, ws):
        i = self.info
        check(self.lib.hps_leaf_adjoint_solve(
            self.handle, nbox, _ptr(LU, self.elem, nbox * i.n_pad * i.n_pad, "LU"),
            _ptr(perm, torch.int32, nbox * i.n_pad, "perm"),
            _ptr(dinv, self.elem, nbox * i.dinv_bytes // i.elem_bytes, "dinv"),
            _ptr(b, torch.float64, nbox * i.n_i, "b"), _ptr(w_i, torch.float64, nbox * i.n_i, "w_i"),
            _ptr(lam_b, torch.float64, nbox * i.n_b, "lam_b"), _ptr(z, torch.float64, nbox * i.n_i, "z"),
            _ptr(y_b, torch.float64, nbox * i.n_b, "y_b"),
            _ptr(ws, torch.uint8, self.hps_leaf_workspace_bytes("adjoint_solve", nbox), "ws"),
            _stream()), "hps_leaf_adjoint_solve")

    def hps_leaf_adjoint_grad(self, nbox: int, lam_i, u_i, grad):
        i = self.info
        check(self.lib.hps_leaf_adjoint_grad(self.handle, nbox, _ptr(lam_i, torch.float64, nbox * i.n_i, "lam_i"),
                                             _ptr(u_i, torch.float64, nbox * i.n_i, "u_i"),
                                             _ptr(grad, torch.float64, nbox * i.n_i, "grad"), _stream()),
              "hps_leaf_adjoint_grad")


def hps_interface_reduce(triples: torch.Tensor, block_elems: int, T_vals: torch.Tensor):
    """T_vals[dst] = T_vals[lo] + T_vals[hi] for the (dst, lo, hi) rows of triples [n, 3] int64."""
    lib = _lib.load()
    n = triples.shape[0] if triples is not None else 0
    check(lib.hps_interface_reduce(n, _ptr(triples, torch.int64, 3 * n, "triples"), int(block_elems),
                                   _ptr(T_vals, torch.float64, 1, "T_vals"), _stream()), "hps_interface_reduce")
