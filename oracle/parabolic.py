"""Crank-Nicolson time stepping on the global collocation system (paper Sec. 4.4).

TEST INFRASTRUCTURE ONLY (see the package header).

For u_t = M u with M u = nu Lap u + kappa^2 b u and u = 0 on the boundary, the
Crank-Nicolson step (I - dt/2 M) u^{n+1} = (I + dt/2 M) u^n is, after multiplying by
2/(nu dt), the elliptic problem

    L u^{n+1} = c u^n - L u^n,   L = -Lap - b_e,   b_e = kappa^2 b / nu - 2/(nu dt),
                                 c = 4/(nu dt),

with L of the paper's form -Lap u - kappa^2 b u (wavenumber 1, coefficient b_e), so the
same discretization and the same factorization serve every step (the paper builds once
and supplies the previous step as the body load).  Here the discrete L is the dense
global collocation system of brute.py (interior collocation rows and flux-continuity
rows on the internal faces), factored once; the flux rows carry no time derivative, so
their right-hand side stays 0 and the face values follow the interiors every step.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import brute, leaf
from .interface import face_numbering


class _Elliptic:
    """The Problem-like object brute.assemble_global reads: L with b_e, f = 0, g = 0."""

    def __init__(self, pp):
        self.p, self.nboxes, self.lo, self.hi = pp.p, pp.nboxes, pp.lo, pp.hi
        self.kappa = 1.0
        nu, dt, k2 = pp.nu, pp.dt, pp.kappa ** 2
        self.b = lambda x: k2 * pp.b(x) / nu - 2.0 / (nu * dt)
        self.f = lambda x: np.zeros(x.shape[:-1])
        self.g = lambda x: np.zeros(x.shape[:-1])
        self.nbox = pp.nbox
        self.h = pp.h
        self.box_origins = pp.box_origins


def initial_state(pp) -> np.ndarray:
    """[u_int (box-major), u_face (face-major)] of u0 at the global unknowns."""
    p, m = pp.p, pp.p - 2
    mm = m * m
    box_faces, face_boxes = face_numbering(pp.nboxes)
    org = pp.box_origins()
    ui, uf = [], np.zeros(face_boxes.shape[0] * mm)
    for t in range(pp.nbox):
        xi, xb = leaf.box_node_coords(org[t], pp.h, p)
        ui.append(pp.u0(xi))
        for a in range(1, 6, 2):  # the + faces of a box are the faces it is the lower box of
            F = box_faces[t, a]
            if F >= 0:
                uf[F * mm:(F + 1) * mm] = pp.u0(xb[a * mm:(a + 1) * mm])
    return np.concatenate([np.concatenate(ui), uf])


def crank_nicolson(pp, nsteps: int, w0=None):
    """States after 1 .. nsteps steps, each [u_int (box-major), u_face (face-major)]."""
    sysm = brute.assemble_global(_Elliptic(pp))
    lu = scipy.linalg.lu_factor(sysm.A)
    c = 4.0 / (pp.nu * pp.dt)
    w = initial_state(pp) if w0 is None else np.asarray(w0, dtype=np.float64).copy()
    n_int = sysm.n_int
    out = []
    for _ in range(nsteps):
        rhs = np.zeros_like(w)
        rhs[:n_int] = c * w[:n_int] - sysm.A[:n_int] @ w
        w = scipy.linalg.lu_solve(lu, rhs)
        out.append(w.copy())
    return out, sysm
