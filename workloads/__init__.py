"""Seeded synthetic workloads for the leaf-box reduction of the two-level HPS solver.

This module is problem data only: coefficient fields b(x), Dirichlet data g(x),
body loads f(x), exact solutions where one is known, and the seeded random
parameters behind them.  It holds none of the method's arithmetic (no nodes, no
differentiation matrices, no factorizations); the solver and the test oracle
each evaluate these callables at the collocation nodes they compute themselves.

Problem statement (paper Sec. 1, eqs. bvp and bvphelmholtz):
    -Lap u - kappa^2 b(x) u = f   in Omega,    u = g on dOmega,
with Omega = [0,1]^3 cut into n1 x n2 x n3 equal leaf boxes unless stated.

Random draws use numpy.random.default_rng(seed) in the order documented in each
constructor.  The workloads stand in for the paper's test problems (Sec. 4); no
public dataset is involved.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Tuple

import numpy as np

Array = np.ndarray
Field = Callable[[Array], Array]  # x[..., 3] -> values[...]


@dataclass
class Problem:
    """A Helmholtz boundary value problem on a box grid.

    nboxes  -- leaf boxes per axis (n1, n2, n3)
    lo, hi  -- domain corners; each leaf box has side (hi-lo)/nboxes per axis
    p       -- Chebyshev-Gauss-Lobatto nodes per axis per box
    kappa   -- wavenumber
    b, f, g -- coefficient, body load, Dirichlet data (callables on x[...,3])
    u_exact -- exact solution of the continuous problem, if known
    """

    name: str
    nboxes: Tuple[int, int, int]
    p: int
    kappa: float
    b: Field
    f: Field
    g: Field
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    u_exact: Optional[Field] = None
    params: dict = field(default_factory=dict)

    @property
    def nbox(self) -> int:
        return int(self.nboxes[0] * self.nboxes[1] * self.nboxes[2])

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple((self.hi[a] - self.lo[a]) / self.nboxes[a] for a in range(3))

    def box_origins(self) -> Array:
        """Lower corner of every box, box index t = bx + n1*(by + n2*bz)."""
        n1, n2, n3 = self.nboxes
        h = self.h
        bz, by, bx = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
        org = np.stack([self.lo[0] + bx.ravel() * h[0],
                        self.lo[1] + by.ravel() * h[1],
                        self.lo[2] + bz.ravel() * h[2]], axis=1)
        return org.astype(np.float64)


def _zero(x: Array) -> Array:
    return np.zeros(x.shape[:-1])


def _one(x: Array) -> Array:
    return np.ones(x.shape[:-1])


def _unit(v: Array) -> Array:
    return v / np.linalg.norm(v)


def _bumps(centers: Array, amp: float, denom: float) -> Field:
    centers = np.asarray(centers, dtype=np.float64)

    def b(x: Array) -> Array:
        out = np.ones(x.shape[:-1])
        for c in centers:
            out = out + amp * np.exp(-np.sum((x - c) ** 2, axis=-1) / denom)
        return out

    return b


def _plane_wave(kappa: float, d: Array, phi: float) -> Field:
    d = np.asarray(d, dtype=np.float64)

    def g(x: Array) -> Array:
        return np.cos(kappa * (x @ d) + phi)

    return g


# Gaussian bump of width 0.1 read as exp(-|x-c|^2 / (2*0.1^2)).
BUMP_DENOM = 2.0 * 0.1 ** 2


def plane_wave_sine(nboxes=(2, 2, 2), p=6, kappa=2.0, seed=1, name="plane_wave_sine") -> Problem:
    """b = 1, f = 0, exact u = sin(kappa d.x) with a seeded unit vector d.

    Draws: d = unit(normal(3)).  -Lap u = kappa^2 |d|^2 u, so A u = 0 exactly.
    """
    rng = np.random.default_rng(seed)
    d = _unit(rng.normal(size=3))

    def u(x: Array) -> Array:
        return np.sin(kappa * (x @ d))

    return Problem(name=name, nboxes=tuple(nboxes), p=p, kappa=kappa, b=_one, f=_zero,
                   g=u, u_exact=u, params={"d": d, "seed": seed})


def config1() -> Problem:
    """2x2x2 boxes, p=6, kappa=2, manufactured sin(kappa d.x), seed 1."""
    return plane_wave_sine((2, 2, 2), 6, 2.0, 1, name="cfg1_2x2x2_p6")


def single_bump(nboxes=(8, 8, 8), p=12, kappa=20.0, seed=2, name="cfg2") -> Problem:
    """b = 1 - 0.5 exp(-|x-c|^2/0.05), g = cos(kappa d.x + phi), f = 0.

    Draws: c = uniform(3) in [0,1]^3, d = unit(normal(3)), phi = uniform(0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    c = rng.uniform(size=3)
    d = _unit(rng.normal(size=3))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))

    def b(x: Array) -> Array:
        return 1.0 - 0.5 * np.exp(-np.sum((x - c) ** 2, axis=-1) / 0.05)

    return Problem(name=name, nboxes=tuple(nboxes), p=p, kappa=kappa, b=b, f=_zero,
                   g=_plane_wave(kappa, d, phi), params={"c": c, "d": d, "phi": phi, "seed": seed})


def config2() -> Problem:
    """8x8x8 boxes, p=12, kappa=20, single-bump b, plane-wave g, seed 2."""
    return single_bump((8, 8, 8), 12, 20.0, 2, name="cfg2_8x8x8_p12")


def multi_bump(nboxes=(16, 16, 16), p=16, kappa=40.0, seed=3, nbump=8, amp=0.3,
               gaussian_source=False, name="cfg3") -> Problem:
    """b = 1 + amp * sum_m exp(-|x-c_m|^2/(2*0.1^2)), plane-wave g.

    Draws: centers = uniform(size=(nbump,3)), d = unit(normal(3)),
    phi = uniform(0, 2 pi); with gaussian_source also a source center s =
    uniform(3) and f = exp(-|x-s|^2/(2*0.1^2)) (else f = 0).
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(size=(nbump, 3))
    d = _unit(rng.normal(size=3))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))
    f = _zero
    params = {"centers": centers, "d": d, "phi": phi, "seed": seed}
    if gaussian_source:
        s = rng.uniform(size=3)
        params["source"] = s

        def f(x: Array) -> Array:  # noqa: F811
            return np.exp(-np.sum((x - s) ** 2, axis=-1) / BUMP_DENOM)

    return Problem(name=name, nboxes=tuple(nboxes), p=p, kappa=kappa,
                   b=_bumps(centers, amp, BUMP_DENOM), f=f, g=_plane_wave(kappa, d, phi),
                   params=params)


def config3() -> Problem:
    """16^3 boxes, p=16, kappa=40, 8 bumps, seed 3 (the headline workload)."""
    return multi_bump((16, 16, 16), 16, 40.0, 3, name="cfg3_16x16x16_p16")


def config3_p20() -> Problem:
    """4^3 boxes, p=20, kappa=40, 8 bumps, seed 4."""
    return multi_bump((4, 4, 4), 20, 40.0, 4, name="cfg3b_4x4x4_p20")


def config4() -> list:
    """Three independent problems batched together (seeds 41, 42, 43)."""
    return [multi_bump((12, 12, 12), 8, 10.0, 41, name="cfg4a_12^3_p8"),
            multi_bump((8, 8, 8), 12, 20.0, 42, name="cfg4b_8^3_p12"),
            multi_bump((6, 6, 6), 16, 30.0, 43, name="cfg4c_6^3_p16")]


@dataclass
class InverseProblem:
    """Data-misfit problem J(b) = 0.5 * sum_k (u(x_k) - d_k)^2.

    forward   -- the Problem with the current coefficient b
    b_obs     -- coefficient that generated the observations
    obs_nodes -- int array [nobs, 4]: (box t, i, j, k), i,j,k in [1, p-2] are
                 per-axis Chebyshev node indices of box-interior collocation nodes
    """

    forward: Problem
    b_obs: Field
    obs_nodes: Array


def config5(nboxes=(8, 8, 8), p=10, kappa=15.0, seed=5, nobs=500) -> InverseProblem:
    """8^3 boxes, p=10, kappa=15, FP64; gradient of a data misfit w.r.t. b.

    Draws: centers = uniform(size=(8,3)); c_star = uniform(3); d = unit(normal(3));
    phi = uniform(0, 2 pi); obs = choice(nbox*m^3, nobs, replace=False) decoded
    box-major as flat = t*m^3 + (k-1)*m^2 + (j-1)*m + (i-1).
    b_obs = b + 0.2 exp(-|x-c_star|^2/(2*0.1^2)).
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(size=(8, 3))
    c_star = rng.uniform(size=3)
    d = _unit(rng.normal(size=3))
    phi = float(rng.uniform(0.0, 2.0 * np.pi))
    nbox = int(np.prod(nboxes))
    m = p - 2
    flat = rng.choice(nbox * m ** 3, size=nobs, replace=False)
    t, rem = np.divmod(flat, m ** 3)
    k, rem = np.divmod(rem, m * m)
    j, i = np.divmod(rem, m)
    obs = np.stack([t, i + 1, j + 1, k + 1], axis=1).astype(np.int64)
    b = _bumps(centers, 0.3, BUMP_DENOM)

    def b_obs(x: Array) -> Array:
        return b(x) + 0.2 * np.exp(-np.sum((x - c_star) ** 2, axis=-1) / BUMP_DENOM)

    fwd = Problem(name="cfg5_8x8x8_p10", nboxes=tuple(nboxes), p=p, kappa=kappa, b=b,
                  f=_zero, g=_plane_wave(kappa, d, phi),
                  params={"centers": centers, "c_star": c_star, "d": d, "phi": phi, "seed": seed})
    return InverseProblem(forward=fwd, b_obs=b_obs, obs_nodes=obs)


def polynomial(nboxes=(2, 2, 2), p=6, degree=None, seed=7, name="poly") -> Problem:
    """kappa = 0, u = a seeded polynomial of per-axis degree <= p-1, f = -Lap u.

    Draws: coefficients = normal(size=(deg+1,)*3) with deg = p-1 unless given.
    The Laplacian of the polynomial is evaluated analytically (exact
    coefficient differentiation), so this is problem data, not the method.
    """
    deg = p - 1 if degree is None else degree
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(deg + 1,) * 3) / (1.0 + np.arange(deg + 1))[:, None, None]

    def _eval(coef: Array, x: Array) -> Array:
        return np.polynomial.polynomial.polyval3d(x[..., 0], x[..., 1], x[..., 2], coef)

    def u(x: Array) -> Array:
        return _eval(C, x)

    def lap(x: Array) -> Array:
        P = np.polynomial.polynomial
        cxx = P.polyder(C, 2, axis=0)
        cyy = P.polyder(C, 2, axis=1)
        czz = P.polyder(C, 2, axis=2)
        return _eval(cxx, x) + _eval(cyy, x) + _eval(czz, x)

    def f(x: Array) -> Array:
        return -lap(x)

    return Problem(name=name, nboxes=tuple(nboxes), p=p, kappa=0.0, b=_one, f=f, g=u,
                   u_exact=u, params={"coef": C, "seed": seed})


def helmholtz_greens(nboxes=(2, 2, 2), p=8, kappa=16.0, name="greens") -> Problem:
    """Paper Sec. 4.1: u = cos(kappa|x|)/(4 pi |x|) on [-1.1,0.1]x[1,2]x[1.2,2.2], b=1.

    With kappa = 0 this is the Poisson Green's function problem of the same section.
    """

    def u(x: Array) -> Array:
        r = np.linalg.norm(x, axis=-1)
        return np.cos(kappa * r) / (4.0 * np.pi * r)

    return Problem(name=name, nboxes=tuple(nboxes), p=p, kappa=kappa, b=_one, f=_zero, g=u,
                   lo=(-1.1, 1.0, 1.2), hi=(0.1, 2.0, 2.2), u_exact=u)


@dataclass
class ParabolicProblem:
    """u_t = nu Lap u + kappa^2 b(x) u on a box grid, u = 0 on the boundary, u(x, 0) = u0(x)
    (paper Sec. 4.4 steps a parabolic problem with Crank-Nicolson; its example also has a
    convection term, which the operator class here, -Lap u - kappa^2 b u, does not cover:
    this family keeps diffusion and adds a variable reaction term instead).

    u_exact(x, t), when given, is the exact solution of the continuous problem.
    """

    name: str
    nboxes: Tuple[int, int, int]
    p: int
    nu: float
    dt: float
    kappa: float
    b: Field
    u0: Field
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    u_exact: Optional[Callable[[Array, float], Array]] = None
    params: dict = field(default_factory=dict)

    @property
    def nbox(self) -> int:
        return int(self.nboxes[0] * self.nboxes[1] * self.nboxes[2])

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple((self.hi[a] - self.lo[a]) / self.nboxes[a] for a in range(3))

    def box_origins(self) -> Array:
        n1, n2, n3 = self.nboxes
        t = np.arange(n1 * n2 * n3)
        bx, rem = t % n1, t // n1
        by, bz = rem % n2, rem // n2
        h = self.h
        return np.stack([self.lo[0] + bx * h[0], self.lo[1] + by * h[1], self.lo[2] + bz * h[2]], axis=1)


def heat_sine(nboxes=(2, 2, 2), p=10, nu=0.1, dt=0.05, name="heat_sine") -> ParabolicProblem:
    """u_t = nu Lap u on [0,1]^3 with u = exp(-3 pi^2 nu t) sin(pi x) sin(pi y) sin(pi z)
    (zero on the boundary, exact).  No random draws."""

    def s(x: Array) -> Array:
        return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])

    def u_exact(x: Array, t: float) -> Array:
        return np.exp(-3.0 * np.pi ** 2 * nu * t) * s(x)

    return ParabolicProblem(name=name, nboxes=tuple(nboxes), p=p, nu=nu, dt=dt, kappa=0.0, b=_one, u0=s,
                            u_exact=u_exact)


def diffusion_reaction(nboxes=(2, 2, 2), p=8, nu=0.05, dt=0.02, kappa=1.0, seed=9, nbump=3, amp=0.5,
                       width2=0.02, name="diffusion_reaction") -> ParabolicProblem:
    """On [-0.5, 0.5]^3: reaction coefficient b = 1 + amp * (seeded Gaussian bumps, width 0.1)
    and a Gaussian initial blob below the centre, u0 = exp(-(x^2 + (y + 0.3)^2 + z^2)/width2)
    (the paper's initial condition has width2 = 0.002 and, as printed, a positive exponent;
    the decaying blob is meant).  u = 0 on the boundary.

    Draws: centers = uniform(-0.5, 0.5, size=(nbump, 3))."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-0.5, 0.5, size=(nbump, 3))

    def u0(x: Array) -> Array:
        return np.exp(-(x[..., 0] ** 2 + (x[..., 1] + 0.3) ** 2 + x[..., 2] ** 2) / width2)

    return ParabolicProblem(name=name, nboxes=tuple(nboxes), p=p, nu=nu, dt=dt, kappa=kappa,
                            b=_bumps(centers, amp, BUMP_DENOM), u0=u0, lo=(-0.5, -0.5, -0.5), hi=(0.5, 0.5, 0.5),
                            params={"centers": centers, "seed": seed})
