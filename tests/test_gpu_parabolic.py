"""Crank-Nicolson stepping on the GPU (paper Sec. 4.4) against the stepping oracle.

One build and one interface factorization, then per step the right-hand side, the
loads, the interface solve and the interiors, all through the C ABI.  Every step's
state (interior and internal-face values) must match the oracle's global collocation
stepping: 1e-10 relative with FP64 factors, 1e-9 with FP32 factors and FP64
refinement.  The exact heat mode also checks the closed-form decay factor.
"""
import numpy as np
import pytest

import workloads as W
from oracle import parabolic as op
from tests.gpu_helpers import rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nboxes", [(2, 2, 2), (3, 2, 2)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_ir", 1e-9)])
def test_crank_nicolson_vs_oracle(gpu, precision, tol, nboxes):
    from paper_2503_04033_amd.stepping import CrankNicolson
    pp = W.diffusion_reaction(nboxes, p=8, nu=0.05, dt=0.02, kappa=1.0, seed=9, width2=0.05)
    nsteps = 5
    say(f"crank-nicolson {pp.name} {nboxes} p={pp.p} {precision}")
    cn = CrankNicolson(pp, precision)
    ref, _ = op.crank_nicolson(pp, nsteps)
    for n in range(nsteps):
        cn.step()
        w = np.concatenate([cn.u_i.cpu().numpy().ravel(), cn.face_solution().cpu().numpy()])
        err = rel(w, ref[n])
        say(f"  step {n + 1}: |u| {np.linalg.norm(ref[n]):.4e}, rel err {err:.2e}")
        assert err < tol


def test_crank_nicolson_heat_mode_decay(gpu):
    from paper_2503_04033_amd.stepping import CrankNicolson
    pp = W.heat_sine((2, 2, 2), 10, nu=0.1, dt=0.025)
    cn = CrankNicolson(pp, "fp64")
    w0 = np.concatenate([cn.u_i.cpu().numpy().ravel(), cn.face_solution().cpu().numpy()])
    x = 3.0 * np.pi ** 2 * pp.nu * pp.dt
    r = (1.0 - x / 2) / (1.0 + x / 2)
    for n in range(8):
        cn.step()
    w = np.concatenate([cn.u_i.cpu().numpy().ravel(), cn.face_solution().cpu().numpy()])
    err = np.abs(w - r ** 8 * w0).max() / np.abs(w0).max()
    say(f"  heat mode after 8 steps vs r^8 u0: {err:.2e}")
    assert err < 1e-7
