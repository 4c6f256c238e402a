"""Pins of the Crank-Nicolson oracle (oracle/parabolic.py, paper Sec. 4.4).

* Second order in time: for the exact decaying mode of the heat equation, the error at
  a fixed time falls by ~4 each time dt halves (the spatial error at p = 10 is far below).
* The reaction term enters with the right sign: with kappa^2 b = 3 pi^2 nu the same mode
  is a steady state of u_t = nu Lap u + kappa^2 b u and stays put; flipping the sign of the
  reaction term (a planted mistake) makes it grow.
"""
import dataclasses

import numpy as np

import workloads as W
from oracle import parabolic as op


def _exact_state(pp, t):
    """[u_int, u_face] of u_exact(., t) at the global unknowns (initial_state with u0 = u(., t))."""
    return op.initial_state(dataclasses.replace(pp, u0=lambda x: pp.u_exact(x, t)))


def test_crank_nicolson_second_order_in_time():
    # the mode decays by the Crank-Nicolson factor r = (1 - x/2)/(1 + x/2), x = 3 pi^2 nu dt, per
    # step (a closed form: the mode is an eigenfunction of the Laplacian, resolved to ~1e-9
    # at p = 10), and the error against exp(-3 pi^2 nu t) falls ~4-fold per halving of dt
    errs = []
    T, nu = 0.2, 0.1
    for dt in (0.05, 0.025, 0.0125):
        pp = W.heat_sine((2, 2, 2), 10, nu=nu, dt=dt)
        nsteps = int(round(T / dt))
        states, _ = op.crank_nicolson(pp, nsteps)
        w0 = op.initial_state(pp)
        x = 3.0 * np.pi ** 2 * nu * dt
        r = (1.0 - x / 2) / (1.0 + x / 2)
        assert np.abs(states[-1] - r ** nsteps * w0).max() / np.abs(w0).max() < 1e-7
        ref = _exact_state(pp, T)
        errs.append(np.abs(states[-1] - ref).max() / np.abs(ref).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert errs[0] < 2e-3
    assert all(3.7 < q < 4.3 for q in ratios), (errs, ratios)


def test_reaction_term_sign_steady_mode():
    nu = 0.1
    pp = W.heat_sine((2, 2, 2), 10, nu=nu, dt=0.05)
    pp = dataclasses.replace(pp, kappa=float(np.sqrt(3.0 * np.pi ** 2 * nu)))
    w0 = op.initial_state(pp)
    states, _ = op.crank_nicolson(pp, 8)
    drift = np.abs(states[-1] - w0).max() / np.abs(w0).max()
    assert drift < 1e-6  # steady up to the spatial error of the mode at p = 10
    flipped = dataclasses.replace(pp, b=lambda x: -np.ones(x.shape[:-1]))
    states_f, _ = op.crank_nicolson(flipped, 8)
    assert np.abs(states_f[-1]).max() < 0.5 * np.abs(w0).max()  # decays at twice the rate instead
