"""Pins for the oracle's misfit gradient dJ/db (adjoint of the two-level factorization).

* The two-level transposed-solve gradient equals the gradient from the dense
  global system (A^T lambda = P^T r).
* Central finite differences of J agree with grad . v for seeded directions.
* Dot-product test for the transposed interface solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, interface


def _small_inverse_problem(seed=5, p=6):
    inv = W.config5(nboxes=(2, 2, 2), p=p, kappa=6.0, seed=seed, nobs=40)
    prob = inv.forward
    res_obs = interface.solve(prob, b_field=inv.b_obs)
    data = adjoint.observe(res_obs.u_i, inv.obs_nodes, p)
    return inv, prob, data


def test_two_level_gradient_matches_dense_global():
    inv, prob, data = _small_inverse_problem()
    J1, g1, _ = adjoint.two_level_gradient(prob, inv.obs_nodes, data)
    J2, g2 = adjoint.brute_gradient(prob, inv.obs_nodes, data)
    assert J1 == pytest.approx(J2, rel=1e-11)
    assert interface.rel_l2(g1, g2) < 1e-10


def test_gradient_matches_central_differences():
    inv, prob, data = _small_inverse_problem()
    J, grad, res = adjoint.two_level_gradient(prob, inv.obs_nodes, data)
    rng = np.random.default_rng(17)
    xs = [bd.xi for bd in res.boxes]
    for trial in range(3):
        c = rng.uniform(size=3)

        def v(x):
            return np.exp(-np.sum((x - c) ** 2, axis=-1) / 0.05)

        hstep = 1e-6

        def J_at(s):
            def bf(x):
                return prob.b(x) + s * v(x)
            r = interface.solve(prob, b_field=bf)
            return adjoint.misfit(r.u_i, inv.obs_nodes, data, prob.p)

        fd = (J_at(hstep) - J_at(-hstep)) / (2 * hstep)
        an = float(sum((grad[t] * v(xs[t])).sum() for t in range(len(xs))))
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(J))


def test_gradient_vanishes_without_misfit():
    inv, prob, _ = _small_inverse_problem()
    res = interface.solve(prob)
    data = adjoint.observe(res.u_i, inv.obs_nodes, prob.p)
    J, grad, _ = adjoint.two_level_gradient(prob, inv.obs_nodes, data)
    assert J < 1e-25 and np.abs(grad).max() < 1e-10


def test_interface_transpose_dot_product():
    prob = W.multi_bump((2, 2, 2), 6, 5.0, 8)
    res = interface.solve(prob)
    rng = np.random.default_rng(3)
    x = rng.normal(size=res.T_ff.shape[0])
    y = rng.normal(size=res.T_ff.shape[0])
    lhs = y @ res.lu.solve(x)
    rhs = x @ res.lu.solve(y, trans="T")
    assert lhs == pytest.approx(rhs, rel=1e-12)
