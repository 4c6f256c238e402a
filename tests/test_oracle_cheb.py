"""Pins for the Chebyshev tables of the oracle (paper Sec. 2.1: tensor Chebyshev
nodes, spectral collocation).  Each check is a closed form or an exactness
property, never a retyping of the oracle's own formula."""
import numpy as np
import pytest

from oracle import cheb


def test_p3_matrix_closed_form():
    # Three Lobatto points -1, 0, 1: the derivative of the quadratic interpolant.
    D = cheb.diffmat(3)
    ref = np.array([[-1.5, 2.0, -0.5],
                    [-0.5, 0.0, 0.5],
                    [0.5, -2.0, 1.5]])
    np.testing.assert_allclose(D, ref, atol=1e-15)


@pytest.mark.parametrize("p", [4, 6, 9, 16, 20])
def test_corner_entries_closed_form(p):
    # D at the end points of the Chebyshev-Lobatto grid: -/+ (2N^2 + 1)/6, N = p - 1.
    N = p - 1
    D = cheb.diffmat(p)
    assert D[0, 0] == pytest.approx(-(2 * N * N + 1) / 6.0, rel=1e-12)
    assert D[-1, -1] == pytest.approx((2 * N * N + 1) / 6.0, rel=1e-12)


@pytest.mark.parametrize("p", [3, 5, 8, 12, 16, 20])
def test_exact_on_polynomials(p):
    t = cheb.nodes(p)
    D = cheb.diffmat(p)
    for deg in range(p):
        err = np.abs(D @ t ** deg - deg * t ** max(deg - 1, 0) * (deg > 0)).max()
        assert err < 1e-10 * max(1.0, deg ** 2 * p ** 2), (deg, err)
    # and not exact one degree higher (the interpolant has degree p-1)
    assert np.abs(D @ t ** p - p * t ** (p - 1)).max() > 1e-6


@pytest.mark.parametrize("p", [4, 7, 16])
def test_nodes_and_symmetry(p):
    t = cheb.nodes(p)
    assert t[0] == -1.0 and t[-1] == pytest.approx(1.0)
    assert np.all(np.diff(t) > 0)
    np.testing.assert_allclose(t, -t[::-1], atol=1e-15)
    D = cheb.diffmat(p)
    # reflecting the grid negates the derivative: D[N-i, N-j] = -D[i, j]
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-11 * p * p)


def test_box_scaling():
    # d/dx on [lo, lo+h]: applying (2/h) D to x^2 at the physical nodes gives 2x.
    p, lo, h = 7, 0.3, 0.25
    x = cheb.box_axis_coords(lo, h, p)
    np.testing.assert_allclose((2.0 / h) * cheb.diffmat(p) @ x ** 2, 2 * x, atol=1e-12)
    assert x[0] == pytest.approx(lo) and x[-1] == pytest.approx(lo + h)
