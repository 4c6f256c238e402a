"""Pins for the oracle's local blocks and per-box reduction (paper eq. Aentries,
eq. blocksys1, definitions of S and T in Sec. 2.2, eq. t-block, Alg. 1/2).

Every expected value comes from calculus on polynomials (exact for the
collocation when the per-axis degree is <= p-1) or from an invariant of the
DtN map, not from the oracle's own formulas."""
import numpy as np
import pytest

from oracle import leaf

P = np.polynomial.polynomial


def _poly(seed, deg):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(deg + 1,) * 3)


def _ev(C, x):
    return P.polyval3d(x[..., 0], x[..., 1], x[..., 2], C)


def _grad(C, x):
    return np.stack([_ev(P.polyder(C, 1, axis=a), x) for a in range(3)], axis=-1)


def _lap(C, x):
    return sum(_ev(P.polyder(C, 2, axis=a), x) for a in range(3))


NORMALS = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], float)


def _face_normals(p):
    mm = (p - 2) ** 2
    return np.repeat(NORMALS, mm, axis=0)


@pytest.mark.parametrize("p", [4, 6, 9])
def test_edges_and_corners_never_coupled(p):
    # Remark 1: without cross terms no row touches an edge or corner node.
    ec = leaf.edge_corner_full_index(p)
    h = (0.3, 0.5, 0.7)
    L = leaf.full_operator_rows(p, h, 3.0, np.linspace(1, 2, p ** 3))[leaf.interior_full_index(p)]
    N = leaf.neumann_rows(p, h)
    assert np.abs(L[:, ec]).max() == 0.0
    assert np.abs(N[:, ec]).max() == 0.0
    assert len(ec) == p ** 3 - (p - 2) ** 3 - 6 * (p - 2) ** 2


@pytest.mark.parametrize("p,kappa", [(5, 0.0), (6, 3.0), (8, 11.0)])
def test_blocks_exact_on_polynomials(p, kappa):
    h = (0.5, 0.25, 0.4)
    org = (0.1, -0.2, 0.3)
    xi, xb = leaf.box_node_coords(org, h, p)
    C = _poly(p, p - 1)
    b = 1.0 + 0.3 * np.sin(xi[:, 0] + 2 * xi[:, 1])
    blk = leaf.local_blocks(p, h, kappa, b)
    ui, ub = _ev(C, xi), _ev(C, xb)
    # interior rows: -Lap u - kappa^2 b u
    lhs = blk.A_ii @ ui + blk.A_ib @ ub
    rhs = -_lap(C, xi) - kappa ** 2 * b * ui
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()
    # face rows: outward normal derivative
    flux = blk.A_bi @ ui + blk.A_bb @ ub
    dn = np.sum(_grad(C, xb) * _face_normals(p), axis=1)
    assert np.abs(flux - dn).max() < 1e-9 * np.abs(dn).max()


def test_node_layout():
    p, h, org = 5, (1.0, 2.0, 3.0), (0.0, 0.0, 0.0)
    xi, xb = leaf.box_node_coords(org, h, p)
    m = p - 2
    # interior order: x fastest, then y, then z
    assert xi[0, 0] < xi[1, 0] and xi[0, 1] == xi[1, 1]
    assert xi[m, 1] > xi[0, 1] and xi[m * m, 2] > xi[0, 2]
    mm = m * m
    for a in range(6):
        axis, side = divmod(a, 2)
        face = xb[a * mm:(a + 1) * mm]
        assert np.all(face[:, axis] == (0.0 if side == 0 else h[axis]))
        tang = [ax for ax in range(3) if ax != axis]
        assert face[1, tang[0]] > face[0, tang[0]]        # lower tangential axis fastest
        assert face[m, tang[1]] > face[0, tang[1]]


@pytest.mark.parametrize("p", [5, 7, 10])
def test_dtn_annihilates_constants(p):
    # kappa = 0: constant face data extends to a constant interior, zero flux.
    blk = leaf.local_blocks(p, (0.3, 0.3, 0.3), 0.0, np.ones((p - 2) ** 3))
    red = leaf.leaf_reduce(blk, np.zeros((p - 2) ** 3))
    assert np.abs(red.T.sum(axis=1)).max() < 1e-11 * np.abs(red.T).max()
    # the A_bb term is what makes this hold; without it the row sums are O(1/h)
    assert np.abs((blk.A_bi @ red.S).sum(axis=1)).max() > 1.0


@pytest.mark.parametrize("p", [5, 8])
def test_dtn_of_linear_is_outward_flux(p):
    h = (0.5, 0.5, 0.25)
    xi, xb = leaf.box_node_coords((0.0, 0.0, 0.0), h, p)
    blk = leaf.local_blocks(p, h, 0.0, np.ones((p - 2) ** 3))
    red = leaf.leaf_reduce(blk, np.zeros((p - 2) ** 3))
    a = np.array([0.7, -1.3, 2.1])
    ub = xb @ a + 0.4
    np.testing.assert_allclose(red.T @ ub, _face_normals(p) @ a, atol=1e-10)


@pytest.mark.parametrize("p,kappa", [(6, 0.0), (7, 4.0)])
def test_reduction_with_load(p, kappa):
    # u polynomial, f = -Lap u - kappa^2 b u: interior = v + S u_b, flux = T u_b - g.
    h = (0.4, 0.4, 0.4)
    xi, xb = leaf.box_node_coords((0.2, 0.1, 0.0), h, p)
    C = _poly(11, p - 1)
    b = 1.0 + 0.5 * xi[:, 2]
    f = -_lap(C, xi) - kappa ** 2 * b * _ev(C, xi)
    blk = leaf.local_blocks(p, h, kappa, b)
    red = leaf.leaf_reduce(blk, f)
    ub = _ev(C, xb)
    ui = red.v + red.S @ ub
    np.testing.assert_allclose(ui, _ev(C, xi), atol=1e-9 * np.abs(_ev(C, xi)).max())
    dn = np.sum(_grad(C, xb) * _face_normals(p), axis=1)
    np.testing.assert_allclose(red.T @ ub - red.g, dn, atol=1e-8 * np.abs(dn).max())
    # X columns solve A_ii X = [A_ib | f]
    B = np.concatenate([blk.A_ib, f[:, None]], axis=1)
    assert np.abs(blk.A_ii @ red.X - B).max() < 1e-10 * np.abs(B).max()


# ---- interior solve with given face values (Sec. 2.2 four-step solve, step 4) ------

@pytest.mark.parametrize("p,kappa", [(5, 0.0), (7, 0.0), (6, 3.5)])
def test_interior_solve_reproduces_polynomial(p, kappa):
    # u of per-axis degree <= p-1, f = -Lap u - kappa^2 b u from calculus: given the face
    # values of u, the interior values must be those of u (collocation is exact there).
    h = (0.5, 0.25, 0.4)
    xi, xb = leaf.box_node_coords((0.1, -0.2, 0.3), h, p)
    C = _poly(23 + p, p - 1)
    b = 1.0 + 0.3 * xi[:, 0] * xi[:, 1]
    f = -_lap(C, xi) - kappa ** 2 * b * _ev(C, xi)
    blk = leaf.local_blocks(p, h, kappa, b)
    ui = leaf.interior_solve(blk, f, _ev(C, xb))
    ex = _ev(C, xi)
    np.testing.assert_allclose(ui, ex, atol=1e-10 * np.abs(ex).max())


def test_interior_solve_equals_reconstruction():
    # u_i = A_ii^{-1}(f_i - A_ib u_b) = v + S u_b for arbitrary face values and loads
    p, h, kappa = 6, (0.5,) * 3, 4.0
    rng = np.random.default_rng(31)
    xi, _ = leaf.box_node_coords((0.0, 0.0, 0.0), h, p)
    b = 1.0 + 0.2 * rng.random(xi.shape[0])
    f = rng.normal(size=xi.shape[0])
    ub = rng.normal(size=6 * (p - 2) ** 2)
    blk = leaf.local_blocks(p, h, kappa, b)
    red = leaf.leaf_reduce(blk, f)
    np.testing.assert_allclose(leaf.interior_solve(blk, f, ub), red.v + red.S @ ub, rtol=0, atol=1e-12)


def test_planted_interior_solve_sign_is_caught():
    # f_i + A_ib u_b instead of f_i - A_ib u_b must break polynomial reproduction
    p, kappa, h = 6, 2.0, (0.5, 0.5, 0.5)
    xi, xb = leaf.box_node_coords((0.0, 0.0, 0.0), h, p)
    C = _poly(5, p - 1)
    b = np.ones(xi.shape[0])
    f = -_lap(C, xi) - kappa ** 2 * _ev(C, xi)
    blk = leaf.local_blocks(p, h, kappa, b)
    bad = np.linalg.solve(blk.A_ii, f + blk.A_ib @ _ev(C, xb))
    ex = _ev(C, xi)
    assert np.abs(bad - ex).max() > 1e-3 * np.abs(ex).max()
