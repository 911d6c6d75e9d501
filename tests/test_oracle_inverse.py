"""Pins of the oracle's inverse elasticity problem (eqs. cost, f-prob, g-prob,
w-f, w-g, the adjoints of eqs. dL1/dL2 and the shape derivative of eq.
SDelast_inv) against facts that do not come from its formulas: central
finite differences of the discrete cost under a smooth mesh motion that
fixes the boundary (exact for P1 with a linear g and A frozen per element),
the vanishing of cost, adjoints and derivative at the true inclusion, and
the boundary conditions of each solution."""
import numpy as np
import pytest

import fo_inputs as fi
from oracle import inverse as oi


def bubble(X, lengths):
    d = X.shape[1]
    bub = np.ones(X.shape[0])
    for k in range(d):
        bub *= X[:, k] * (lengths[k] - X[:, k])
    cols = [bub * (1.0 + 0.5 * X[:, 0]), bub * np.sin(3.0 * X[:, 1] + 0.2)]
    if d == 3:
        cols.append(bub * (X[:, 2] - 0.3 * X[:, 0]))
    th = np.stack(cols, axis=1)
    return th / np.abs(th).max()


def moved_cost(wi, X, a):
    """Cost of the inverse problem on the mesh moved to X (A frozen by phi,
    g = x_0 a re-evaluated at the moved nodes)."""
    g = (X[:, :1] * a[None, :]).ravel()
    wj = fi.InverseWorkload(wi.mesh, wi.fixed0, wi.fixed_all, wi.f, g, wi.phi, wi.kappa, wi.alpha, wi.beta,
                            wi.E, wi.nu, wi.plane_stress)
    return oi.inverse_iteration(wj, X=X)["J"]


@pytest.mark.parametrize("dim", [2, 3])
def test_shape_derivative_matches_finite_differences(dim):
    cells = (24, 12) if dim == 2 else (12, 6, 6)
    wi = fi.inverse_elasticity(cells)
    m = wi.mesh
    a = np.array([0.02, -0.01, 0.015][:dim])
    r = oi.inverse_iteration(wi)
    assert 0 < r["chi"].sum() < m.n_elems
    assert r["J"] > 0
    theta = bubble(m.coords, m.lengths)
    dJ = -float(r["rhs"] @ theta.ravel())
    t = 1e-4
    fd = (moved_cost(wi, m.coords + t * theta, a) - moved_cost(wi, m.coords - t * theta, a)) / (2 * t)
    assert abs(fd - dJ) <= 1e-6 * abs(dJ), (fd, dJ)


@pytest.mark.parametrize("dim", [2, 3])
def test_true_inclusion_gives_zero_cost_and_derivative(dim):
    """With g the f-problem's solution for the inclusion itself, y = u: the
    lifted part v and both adjoints vanish, and so do J and S."""
    cells = (24, 12) if dim == 2 else (12, 6, 6)
    wi = fi.inverse_elasticity(cells)
    r0 = oi.inverse_iteration(wi)
    wi.g = r0["u"].copy()
    r = oi.inverse_iteration(wi)
    scale = np.abs(r0["u"]).max()
    assert np.abs(r["v"]).max() <= 1e-12 * scale
    assert r["J"] <= 1e-24
    assert np.abs(r["p"]).max() <= 1e-14 and np.abs(r["q"]).max() <= 1e-14
    assert np.abs(r["rhs"]).max() <= 1e-12 * np.abs(r0["rhs"]).max()


def test_boundary_conditions_of_each_solution():
    wi = fi.inverse_elasticity((24, 12))
    r = oi.inverse_iteration(wi)
    assert np.all(r["u"][wi.fixed0 == 1] == 0) and np.all(r["p"][wi.fixed0 == 1] == 0)
    assert np.all(r["v"][wi.fixed_all == 1] == 0) and np.all(r["q"][wi.fixed_all == 1] == 0)
    # g vanishes on Gamma_0, so y = v + g meets u's clamp there
    assert np.all(wi.g[wi.fixed0 == 1] == 0)
    # theta in H^1_0
    th, info = oi.velocity(wi, r["rhs"])
    assert info.status == 0 and np.all(th[wi.fixed_all == 1] == 0)
    assert float(th @ r["rhs"]) > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_matrices_integrate_exactly(dim):
    """The vector mass integrates products of P1 fields exactly over D, the
    facet mass over Gamma_1 (the boundary without the face x = 0):
    1^T M 1 = d |D|, int x_0 over D, and 1^T M_G 1 = d |Gamma_1|, int x_0^2
    over Gamma_1, in closed form for [0,2]x[0,1]^(d-1)."""
    wi = fi.inverse_elasticity((12, 6) if dim == 2 else (6, 3, 3))
    m = wi.mesh
    M = oi.vector_mass(dim, m.coords, m.conn)
    MG = oi.facet_mass(dim, m.coords, m.bfacets)
    one = np.ones(m.n_dofs)
    x0 = np.repeat(m.coords[:, 0], dim)
    vol = 2.0
    area = 5.0 if dim == 2 else 9.0
    assert one @ (M @ one) == pytest.approx(dim * vol, rel=1e-13)
    assert x0 @ (M @ one) == pytest.approx(dim * 2.0 * 1.0 * (1.0 if dim == 2 else 1.0), rel=1e-13)
    assert one @ (MG @ one) == pytest.approx(dim * area, rel=1e-13)
    # int_Gamma1 x_0^2: the faces y = 0, 1 (and z = 0, 1) give int_0^2 x^2 = 8/3 each, the face x = 2 gives 4
    faces = 2 if dim == 2 else 4
    assert x0 @ (MG @ x0) == pytest.approx(dim * (faces * 8.0 / 3.0 + 4.0), rel=1e-13)


def test_inverse_loop_decreases_the_cost_and_sums_the_pairs():
    """Algorithm 1 on the inverse problem: the cost falls over the first
    iterations; a workload holding the same pair twice doubles the cost and
    the right-hand side, so theta doubles and B(theta, theta) quadruples;
    the stopping rule on the cost ends the loop where its definition says."""
    wi = fi.inverse_elasticity((37, 19))
    r = oi.optimize_inverse(wi, 5)
    Js = [rec.J for rec in r.records]
    assert all(b < a for a, b in zip(Js, Js[1:]))
    assert all(rec.B_tt > 0 and rec.steps >= 8 for rec in r.records)
    twice = fi.InverseWorkload(wi.mesh, wi.fixed0, wi.fixed_all, wi.f, wi.g, wi.phi, wi.kappa, wi.alpha, wi.beta,
                               wi.E, wi.nu, wi.plane_stress, fs=[wi.f, wi.f], gs=[wi.g, wi.g])
    r2 = oi.optimize_inverse(twice, 1)
    assert r2.records[0].J == pytest.approx(2.0 * r.records[0].J, rel=1e-13)
    assert r2.records[0].B_tt == pytest.approx(4.0 * r.records[0].B_tt, rel=1e-9)
    # |J_3 - J_j| < 0.5 |J_3| for j = 1, 2: the first test, at i = 3, stops
    rs = oi.optimize_inverse(wi, 8, start_to_check=2, prev=2, cost_tol=0.5)
    assert rs.stopped and len(rs.records) == 4 and rs.records[-1].steps == 0
