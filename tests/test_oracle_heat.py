"""Pins of the oracle's heat-conduction model (eqs. heat_cost, heat_prob,
heat_weak, and the shape derivative components S0 = 2 u grad f, S1 = (2 u f
- A |grad u|^2) I + 2 A grad u (x) grad u) against facts that do not come
from its element integrals: central finite differences of the discrete cost
under a smooth mesh motion (the identity is exact for P1 with a linear f
and A frozen per element), the constraint term likewise, J = int f u, and
the nodally exact one-dimensional solution on a strip."""
import numpy as np
import pytest

import fo_inputs as fi
from oracle import element_coef, element_geometry
from oracle import heat as oh


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


def linear_f(X):
    return 1.0 + 0.4 * X[:, 0] - 0.7 * X[:, 1] + (0.2 * X[:, 2] if X.shape[1] == 3 else 0.0)


def gamma0(m):
    # temperature fixed on the x = 0 face
    return (np.abs(m.coords[:, 0]) < 1e-12).astype(np.uint8)


def cost(m, X, A, fixed):
    f = linear_f(X)
    K = oh.stiffness(m.dim, X, m.conn, A)
    u = oh.solve_state(K, oh.mass(m.dim, X, m.conn) @ f, fixed)
    return float(u @ (K @ u))


@pytest.mark.parametrize("dim", [2, 3])
def test_shape_derivative_matches_finite_differences(dim):
    w = fi.cantilever_2d((24, 12)) if dim == 2 else fi.cantilever_3d((16, 8, 8))
    m = w.mesh
    fixed = gamma0(m)
    A, chi = element_coef(dim, m.conn, w.phi, 1e-3)
    assert 0 < chi.sum() < m.n_elems
    f = linear_f(m.coords)
    u, J, vol, rhs, A2, chi2 = oh.heat_iteration(dim, m.coords, m.conn, w.phi, f, fixed)
    theta = bubble(m.coords, m.lengths)
    dJ = -(rhs * theta).sum()
    t = 1e-4
    fd = (cost(m, m.coords + t * theta, A, fixed) - cost(m, m.coords - t * theta, A, fixed)) / (2 * t)
    assert abs(fd - dJ) <= 1e-7 * abs(dJ), (fd, dJ)
    # the adjoint is -u: the cost equals int f u
    b = oh.mass(dim, m.coords, m.conn) @ f
    assert J == pytest.approx(float(b @ u), rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_constraint_term_matches_finite_differences(dim):
    w = fi.cantilever_2d((24, 12)) if dim == 2 else fi.cantilever_3d((16, 8, 8))
    m = w.mesh
    A, chi = element_coef(dim, m.conn, w.phi, 1e-3)
    V = 0.7
    rhs = oh.derivative(dim, m.coords, m.conn, A, chi, np.zeros(m.n_nodes), np.zeros(m.n_nodes), 1.0, V)
    theta = bubble(m.coords, m.lengths)
    t = 1e-4

    def C(X):
        v, _ = element_geometry(dim, X, m.conn)
        return (chi * v).sum() / V

    fd = (C(m.coords + t * theta) - C(m.coords - t * theta)) / (2 * t)
    assert fd == pytest.approx(-(rhs * theta).sum(), rel=1e-8)


def test_strip_converges_to_the_one_dimensional_solution():
    """A = 1, f = 1, u = 0 at x = 0, insulated elsewhere on [0,1] x [0,0.25]:
    the exact solution is u = x (2 - x) / 2.  The cost error falls as h^2
    (ratio 4 per halving) towards its value 0.25 / 3, and the nodal error
    falls too."""
    errs, costs = [], []
    for n in (8, 16, 32):
        m = fi.structured_mesh((n, max(2, n // 4)), (1.0, 0.25))
        phi = -np.ones(m.n_nodes)
        u, J, vol, rhs, A, chi = oh.heat_iteration(2, m.coords, m.conn, phi, np.ones(m.n_nodes), gamma0(m))
        x = m.coords[:, 0]
        errs.append(np.abs(u - x * (2 - x) / 2).max())
        costs.append(J)
        assert np.all(A == 1.0) and vol == pytest.approx(0.25, rel=1e-14)
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5
    e = [abs(c - 0.25 / 3.0) for c in costs]
    assert e[0] / e[1] > 3.8 and e[1] / e[2] > 3.8
    assert costs[2] == pytest.approx(0.25 / 3.0, rel=1e-3)


def test_heat_loop_direction_multiplier_and_stop():
    """Algorithm 1 on the heat model: without a constraint the cost falls
    and the volume grows (conduction wants material); with a volume target
    below the volume the multiplier rises while the constraint is violated;
    the stopping rule ends the loop where its definition says."""
    w = fi.cantilever_2d((48, 24))
    m = w.mesh
    f = np.ones(m.n_nodes)
    g0 = (np.abs(m.coords[:, 0]) < 1e-12).astype(np.uint8)
    r = oh.optimize_heat(w, f, g0, 4, dfactor=1.0)
    Js = [x.J for x in r.records]
    vols = [x.vol for x in r.records]
    assert all(b < a for a, b in zip(Js, Js[1:])) and all(b > a for a, b in zip(vols, vols[1:]))
    V = 0.9 * vols[0]
    rc = oh.optimize_heat(w, f, g0, 4, V=V, dfactor=1.0)
    lams = [x.lam for x in rc.records]
    assert lams[0] == 0.0 and all(x.C > 1.0 for x in rc.records)
    assert all(b > a for a, b in zip(lams, lams[1:]))
    rs = oh.optimize_heat(w, f, g0, 8, dfactor=1.0, start_to_check=2, prev=2, cost_tol=0.5)
    assert rs.stopped and len(rs.records) == 4 and rs.records[-1].steps == 0
